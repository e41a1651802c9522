// Kernel templates of the fused step march of the second-order
// Trotter-Suzuki step for gfx950 (Wittek & Cucchietti, Sec. 2), instantiated
// per dtype and variant in march_<dtype>_<variant>.hip.
//
// Fused step march (one launch = `S` time steps over the whole mesh):
//   * Each wavefront owns a strip of the mesh: 64 lanes across x, each lane
//     holding PPL consecutive even x-pairs (2j, 2j+1) of one row in registers,
//     and it marches down y over a segment of rows.
//   * Even x-pairs are rotated inside a lane; odd x-pairs (2j+1, 2j+2) that
//     straddle two lanes swap the partner value with a DPP wavefront shift
//     (no LDS, no barrier).
//   * y-pairs are rows held by the same lane: the even pair (2q, 2q+1) is a
//     row pair, the odd pair (2q+1, 2q+2) joins a row pair to the next one.
//   * The S steps form a register pipeline: stage k works on the row pair k
//     behind the one just loaded, so a row pair leaves the last stage S
//     steps older, having been read and written in device memory once.
//   * Lanes at the strip edges and row pairs at the segment ends are a halo
//     whose results are discarded: the dependence of one step reaches one
//     pair along each axis, so S steps need S pairs of halo (plus one for the
//     closing odd factor of the last pass).
// Operation order of one evolution of N steps, h = dt/2 (left applied first):
//   Ox(h) Oy(h) [Ex Ey P Ey Ex](h) { Ox(2h) Oy(2h) [Ex Ey P Ey Ex](h) }^(N-1) Ox(h) Oy(h)
// which equals U2(dt)^N of Sec. 2 exactly in real arithmetic (x and y
// factors commute; two consecutive Ox(h) are one Ox(2h)).  Every site goes
// through the same operations in the same order whatever the strip, segment
// and S, so results are bitwise independent of the schedule.

#pragma once

#include <type_traits>
#include <utility>

#include "tsq_internal.h"

namespace tsq {
namespace {

// ------------------------------------------------------------------ scalars

__device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// DPP wavefront shifts: lane i receives lane i-1 (from_left) or i+1 (from_right).
// Lanes without a source receive 0 (bound_ctrl); they lie in the discarded
// halo.
__device__ __forceinline__ int dpp_from_left(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_from_right(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_from_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_from_right(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v) {
    return __hiloint2double(dpp_from_left(__double2hiint(v)), dpp_from_left(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v) {
    return __hiloint2double(dpp_from_right(__double2hiint(v)), dpp_from_right(__double2loint(v)));
}

// One site of a 2x2 block exponential [[c, i s], [i s, c]] with its partner b:
//   a <- (a - d a) + i s b,   d = 1 - c.
template <class R>
__device__ __forceinline__ void rot_site(R& ar, R& ai, R br, R bi, R s, R d) {
    R nr = mad(-s, bi, mad(-d, ar, ar));
    R ni = mad(s, br, mad(-d, ai, ai));
    ar = nr;
    ai = ni;
}

template <class R>
__device__ __forceinline__ void rot_pair(R& ar, R& ai, R& br, R& bi, R s, R d) {
    R a0 = ar, a1 = ai;
    rot_site(ar, ai, br, bi, s, d);
    rot_site(br, bi, a0, a1, s, d);
}

// Tangent form of a pair rotation: (a, b) <- (a + i t b, b + i t a), which is
// sec(al) times the block exponential for t = tan(al); the cos(al) factors it
// leaves out are applied by the odd x factor of the same step.
template <class R>
__device__ __forceinline__ void rot_pair_t(R& ar, R& ai, R& br, R& bi, R t) {
    const R a0 = ar, a1 = ai;
    ar = mad(-t, bi, ar);
    ai = mad(t, br, ai);
    br = mad(-t, a1, br);
    bi = mad(t, a0, bi);
}

// Potential phase, complex128: psi <- psi * p, p = exp(-i phi) in FP64.
__device__ __forceinline__ void apply_phase(double& re, double& im, const double2 p) {
    double t = im * p.y;
    double nr = mad(re, p.x, -t);
    double ni = mad(re, p.y, im * p.x);
    re = nr;
    im = ni;
}

// Potential phase, complex64: p = (hi.re, hi.im, lo.re, lo.im) with
// hi + lo the table's 31-bit value of exp(-i phi); the lo product is formed
// first so the table's rounding to complex64 adds no coherent per-site error
// step after step.
__device__ __forceinline__ void apply_phase(float& re, float& im, const float4 p) {
    float tr = mad(re, p.z, -(im * p.w));
    float ti = mad(re, p.w, im * p.z);
    float nr = mad(re, p.x, mad(-im, p.y, tr));
    float ni = mad(re, p.y, mad(im, p.x, ti));
    re = nr;
    im = ni;
}

// ------------------------------------------------------------------ time-dependent phase

// Phase factor of step n under V0 + f_n W, g * exp(-i x) with x = theta0 + f_n w
// (tw = (theta0, w) of the site, f = f_n), in FP64, by angle addition:
// x = j pi/1024 + r with j the integer nearest x * 1024/pi and |r| <= pi/2048,
// exp(-i x) = exp(-i j pi/1024) exp(-i r).  `turns` holds the kTurns = 2048
// factors g exp(-i j pi/1024), j mod 2048 (g is the cosine restoration of a
// periodic mesh's tangent form, 1 between walls); exp(-i r) comes from the
// Taylor series of cos and sin on the small interval.  The factor is a
// function of (theta0, w, f_n) alone, so every schedule forms the same bits.
// Reduction: r = x - j C1 in one FMA (the product exact), C1 the double
// nearest pi/1024; the part of j pi/1024 that C1 misses, below |j| 1.2e-19 =
// |x| 3.9e-17, is under half the unit in the last place of x itself, the
// rounding x already carries (a second Cody-Waite term would refine r below
// that).  j comes from adding 1.5 * 2^52 inside the FMA that forms
// x * 1024/pi: the low bits of the sum's significand then hold j, for
// |x| < 2^51 pi/1024 (about 2^42.6).
// FULL (complex128): sin r through r^3, cos r through r^4 (first omitted terms
// below 7.1e-17, under half a unit in the last place of 1, and 1.9e-20).
// Otherwise (complex64, whose state keeps 24 bits): sin r as r, cos r through
// r^2 (omitted below 6.1e-10 and 2.4e-13 per step: the first is a phase offset
// of the order of the complex64 table's own 2^-31 fixed-point rounding).
struct TdTurn {
    double r;   // reduced angle, |r| <= pi/2048
    double2 u;  // g exp(-i j pi/1024) from the table
};
__device__ __forceinline__ TdTurn td_reduce(const double2 tw, double f, const double2* turns) {
    const double C1 = 0x1.921fb54442d18p-9;   // pi/1024 rounded to double
    const double shifter = 0x1.8p52;          // 1.5 * 2^52: unit in the last place 1
    const double x = mad(f, tw.y, tw.x);
    const double t = mad(x, 0x1.45f306dc9c883p+8, shifter);  // x * (1024/pi) + shifter
    const double j = t - shifter;                              // exact
    const unsigned idx = (unsigned)__double2loint(t) & (unsigned)(kTurns - 1);  // j mod 2048
    return TdTurn{mad(-j, C1, x), turns[idx]};
}
template <bool FULL>
__device__ __forceinline__ double2 td_combine(const TdTurn& q) {
    const double r = q.r;
    const double r2 = r * r;
    double sr = r;                              // sin r
    double cr;                                  // cos r
    if constexpr (FULL) {
        sr = mad(r * r2, -1.0 / 6.0, r);
        cr = mad(r2, mad(r2, 1.0 / 24.0, -0.5), 1.0);
    } else {
        cr = mad(r2, -0.5, 1.0);
    }
    const double2 u = q.u;
    // (u.x + i u.y)(cr - i sr)
    return make_double2(mad(u.x, cr, u.y * sr), mad(u.y, cr, -(u.x * sr)));
}

// Apply the factor times the site's scale k (closed meshes; SCALE = false:
// k = 1): complex128 in place; complex64 widened to FP64, multiplied, rounded
// once.
template <bool SCALE>
__device__ __forceinline__ double2 td_factor(const double2 p, double k) {
    if constexpr (SCALE)
        return make_double2(p.x * k, p.y * k);
    else
        return (void)k, p;
}
template <bool SCALE>
__device__ __forceinline__ void apply_phase_td(double& re, double& im, const TdTurn& q, double k) {
    apply_phase(re, im, td_factor<SCALE>(td_combine<true>(q), k));
}
template <bool SCALE>
__device__ __forceinline__ void apply_phase_td(float& re, float& im, const TdTurn& q, double k) {
    const double2 p = td_factor<SCALE>(td_combine<false>(q), k);
    const double r = re, i = im;
    re = (float)mad(r, p.x, -(i * p.y));
    im = (float)mad(r, p.y, i * p.x);
}

// ------------------------------------------------------------------ dtype traits

// R: the real type of psi.  PT: a phase factor as the march holds it in
// registers.  TT: a phase factor as the table stores it in device memory.
struct C128 {
    using R = double;
    using PT = double2;
    using TT = double2;
};
struct C64 {
    using R = float;
    using PT = float4;
    using TT = int2;
};

// Phase table entry -> phase factor.  complex128: exp(-i phi) as is.
// complex64: the table holds cos(phi) and -sin(phi) as 32-bit fixed-point
// numbers (scale 2^30; 8 bytes, the size of a complex64, but about 31 bits
// per part instead of 24, so the coherent per-site error of a rounded table,
// repeated every step, stays below 7e-10 per step); they split exactly into a
// hi float (the top 24 bits) and a lo float (the low 7 bits), the pair the
// complex64 phase multiply takes.
__device__ __forceinline__ double2 decode_phase(double2 t) { return t; }
__device__ __forceinline__ float4 decode_phase(int2 t) {
    const float sc = 0x1p-30f;
    const int hx = t.x & ~0x7f, hy = t.y & ~0x7f;
    return make_float4((float)hx * sc, (float)hy * sc, (float)(t.x - hx) * sc,
                       (float)(t.y - hy) * sc);
}

template <class R, int SPL>
struct Row {
    R re[SPL];
    R im[SPL];
};

// Load / store one x-pair (2 sites starting at even column `x`) of row `r`.
template <int SPL>
__device__ __forceinline__ void load_pair(const void* base, long long off, Row<double, SPL>& row, int p) {
    const double2* q = reinterpret_cast<const double2*>(base) + off;
    double2 a = q[0], b = q[1];
    row.re[2 * p] = a.x; row.im[2 * p] = a.y;
    row.re[2 * p + 1] = b.x; row.im[2 * p + 1] = b.y;
}
template <int SPL>
__device__ __forceinline__ void load_pair(const void* base, long long off, Row<float, SPL>& row, int p) {
    const float4 a = *reinterpret_cast<const float4*>(reinterpret_cast<const float2*>(base) + off);
    row.re[2 * p] = a.x; row.im[2 * p] = a.y;
    row.re[2 * p + 1] = a.z; row.im[2 * p + 1] = a.w;
}
// Stores are nontemporal: a pass writes each site once and nothing reads it
// back before the next pass, so the lines should not displace the halo rows
// that neighbouring tiles re-read from L2.
typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float4 __attribute__((ext_vector_type(4)));
template <int SPL>
__device__ __forceinline__ void store_pair(void* base, long long off, const Row<double, SPL>& row, int p) {
    nt_double2* q = reinterpret_cast<nt_double2*>(base) + off;
    const nt_double2 a = {row.re[2 * p], row.im[2 * p]};
    const nt_double2 b = {row.re[2 * p + 1], row.im[2 * p + 1]};
    __builtin_nontemporal_store(a, q);
    __builtin_nontemporal_store(b, q + 1);
}
template <int SPL>
__device__ __forceinline__ void store_pair(void* base, long long off, const Row<float, SPL>& row, int p) {
    const nt_float4 v = {row.re[2 * p], row.im[2 * p], row.re[2 * p + 1], row.im[2 * p + 1]};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_float4*>(reinterpret_cast<float2*>(base) + off));
}

// ------------------------------------------------------------------ row operators

// Which x-pairs of a lane exist.  Periodic meshes have every pair (the
// struct is empty and the checks vanish); closed meshes have no pair that
// crosses a wall: such a pair is rotated with zero coefficients (s = d = 0
// leaves both sites exactly as they were, up to the sign of a zero), so the
// sites inside keep their values and whatever a site outside the mesh holds
// never reaches one inside.
template <int PPL, bool CLOSED>
struct XPairs {
    bool even[PPL];      // (x, x+1) of pair p
    bool inner[PPL];     // (x+1, x+2) inside the lane, p < PPL-1
    bool left, right;    // odd pairs shared with the neighbouring lanes
    double kx[2 * PPL];  // time-dependent phase: the site's column scale (last odd column)
};
template <int PPL>
struct XPairs<PPL, false> {};

// The coefficient of a pair that exists, else 0.
template <bool CLOSED, class R>
__device__ __forceinline__ R pair_coef(bool exists, R c) {
    if constexpr (CLOSED)
        return exists ? c : R(0);
    else
        return (void)exists, c;
}

// Even x-pairs: inside the lane.
template <bool CLOSED, class R, int SPL>
__device__ __forceinline__ void even_x(Row<R, SPL>& w, R s, R d, const XPairs<SPL / 2, CLOSED>& m) {
#pragma unroll
    for (int p = 0; p < SPL / 2; ++p) {
        bool ok = true;
        if constexpr (CLOSED) ok = m.even[p];
        rot_pair(w.re[2 * p], w.im[2 * p], w.re[2 * p + 1], w.im[2 * p + 1],
                 pair_coef<CLOSED>(ok, s), pair_coef<CLOSED>(ok, d));
    }
}

// Odd x-pairs in the tangent form (periodic meshes): inner ones inside the
// lane, the two at the lane edges across lanes.
template <class R, int SPL>
__device__ __forceinline__ void odd_x_t(Row<R, SPL>& w, R t) {
    const R rr = from_right(w.re[0]), ri = from_right(w.im[0]);
    const R lr = from_left(w.re[SPL - 1]), li = from_left(w.im[SPL - 1]);
#pragma unroll
    for (int p = 0; p + 1 < SPL / 2; ++p)
        rot_pair_t(w.re[2 * p + 1], w.im[2 * p + 1], w.re[2 * p + 2], w.im[2 * p + 2], t);
    w.re[SPL - 1] = mad(-t, ri, w.re[SPL - 1]);
    w.im[SPL - 1] = mad(t, rr, w.im[SPL - 1]);
    w.re[0] = mad(-t, li, w.re[0]);
    w.im[0] = mad(t, lr, w.im[0]);
}

// Odd x-pairs: inner ones inside the lane, the two at the lane edges across lanes.
template <bool CLOSED, class R, int SPL>
__device__ __forceinline__ void odd_x(Row<R, SPL>& w, R s, R d, const XPairs<SPL / 2, CLOSED>& m) {
    R rr = from_right(w.re[0]), ri = from_right(w.im[0]);
    R lr = from_left(w.re[SPL - 1]), li = from_left(w.im[SPL - 1]);
#pragma unroll
    for (int p = 0; p + 1 < SPL / 2; ++p) {
        bool ok = true;
        if constexpr (CLOSED) ok = m.inner[p];
        rot_pair(w.re[2 * p + 1], w.im[2 * p + 1], w.re[2 * p + 2], w.im[2 * p + 2],
                 pair_coef<CLOSED>(ok, s), pair_coef<CLOSED>(ok, d));
    }
    bool ok_r = true, ok_l = true;
    if constexpr (CLOSED) {
        ok_r = m.right;
        ok_l = m.left;
    }
    rot_site(w.re[SPL - 1], w.im[SPL - 1], rr, ri, pair_coef<CLOSED>(ok_r, s), pair_coef<CLOSED>(ok_r, d));
    rot_site(w.re[0], w.im[0], lr, li, pair_coef<CLOSED>(ok_l, s), pair_coef<CLOSED>(ok_l, d));
}

// y-pair made of row `u` (upper, smaller y) and row `v` (next row).
template <class R, int SPL>
__device__ __forceinline__ void pair_y(Row<R, SPL>& u, Row<R, SPL>& v, R s, R d) {
#pragma unroll
    for (int i = 0; i < SPL; ++i) rot_pair(u.re[i], u.im[i], v.re[i], v.im[i], s, d);
}

// The same in the tangent form (periodic meshes).
template <class R, int SPL>
__device__ __forceinline__ void pair_y_t(Row<R, SPL>& u, Row<R, SPL>& v, R t) {
#pragma unroll
    for (int i = 0; i < SPL; ++i) rot_pair_t(u.re[i], u.im[i], v.re[i], v.im[i], t);
}

// Even x-pairs in the tangent form (closed meshes: a zero tangent for a pair
// that reaches beyond the wall).
template <bool CLOSED, class R, int SPL>
__device__ __forceinline__ void even_x_t(Row<R, SPL>& w, R t, const XPairs<SPL / 2, CLOSED>& m) {
#pragma unroll
    for (int p = 0; p < SPL / 2; ++p) {
        bool ok = true;
        if constexpr (CLOSED) ok = m.even[p];
        rot_pair_t(w.re[2 * p], w.im[2 * p], w.re[2 * p + 1], w.im[2 * p + 1], pair_coef<CLOSED>(ok, t));
    }
}

template <class PT, class R, int SPL>
__device__ __forceinline__ void phase_row(Row<R, SPL>& w, const PT* p) {
#pragma unroll
    for (int i = 0; i < SPL; ++i) apply_phase(w.re[i], w.im[i], p[i]);
}

// Both rows of a pair: every site's reduction and table read first, so the
// LDS reads are in flight together, then the factors.  SCALE (closed meshes):
// site i of row a (b) takes the scale kx[i] * ka (kx[i] * kb).
template <bool SCALE, class R, int SPL>
__device__ __forceinline__ void phase_rows_td(Row<R, SPL>& a, Row<R, SPL>& b, const double2* pa,
                                              const double2* pb, double f, const double2* turns,
                                              const double* kx, double ka, double kb) {
    TdTurn qa[SPL], qb[SPL];
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        qa[i] = td_reduce(pa[i], f, turns);
        qb[i] = td_reduce(pb[i], f, turns);
    }
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        apply_phase_td<SCALE>(a.re[i], a.im[i], qa[i], SCALE ? kx[i] * ka : 1.0);
        apply_phase_td<SCALE>(b.re[i], b.im[i], qb[i], SCALE ? kx[i] * kb : 1.0);
    }
}

// Calls f(integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>());
}
// f(integral_constant<int, i>) for i = 0 .. N-1 while the calls return true;
// true if all did.
template <class F, int... Is>
__device__ __forceinline__ bool static_all_impl(F&& f, std::integer_sequence<int, Is...>) {
    return (f(std::integral_constant<int, Is>{}) && ...);
}
template <int N, class F>
__device__ __forceinline__ bool static_all(F&& f) {
    return static_all_impl(f, std::make_integer_sequence<int, N>());
}

// Row pairs of a march are named by the direction of travel: row F of a pair
// faces the pairs marched before it, row G the pairs marched after it.
// Marching down (increasing y) F is the pair's top row 2t and G its bottom
// row 2t+1; marching up the two swap.  The odd y-pair joining an older pair
// to the next newer one is (G of the older, F of the newer) either way, and
// the rotation of a pair is symmetric in its two sites, so one code path
// serves both directions with every site seeing the same operations in the
// same order.
template <class R, int SPL>
struct PairRows {
    Row<R, SPL> f, g;
};

template <class PT, int SPL>
struct PhasePair {
    PT f[SPL], g[SPL];
};

__device__ __forceinline__ int rstep_of(bool rev) { return rev ? -2 : 2; }

__device__ __forceinline__ int wrap(long long v, int n) {
    long long m = v % n;
    return (int)(m < 0 ? m + n : m);
}

// Stage k on a closed mesh (see pipeline_stage): the odd factors in the delta
// form, the even factors in the tangent form with the phase factor restoring
// their cosines site by site (see MarchArgs).  A pair that reaches beyond a
// wall rotates with zero coefficients (x: per lane; y: a wavefront-uniform
// choice, no branch).
template <int S, bool TD, class R, int SPL, class PhaseFn>
__device__ __forceinline__ void closed_stage(int k, PairRows<R, SPL>& o, PairRows<R, SPL>& n,
                                             const MarchArgs<R>& a, const XPairs<SPL / 2, true>& xm,
                                             int qk, bool rev, const double2* turns, PhaseFn&& phase,
                                             R oxs, R oxd, R oys, R oyd) {
    // odd y-pair: rows (2qk+1, 2qk+2) marching down, (2qk-1, 2qk) marching up;
    // even y-pair of o: rows (2qk, 2qk+1)
    const bool oy_ok = rev ? (qk >= 1 && 2 * qk < a.ny) : (qk >= 0 && 2 * qk + 2 < a.ny);
    const bool ey_ok = qk >= 0 && 2 * qk + 1 < a.ny;
    odd_x<true>(o.g, oxs, oxd, xm);
    odd_x<true>(n.f, oxs, oxd, xm);
    pair_y(o.g, n.f, oy_ok ? oys : R(0), oy_ok ? oyd : R(0));
    if (k < S) {
        const auto ph = phase(k);
        const R eyt = ey_ok ? a.ehys : R(0);
        even_x_t<true>(o.f, a.ehxs, xm);
        even_x_t<true>(o.g, a.ehxs, xm);
        pair_y_t(o.f, o.g, eyt);
        if constexpr (TD) {
            // the shared factors carry the cosines of a site with both even
            // partners; the last column (row) of an odd width (height) takes
            // the scale of the factor it sits out of
            const int rf = rev ? 2 * qk + 1 : 2 * qk, rg = rev ? 2 * qk : 2 * qk + 1;
            const bool odd_h = (a.ny & 1) != 0;
            const double kf = (odd_h && rf == a.ny - 1) ? a.kyw : 1.0;
            const double kg = (odd_h && rg == a.ny - 1) ? a.kyw : 1.0;
            phase_rows_td<true>(o.f, o.g, ph.f, ph.g, a.g[k], turns, xm.kx, kf, kg);
        } else {
            phase_row(o.f, ph.f);
            phase_row(o.g, ph.g);
        }
        pair_y_t(o.f, o.g, eyt);
        even_x_t<true>(o.f, a.ehxs, xm);
        even_x_t<true>(o.g, a.ehxs, xm);
    }
}

// Stage k of the S-stage pipeline.  `o` is the older row pair, the one stage
// k completes; `n` is the newer pair right behind it, just finished by stage
// k-1 (or just loaded, for k = 0).  Stage k applies the odd factors on the
// boundary of the two (o's G row and n's F row; n's G row gets the same
// factors in stage k+1, where n is the older pair), then, for k < S, step
// k+1's even factors and the potential phase on o.  Stage K-1 = S of the
// last pass applies only the closing odd factors.  With a time-dependent
// potential (TD) the phase pair holds (theta0, w) per site and stage k forms
// step k's factor from a.g[k] and `turns` (LDS).  Closed meshes rotate the
// pairs that cross a wall with zero coefficients (y: `qk` is the pair stage k
// completes; a wavefront-uniform test) and apply the odd factors in the
// delta form, the even factors in the tangent form; periodic meshes apply the
// tangent form, the
// odd x factors of stage 0 and of the closing stage in the delta form that
// restores the cosines the phase factor does not (see MarchArgs).
template <int S, int K, bool CLOSED, bool TD, bool U4, class R, int SPL, class PT, class PhaseFn>
__device__ __forceinline__ void pipeline_stage(int k, PairRows<R, SPL>& o, PairRows<R, SPL>& n,
                                               const MarchArgs<R>& a,
                                               const XPairs<SPL / 2, CLOSED>& xm, int qk, bool rev,
                                               const double2* turns, PhaseFn&& phase) {
    if constexpr (U4) {
        // one fourth-order step: sub-steps p, p, m, p, p (Eq. "fourthorder");
        // stage k's odd x factor (delta form) carries its own cosines over
        // those its table holds, its odd y and even factors are tangents of
        // its kinds, stage 2 takes the m table
        (void)qk; (void)rev;
        odd_x<false>(o.g, a.u4.xs[k], a.u4.xd[k], xm);
        odd_x<false>(n.f, a.u4.xs[k], a.u4.xd[k], xm);
        pair_y_t(o.g, n.f, a.u4.yt[k]);
        if (k < S) {
            const int q = k == 2 ? 1 : 0;
            const PhasePair<PT, SPL> ph = phase(k);
            even_x_t<CLOSED>(o.f, a.u4.ext[q], xm);
            even_x_t<CLOSED>(o.g, a.u4.ext[q], xm);
            pair_y_t(o.f, o.g, a.u4.eyt[q]);
            phase_row(o.f, ph.f);
            phase_row(o.g, ph.g);
            pair_y_t(o.f, o.g, a.u4.eyt[q]);
            even_x_t<CLOSED>(o.f, a.u4.ext[q], xm);
            even_x_t<CLOSED>(o.g, a.u4.ext[q], xm);
        }
        return;
    }
    R oxs, oxd, oys, oyd;
    if (k == 0) {
        oxs = a.o1xs; oxd = a.o1xd; oys = a.o1ys; oyd = a.o1yd;
    } else if (k < S) {
        oxs = a.o2xs; oxd = a.o2xd; oys = a.o2ys; oyd = a.o2yd;
    } else {
        oxs = a.c1xs; oxd = a.c1xd; oys = a.c1ys; oyd = a.c1yd;
    }
    if constexpr (!CLOSED) {
        (void)oyd; (void)qk; (void)rev;
        if (k == 0 || k == S) {
            odd_x<false>(o.g, oxs, oxd, xm);
            odd_x<false>(n.f, oxs, oxd, xm);
        } else {
            odd_x_t(o.g, oxs);
            odd_x_t(n.f, oxs);
        }
        pair_y_t(o.g, n.f, oys);
        if (k < S) {
            const PhasePair<PT, SPL> ph = phase(k);
            even_x_t<false>(o.f, a.ehxs, xm);
            even_x_t<false>(o.g, a.ehxs, xm);
            pair_y_t(o.f, o.g, a.ehys);
            if constexpr (TD) {
                phase_rows_td<false>(o.f, o.g, ph.f, ph.g, a.g[k], turns, nullptr, 1.0, 1.0);
            } else {
                phase_row(o.f, ph.f);
                phase_row(o.g, ph.g);
            }
            pair_y_t(o.f, o.g, a.ehys);
            even_x_t<false>(o.f, a.ehxs, xm);
            even_x_t<false>(o.g, a.ehxs, xm);
        }
    } else {
        closed_stage<S, TD>(k, o, n, a, xm, qk, rev, turns, phase, oxs, oxd, oys, oyd);
    }
}

// Phase factors of the row pairs inside the pipeline are held either in
// registers (LDS = false) or, for stages 1..S-1, in a per-lane LDS ring
// (LDS = true; stage 0 reads registers).
// LDS ring of one wavefront: [slot][row][site][lane] phase factors.
template <class PT, int S, int PPL, bool LDS>
struct WaveRing {
    static constexpr int kSlots = (LDS && S > 1) ? S - 1 : 1;
    PT v[kSlots][2][2 * PPL][kWaveSize];
};

// Site-wise loads and stores for closed meshes (odd sides allowed, so rows
// need not start on a 16-byte boundary).
__device__ __forceinline__ void load_site(const void* base, long long off, double& re, double& im) {
    const double2 v = reinterpret_cast<const double2*>(base)[off];
    re = v.x;
    im = v.y;
}
__device__ __forceinline__ void load_site(const void* base, long long off, float& re, float& im) {
    const float2 v = reinterpret_cast<const float2*>(base)[off];
    re = v.x;
    im = v.y;
}
__device__ __forceinline__ void store_site(void* base, long long off, double re, double im) {
    reinterpret_cast<double2*>(base)[off] = make_double2(re, im);
}
__device__ __forceinline__ void store_site(void* base, long long off, float re, float im) {
    reinterpret_cast<float2*>(base)[off] = make_float2(re, im);
}
template <class PT>
__device__ __forceinline__ PT zero_phase() {
    PT z;
    if constexpr (sizeof(PT) == 16 && alignof(PT) == 16 && sizeof(z.x) == 4) {
        z.x = z.y = z.z = z.w = 0.f;
    } else {
        z.x = z.y = 0.0;
    }
    return z;
}

// March one tile (strip, segment) of one pass; `ring` is this lane's column of
// the wavefront's LDS ring (unused with register phases).  `rev` marches the
// segment upwards: odd segments do, so two neighbouring segments cross the
// rows they both read (each other's warm-up halo) at the same time, start or
// end, and the second read can hit L2.  CLOSED: hard walls instead of
// periodic wrap (rows and columns outside the mesh hold values that no
// rotation carries inside and that are never stored).
//
// Register homes: the row pair that enters the pipeline in iteration j lives
// in home j mod NH until it is stored K iterations later; stage k of
// iteration j works on homes j-1-k (older) and j-k (newer).  Loads run PF
// iterations ahead: the pair for iteration j+PF is loaded into home j+PF
// meanwhile, so a load has PF iterations of stages to arrive (one iteration
// of one wavefront does not cover the memory latency at the occupancy the LDS
// ring allows), and NH = K+1+PF homes suffice; the march loop, unrolled by
// NH, moves no data between registers.  Phases: the phase rows of pair j are
// loaded in iteration j+1-PF and first used by stage 0 in iteration j+1;
// register phases keep one home per psi home, the LDS ring keeps PF+1
// register homes (pairs j+PF-1 .. j-1) and moves pair j-1's phase to the
// ring at the end of iteration j.  complex64 runs PF = 2; complex128, the
// time-dependent march and the fourth-order pass PF = 1.  The fourth-order
// pass keeps PF+1 homes of m-table phases as well (its stage 2 takes the m
// table).
template <class T, bool TD>
using PhaseT = std::conditional_t<TD, double2, typename T::PT>;
template <class T, bool TD>
using TableT = std::conditional_t<TD, double2, typename T::TT>;

template <class T, int S, bool LAST, int PPL, bool LDS, bool CLOSED, bool TD, bool U4>
__device__ __forceinline__ void march_tile(const MarchArgs<typename T::R>& a, int strip, int seg,
                                           bool rev, int lane, PhaseT<T, TD>* ring,
                                           const double2* turns) {
    using R = typename T::R;
    using PT = PhaseT<T, TD>;
    constexpr int SPL = 2 * PPL;
    constexpr int K = S + (LAST ? 1 : 0);
    constexpr int HL = (K + PPL - 1) / PPL;
    constexpr int NL = WaveRing<PT, S, PPL, LDS>::kSlots;
    // load distance (iterations): complex128 rows already put twice the bytes
    // in flight per load and its registers are full at two wavefronts per SIMD;
    // the time-dependent and fourth-order marches are bound by their
    // arithmetic, not their loads (two ahead measured 2-8% slower there)
    constexpr int PF = (U4 || TD || sizeof(R) == 8) ? 1 : 2;
    constexpr int NH0 = K + 1 + PF;
    constexpr int NP = LDS ? PF + 1 : NH0;             // phase homes
    // with the LDS ring a multiple of NP, so every phase home index is static
    constexpr int NH = LDS ? (NH0 + NP - 1) / NP * NP : NH0;
    static_assert(!U4 || (LDS && S == 5 && !CLOSED && !TD && PPL == 1),
                  "the fourth-order pass is 5 sub-steps, LDS ring, periodic, one pair per lane");
    const int nx = a.nx, ny = a.ny;

    // x: unwrapped column of the lane's first site; wrapped (periodic) or
    // unwrapped (closed) column of each pair; which sites exist and which
    // lanes store.
    const long long xu0 = (long long)strip * a.strip_sites + (long long)(lane - HL) * SPL;
    const bool inner = lane >= HL && lane < kWaveSize - HL;
    int col[PPL];
    bool keep[PPL];
    bool site_ok[SPL];
    XPairs<PPL, CLOSED> xm;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        col[p] = CLOSED ? (int)(xu0 + 2 * p) : wrap(xu0 + 2 * p, nx);
        keep[p] = inner && (xu0 + 2 * p) < nx;
    }
#pragma unroll
    for (int i = 0; i < SPL; ++i) site_ok[i] = !CLOSED || (xu0 + i >= 0 && xu0 + i < nx);
    if constexpr (CLOSED) {
        auto in = [&](long long x) { return x >= 0 && x < nx; };
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            xm.even[p] = in(xu0 + 2 * p) && in(xu0 + 2 * p + 1);
            xm.inner[p] = in(xu0 + 2 * p + 1) && in(xu0 + 2 * p + 2);
        }
        xm.left = in(xu0 - 1) && in(xu0);
        xm.right = in(xu0 + SPL - 1) && in(xu0 + SPL);
#pragma unroll
        for (int i = 0; i < SPL; ++i) xm.kx[i] = ((nx & 1) && xu0 + i == nx - 1) ? a.kxw : 1.0;
    }
    // Closed meshes: a site outside the mesh loads any site inside (its column
    // and row clamped to the mesh) instead of a zero, since no rotation lets
    // its value reach a site inside (x-pairs reaching outside run with zero
    // coefficients, y-pairs reaching outside are skipped) and it is never
    // stored; the loads need no condition.
    int ccol[SPL];
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        const long long x = xu0 + i;
        ccol[i] = CLOSED ? (int)(x < 0 ? 0 : (x >= nx ? nx - 1 : x)) : 0;
    }
    auto clamp_row = [&](int r) { return r < 0 ? 0 : (r >= ny ? ny - 1 : r); };

    // y: output row pairs [q0, q1); input pairs [q0 - K, q1 - 1 + K], visited in
    // increasing order (decreasing when marching up).  `rpsi` and `rph` are the
    // first rows of the next pair whose psi, respectively phase, is loaded,
    // stepped by two rows (periodic wrap; closed meshes leave them unwrapped
    // and load rows outside [0, ny) from the nearest row of the mesh).
    const int hp = CLOSED ? (ny + 1) >> 1 : ny >> 1;
    const int q0 = seg * (a.seg_rows >> 1);
    const int q1 = min(q0 + (a.seg_rows >> 1), hp);
    const int nit = (q1 - q0) + 2 * K;
    const int tstart = rev ? q1 - 1 + K : q0 - K;
    const int fo = rev ? 1 : 0;  // row offset of F within a pair; G is at 1 - fo
    int rpsi = CLOSED ? 2 * tstart : wrap(2LL * tstart, ny);
    int rph = rpsi;
    // fourth order: the m-table phase of the pair stage 2 completes PF
    // iterations later, i.e. two pairs behind the pair whose phase `rph` loads
    // in the same iteration (3 - PF pairs behind the first psi pair; the
    // fourth-order pass is periodic only)
    int rphm = rpsi;
    if constexpr (U4) rphm = wrap((long long)rpsi - (3 - PF) * rstep_of(rev), ny);
    int qout = rev ? q1 - 1 + 2 * K : q0 - 2 * K;  // pair leaving the pipeline this iteration

    const int rstep = rev ? -2 : 2;
    auto step_row = [&](int& r) {
        r += rstep;
        if constexpr (!CLOSED) {
            r = r < 0 ? r + ny : r;
            r = r >= ny ? r - ny : r;
        }
    };
    auto load_row = [&](int r, Row<R, SPL>& w) {
        if constexpr (CLOSED) {
            const long long off = (long long)clamp_row(r) * nx;
#pragma unroll
            for (int i = 0; i < SPL; ++i) load_site(a.src, off + ccol[i], w.re[i], w.im[i]);
        } else {
            const long long off = (long long)r * nx;
#pragma unroll
            for (int p = 0; p < PPL; ++p) load_pair(a.src, off + col[p], w, p);
        }
    };
    auto load_psi = [&](PairRows<R, SPL>& h) {
        load_row(rpsi + fo, h.f);
        load_row(rpsi + 1 - fo, h.g);
        step_row(rpsi);
    };
    auto load_phase_row = [&](int r, PT (&v)[SPL]) {
        const TableT<T, TD>* P = reinterpret_cast<const TableT<T, TD>*>(a.ptab);
        if constexpr (CLOSED) {
            const long long off = (long long)clamp_row(r) * nx;
#pragma unroll
            for (int i = 0; i < SPL; ++i) v[i] = decode_phase(P[off + ccol[i]]);
        } else {
            const long long off = (long long)r * nx;
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                v[2 * p] = decode_phase(P[off + col[p]]);
                v[2 * p + 1] = decode_phase(P[off + col[p] + 1]);
            }
        }
    };
    auto load_phase = [&](PhasePair<PT, SPL>& ph) {
        load_phase_row(rph + fo, ph.f);
        load_phase_row(rph + 1 - fo, ph.g);
        step_row(rph);
    };
    auto load_phase_m = [&](PhasePair<PT, SPL>& ph) {
        if constexpr (U4) {
            const typename T::TT* P = reinterpret_cast<const typename T::TT*>(a.ptab2);
            const long long offf = (long long)(rphm + fo) * nx;
            const long long offg = (long long)(rphm + 1 - fo) * nx;
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                ph.f[2 * p] = decode_phase(P[offf + col[p]]);
                ph.f[2 * p + 1] = decode_phase(P[offf + col[p] + 1]);
                ph.g[2 * p] = decode_phase(P[offg + col[p]]);
                ph.g[2 * p + 1] = decode_phase(P[offg + col[p] + 1]);
            }
            step_row(rphm);
        } else {
            (void)ph;
        }
    };
    auto store_out = [&](const PairRows<R, SPL>& h) {
        const int qo = qout;
        qout += rev ? -1 : 1;
        if (rev ? (qo >= q1) : (qo < q0)) return;  // still warming up
        const long long rf = 2LL * qo + fo, rg = 2LL * qo + 1 - fo;
        if constexpr (CLOSED) {
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                if (inner && site_ok[i]) {
                    if (rf < ny) store_site(a.dst, rf * nx + xu0 + i, h.f.re[i], h.f.im[i]);
                    if (rg < ny) store_site(a.dst, rg * nx + xu0 + i, h.g.re[i], h.g.im[i]);
                }
            }
        } else {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                if (keep[p]) {
                    store_pair(a.dst, rf * nx + col[p], h.f, p);
                    store_pair(a.dst, rg * nx + col[p], h.g, p);
                }
            }
        }
    };

    PairRows<R, SPL> home[NH];
    PhasePair<PT, SPL> ph[NP];
    PhasePair<PT, SPL> phm[U4 ? PF + 1 : 1];  // m-table phases (fourth order)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
            home[h].f.re[i] = home[h].f.im[i] = R(0);
            home[h].g.re[i] = home[h].g.im[i] = R(0);
        }
    }
#pragma unroll
    for (int h = 0; h < NP; ++h) {
#pragma unroll
        for (int i = 0; i < SPL; ++i) ph[h].f[i] = ph[h].g[i] = zero_phase<PT>();
    }
#pragma unroll
    for (int h = 0; h < (U4 ? PF + 1 : 1); ++h) {
#pragma unroll
        for (int i = 0; i < SPL; ++i) phm[h].f[i] = phm[h].g[i] = zero_phase<PT>();
    }

    constexpr int SLOT = 2 * SPL * kWaveSize;  // PT elements per LDS slot
    int wslot = 0;  // LDS slot receiving the phase of pair j-1 at the end of iteration j
    int q = rev ? tstart + 1 : tstart - 1;  // pair stage 0 completes this iteration
    const int qend = rev ? q - nit : q + nit;  // ... one past the last iteration
    // Stage k in iteration i (0-based) completes the pair 1+k behind the one
    // loaded, which reaches the region the stored pairs depend on (K-k pairs
    // of halo ahead of them along the march, one more for the odd boundary)
    // only from i = 2k+1 on: earlier runs fill the pipeline with values no
    // stored site depends on, and are skipped (a wavefront-uniform branch).
    int it = 0;
    load_psi(home[0]);
    if constexpr (PF == 2) {
        load_psi(home[1]);
        load_phase(ph[0]);
    }
    // One march iteration with static home indices (u = j mod NH).
    auto iteration = [&](auto U) {
        constexpr int u = decltype(U)::value;
        // The last iterations load PF pairs more than the march uses (always
        // rows of the mesh): an unconditional load keeps the homes free of
        // merges.
        load_psi(home[(u + PF) % NH]);
        load_phase(ph[(u + PF - 1) % NP]);
        if constexpr (U4) load_phase_m(phm[(u + PF) % (PF + 1)]);
        static_for<K>([&](auto KK) {
            constexpr int k = decltype(KK)::value;
            if (it > 2 * k)
            pipeline_stage<S, K, CLOSED, TD, U4, R, SPL, PT>(
                k, home[(u - 1 - k + 2 * NH) % NH], home[(u - k + 2 * NH) % NH], a, xm,
                rev ? q + k : q - k, rev, turns, [&](int kk) {
                    if (U4 && kk == 2) return phm[U4 ? u % (PF + 1) : 0];
                    if (!LDS || kk == 0) return ph[(u - 1 - kk + 2 * NP) % NP];
                    int slot = wslot - kk;
                    if (slot < 0) slot += NL;
                    PhasePair<PT, SPL> r;
#pragma unroll
                    for (int i = 0; i < SPL; ++i) {
                        r.f[i] = ring[slot * SLOT + i * kWaveSize];
                        r.g[i] = ring[slot * SLOT + (SPL + i) * kWaveSize];
                    }
                    return r;
                });
            // keep each stage's phase reads and temporaries inside the stage:
            // hoisting them across stages costs more registers than it hides
            __builtin_amdgcn_sched_barrier(0);
        });
        store_out(home[(u - K + 2 * NH) % NH]);
        q += rev ? -1 : 1;
        ++it;
        if constexpr (LDS && S > 1) {
            const PhasePair<PT, SPL>& p0 = ph[(u - 1 + 2 * NP) % NP];
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                ring[wslot * SLOT + i * kWaveSize] = p0.f[i];
                ring[wslot * SLOT + (SPL + i) * kWaveSize] = p0.g[i];
            }
            wslot = (wslot + 1 == NL) ? 0 : wslot + 1;
        }
        return q != qend;  // another iteration follows
    };
    // nit >= 2K >= 2 iterations; each round runs NH of them and the march
    // leaves right after the last (a wavefront-uniform exit, with no path
    // that carries the homes past it).
    while (static_all<NH>(iteration)) {
    }
}

// One problem, one tile per wavefront.
template <class T, int S, bool LAST, int PPL, bool LDS, bool CLOSED, bool TD, bool U4 = false>
__global__ void __launch_bounds__(kWaveSize * kWavesPerBlock)
march_kernel(const MarchArgs<typename T::R> a) {
    __shared__ WaveRing<PhaseT<T, TD>, S, PPL, LDS> rings[LDS ? kWavesPerBlock : 1];
    __shared__ double2 turns[TD ? kTurns : 1];
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    // XCD-aware block order: blocks are dealt round-robin to the 8 XCDs, so
    // block b runs on XCD b % 8; give each XCD a contiguous run of tiles, in
    // segment-major order, so the halo columns neighbouring strip groups of
    // one band of rows share (2K lanes of every 64, the larger halo) are read
    // at about the same time through one L2.  A block marches one segment of
    // kWavesPerBlock neighbouring strips (one per wavefront): the halo columns
    // two of its strips share are read by two wavefronts of one compute unit
    // at about the same time, so the second read hits the cache.
    const int nb = gridDim.x;
    const int full = nb & ~7;
    const int b = blockIdx.x;
    const int lb = (b < full) ? ((b & 7) * (full >> 3) + (b >> 3)) : b;
    const int ngroups = (a.nstrips + kWavesPerBlock - 1) / kWavesPerBlock;
    if (lb >= ngroups * a.nsegs) return;  // uniform per block
    if constexpr (TD) {
        // the time-dependent phase's table of kTurns factors, kTurns / 256 per thread
        constexpr int kThreads = kWaveSize * kWavesPerBlock;
        static_assert(kTurns % kThreads == 0, "whole table entries per thread");
#pragma unroll
        for (int e = 0; e < kTurns / kThreads; ++e)
            turns[threadIdx.x + e * kThreads] =
                reinterpret_cast<const double2*>(a.ptab2)[threadIdx.x + e * kThreads];
        __syncthreads();
    }
    const int seg = lb / ngroups;
    const int grp = lb - seg * ngroups;
    const int strip = grp * kWavesPerBlock + wave;
    if (strip >= a.nstrips) return;  // uniform per wavefront
    march_tile<T, S, LAST, PPL, LDS, CLOSED, TD, U4>(a, strip, seg, seg & 1, lane,
                                                 &rings[LDS ? wave : 0].v[0][0][0][lane], turns);
}

// Many problems: a fixed grid of wavefronts walks a work list of tiles
// (job, strip, segment), wavefront w taking tiles w, w + W, w + 2W, ...; the
// host sorts the list by tile height so the strided walk balances the load.
template <class T, int S, bool LAST, int PPL, bool LDS>
__global__ void __launch_bounds__(kWaveSize * kWavesPerBlock)
march_batch_kernel(const MarchArgs<typename T::R>* __restrict__ jobs,
                   const BatchTile* __restrict__ tiles, int ntiles) {
    __shared__ WaveRing<typename T::PT, S, PPL, LDS> rings[LDS ? kWavesPerBlock : 1];
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    const int nw = gridDim.x * kWavesPerBlock;
    for (int i = blockIdx.x * kWavesPerBlock + wave; i < ntiles; i += nw) {
        const BatchTile t = tiles[i];
        const MarchArgs<typename T::R> a = jobs[t.job];
        march_tile<T, S, LAST, PPL, LDS, false, false, false>(a, t.strip, t.seg, t.seg & 1, lane,
                                                       &rings[LDS ? wave : 0].v[0][0][0][lane],
                                                       nullptr);
    }
}

// Instances: periodic register ring for 1..kMaxRegSteps steps per pass with
// 1 pair per lane, 1..kMaxRegSteps2 with 2, periodic LDS ring for
// 1..kMaxSteps (1 pair per lane), single and batched; closed meshes: both
// rings with 1 pair per lane, single only; time-dependent potentials
// (periodic or closed): both rings, 1 pair per lane, at most kMaxTdSteps
// steps per pass, single only.
enum class Variant { Single, Batch, Closed, TimeDep, ClosedTimeDep, Order4 };

template <class T, int S, bool LAST, int PPL, bool LDS, Variant V>
const void* kernel_ptr() {
    if constexpr (V == Variant::Order4) {
        if constexpr (S == 5 && PPL == 1 && LDS)
            return reinterpret_cast<const void*>(&march_kernel<T, 5, LAST, 1, true, false, false, true>);
        else
            return nullptr;
    } else if constexpr (V == Variant::Single)
        return reinterpret_cast<const void*>(&march_kernel<T, S, LAST, PPL, LDS, false, false>);
    else if constexpr (V == Variant::Batch)
        return reinterpret_cast<const void*>(&march_batch_kernel<T, S, LAST, PPL, LDS>);
    else if constexpr (PPL != 1)
        return nullptr;
    else if constexpr (V == Variant::Closed)
        return reinterpret_cast<const void*>(&march_kernel<T, S, LAST, PPL, LDS, true, false>);
    else if constexpr (V == Variant::TimeDep)
        return reinterpret_cast<const void*>(&march_kernel<T, S, LAST, PPL, LDS, false, true>);
    else
        return reinterpret_cast<const void*>(&march_kernel<T, S, LAST, PPL, LDS, true, true>);
}

template <class T, Variant V, bool LAST, int PPL, bool LDS, int... Ss>
const void* pick_steps(int steps, std::integer_sequence<int, Ss...>) {
    const void* f = nullptr;
    ((steps == Ss + 1 ? (f = kernel_ptr<T, Ss + 1, LAST, PPL, LDS, V>(), 0) : 0), ...);
    return f;
}

template <class T, Variant V, bool LAST>
const void* pick_variant(int steps, int ppl, bool lds) {
    if constexpr (V == Variant::Order4)
        return (steps == 5 && ppl == 1 && lds) ? kernel_ptr<T, 5, LAST, 1, true, V>() : nullptr;
    if (lds) {
        if (ppl != 1) return nullptr;
        // the time-dependent march forms a phase factor per site and step;
        // beyond 6 steps per pass its loop outgrows the instruction cache
        if constexpr (V == Variant::TimeDep || V == Variant::ClosedTimeDep)
            return pick_steps<T, V, LAST, 1, true>(steps, std::make_integer_sequence<int, kMaxTdSteps>());
        else
            return pick_steps<T, V, LAST, 1, true>(steps, std::make_integer_sequence<int, kMaxSteps>());
    }
    if (ppl == 2) {
        if constexpr (V != Variant::Single && V != Variant::Batch) return nullptr;
        return pick_steps<T, V, LAST, 2, false>(steps, std::make_integer_sequence<int, kMaxRegSteps2>());
    }
    if constexpr (V == Variant::TimeDep || V == Variant::ClosedTimeDep)
        return pick_steps<T, V, LAST, 1, false>(steps, std::make_integer_sequence<int, kMaxTdSteps>());
    else
        return pick_steps<T, V, LAST, 1, false>(steps, std::make_integer_sequence<int, kMaxRegSteps>());
}

// Kernel of one instance of variant V (instantiates only that variant).
template <class T, Variant V>
const void* pick_kernel(int steps, bool last, int ppl, bool lds) {
    return last ? pick_variant<T, V, true>(steps, ppl, lds) : pick_variant<T, V, false>(steps, ppl, lds);
}

}  // namespace
}  // namespace tsq
