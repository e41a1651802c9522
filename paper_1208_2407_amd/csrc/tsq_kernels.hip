// HIP kernels for gfx950 of the second-order Trotter-Suzuki step
// (Wittek & Cucchietti, Sec. 2): phase-table setup, the fused step march,
// and the FP64 norm/energy reductions.
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

#include <utility>

#include "tsq_internal.h"

namespace tsq {
namespace {

// ------------------------------------------------------------------ scalars

__device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// DPP wavefront shifts: lane i receives lane i-1 (from_left) or i+1 (from_right).
// Lanes without a source receive 0; they lie in the discarded halo.
__device__ __forceinline__ int dpp_from_left(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_from_right(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
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
//   a <- a + (i s b - d a),   d = 1 - c.
template <class R>
__device__ __forceinline__ void rot_site(R& ar, R& ai, R br, R bi, R s, R d) {
    R nr = mad(-d, ar, mad(-s, bi, ar));
    R ni = mad(-d, ai, mad(s, br, ai));
    ar = nr;
    ai = ni;
}

template <class R>
__device__ __forceinline__ void rot_pair(R& ar, R& ai, R& br, R& bi, R s, R d) {
    R a0 = ar, a1 = ai;
    rot_site(ar, ai, br, bi, s, d);
    rot_site(br, bi, a0, a1, s, d);
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
// exp(-i phi) = hi + lo to ~48 bits; the lo product is formed first so the
// table contributes no coherent per-site error step after step.
__device__ __forceinline__ void apply_phase(float& re, float& im, const float4 p) {
    float tr = mad(re, p.z, -(im * p.w));
    float ti = mad(re, p.w, im * p.z);
    float nr = mad(re, p.x, mad(-im, p.y, tr));
    float ni = mad(re, p.y, mad(im, p.x, ti));
    re = nr;
    im = ni;
}

// ------------------------------------------------------------------ dtype traits

struct C128 {
    using R = double;
    using PT = double2;
};
struct C64 {
    using R = float;
    using PT = float4;
};

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
template <int SPL>
__device__ __forceinline__ void store_pair(void* base, long long off, const Row<double, SPL>& row, int p) {
    double2* q = reinterpret_cast<double2*>(base) + off;
    q[0] = make_double2(row.re[2 * p], row.im[2 * p]);
    q[1] = make_double2(row.re[2 * p + 1], row.im[2 * p + 1]);
}
template <int SPL>
__device__ __forceinline__ void store_pair(void* base, long long off, const Row<float, SPL>& row, int p) {
    *reinterpret_cast<float4*>(reinterpret_cast<float2*>(base) + off) =
        make_float4(row.re[2 * p], row.im[2 * p], row.re[2 * p + 1], row.im[2 * p + 1]);
}

// ------------------------------------------------------------------ row operators

// Even x-pairs: inside the lane.
template <class R, int SPL>
__device__ __forceinline__ void even_x(Row<R, SPL>& w, R s, R d) {
#pragma unroll
    for (int p = 0; p < SPL / 2; ++p) rot_pair(w.re[2 * p], w.im[2 * p], w.re[2 * p + 1], w.im[2 * p + 1], s, d);
}

// Odd x-pairs: inner ones inside the lane, the two at the lane edges across lanes.
template <class R, int SPL>
__device__ __forceinline__ void odd_x(Row<R, SPL>& w, R s, R d) {
    R rr = from_right(w.re[0]), ri = from_right(w.im[0]);
    R lr = from_left(w.re[SPL - 1]), li = from_left(w.im[SPL - 1]);
#pragma unroll
    for (int p = 0; p + 1 < SPL / 2; ++p)
        rot_pair(w.re[2 * p + 1], w.im[2 * p + 1], w.re[2 * p + 2], w.im[2 * p + 2], s, d);
    rot_site(w.re[SPL - 1], w.im[SPL - 1], rr, ri, s, d);
    rot_site(w.re[0], w.im[0], lr, li, s, d);
}

// y-pair made of row `u` (upper, smaller y) and row `v` (next row).
template <class R, int SPL>
__device__ __forceinline__ void pair_y(Row<R, SPL>& u, Row<R, SPL>& v, R s, R d) {
#pragma unroll
    for (int i = 0; i < SPL; ++i) rot_pair(u.re[i], u.im[i], v.re[i], v.im[i], s, d);
}

template <class PT, class R, int SPL>
__device__ __forceinline__ void phase_row(Row<R, SPL>& w, const PT* p) {
#pragma unroll
    for (int i = 0; i < SPL; ++i) apply_phase(w.re[i], w.im[i], p[i]);
}

template <class PT, int SPL>
struct PhasePair {
    PT top[SPL], bot[SPL];
};

template <class R>
struct MarchArgs {
    const void* src;
    void* dst;
    const void* ptab;
    int nx, ny, strip_sites, seg_rows, nstrips, nsegs;
    R o1xs, o1xd, o1ys, o1yd;  // odd factors opening the pass: tau = dt/2 (first pass) or dt
    R o2xs, o2xd, o2ys, o2yd;  // odd factors between steps, tau = dt
    R ehxs, ehxd, ehys, ehyd;  // even factors and the closing odd factors, tau = dt/2
};

__device__ __forceinline__ int wrap(long long v, int n) {
    long long m = v % n;
    return (int)(m < 0 ? m + n : m);
}

// One iteration of the S-stage pipeline.  On entry (it, ib) is the row pair t
// just loaded; stage k completes pair t-1-k: the odd factors on its boundary
// with pair t-k (whose top row arrives as `it`), then, for k < S, the even
// factors and the phase on the pair itself (phase rows from `phase(k)`).
// Stage K-1 = S of the last pass applies only the closing odd factors.  On
// exit (it, ib) is pair t-K, finished.
template <int S, int K, class R, int SPL, class PT, class PhaseFn>
__device__ __forceinline__ void pipeline_step(Row<R, SPL> (&ht)[K], Row<R, SPL> (&hb)[K],
                                              Row<R, SPL>& it, Row<R, SPL>& ib,
                                              const MarchArgs<R>& a, PhaseFn&& phase) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        R oxs, oxd, oys, oyd;
        if (k == 0) {
            oxs = a.o1xs; oxd = a.o1xd; oys = a.o1ys; oyd = a.o1yd;
        } else if (k < S) {
            oxs = a.o2xs; oxd = a.o2xd; oys = a.o2ys; oyd = a.o2yd;
        } else {
            oxs = a.ehxs; oxd = a.ehxd; oys = a.ehys; oyd = a.ehyd;
        }
        odd_x(hb[k], oxs, oxd);
        odd_x(it, oxs, oxd);
        pair_y(hb[k], it, oys, oyd);
        if (k < S) {
            const PhasePair<PT, SPL> ph = phase(k);
            even_x(ht[k], a.ehxs, a.ehxd);
            even_x(hb[k], a.ehxs, a.ehxd);
            pair_y(ht[k], hb[k], a.ehys, a.ehyd);
            phase_row(ht[k], ph.top);
            phase_row(hb[k], ph.bot);
            pair_y(ht[k], hb[k], a.ehys, a.ehyd);
            even_x(ht[k], a.ehxs, a.ehxd);
            even_x(hb[k], a.ehxs, a.ehxd);
        }
        Row<R, SPL> ot = ht[k], ob = hb[k];
        ht[k] = it;
        hb[k] = ib;
        it = ot;
        ib = ob;
    }
}

// Phase factors of the S row pairs inside the pipeline, plus the pair entering
// it, are held either in a register ring (LDS = false; the march loop is
// unrolled by the ring length so slot indices are static) or in a per-lane
// LDS ring (LDS = true; dynamic slots, no unrolling, for deep pipelines).
template <class T, int S, bool LAST, int PPL, bool LDS>
__global__ void __launch_bounds__(kWaveSize * kWavesPerBlock)
march_kernel(const MarchArgs<typename T::R> a) {
    using R = typename T::R;
    using PT = typename T::PT;
    constexpr int SPL = 2 * PPL;
    constexpr int K = S + (LAST ? 1 : 0);
    constexpr int HL = (K + PPL - 1) / PPL;
    constexpr int NL = LDS ? S + 1 : 1;  // LDS ring slots (1 = unused)
    __shared__ PT lring[LDS ? kWavesPerBlock : 1][NL][2][SPL][kWaveSize];

    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = threadIdx.x / kWaveSize;
    // XCD-aware block order: blocks are dealt round-robin to the 8 XCDs, so
    // block b runs on XCD b % 8; give each XCD a contiguous run of tiles so
    // the halo rows shared by neighbouring segments meet in one L2.
    const int nb = gridDim.x;
    const int full = nb & ~7;
    const int b = blockIdx.x;
    const int lb = (b < full) ? ((b & 7) * (full >> 3) + (b >> 3)) : b;
    const long long tile = (long long)lb * kWavesPerBlock + wave;
    if (tile >= (long long)a.nstrips * a.nsegs) return;  // uniform per wavefront
    const int strip = (int)(tile / a.nsegs);
    const int seg = (int)(tile - (long long)strip * a.nsegs);
    const int nx = a.nx, ny = a.ny;

    // x: unwrapped column of the lane's first site, wrapped column of each pair.
    const long long xu0 = (long long)strip * a.strip_sites + (long long)(lane - HL) * SPL;
    const bool inner = lane >= HL && lane < kWaveSize - HL;
    int col[PPL];
    bool keep[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        col[p] = wrap(xu0 + 2 * p, nx);
        keep[p] = inner && (xu0 + 2 * p) < nx;
    }

    // y: output row pairs [q0, q1); input pairs [q0 - K, q1 - 1 + K].
    const int hp = ny >> 1;
    const int q0 = seg * (a.seg_rows >> 1);
    const int q1 = min(q0 + (a.seg_rows >> 1), hp);
    const int tfirst = q0 - K;
    const int tlast = q1 - 1 + K;

    Row<R, SPL> ht[K], hb[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
            ht[k].re[i] = ht[k].im[i] = R(0);
            hb[k].re[i] = hb[k].im[i] = R(0);
        }
    }

    auto load_psi = [&](int t, Row<R, SPL>& top, Row<R, SPL>& bot) {
        const int r0 = wrap(2LL * t, ny);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            load_pair(a.src, (long long)r0 * nx + col[p], top, p);
            load_pair(a.src, (long long)(r0 + 1) * nx + col[p], bot, p);
        }
    };
    auto load_phase = [&](int t) {
        const int r0 = wrap(2LL * t, ny);
        const PT* P0 = reinterpret_cast<const PT*>(a.ptab) + (long long)r0 * nx;
        const PT* P1 = P0 + nx;
        PhasePair<PT, SPL> ph;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            ph.top[2 * p] = P0[col[p]];
            ph.top[2 * p + 1] = P0[col[p] + 1];
            ph.bot[2 * p] = P1[col[p]];
            ph.bot[2 * p + 1] = P1[col[p] + 1];
        }
        return ph;
    };
    auto store_out = [&](int qo, const Row<R, SPL>& top, const Row<R, SPL>& bot) {
        if (qo < q0) return;
        const long long r0 = 2LL * qo;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            if (keep[p]) {
                store_pair(a.dst, r0 * nx + col[p], top, p);
                store_pair(a.dst, (r0 + 1) * nx + col[p], bot, p);
            }
        }
    };

    Row<R, SPL> nt, nbm;  // psi of the next pair (prefetched one iteration ahead)
    load_psi(tfirst, nt, nbm);

    if constexpr (!LDS) {
        constexpr int NP = S + 2;
        PhasePair<PT, SPL> pr[NP];
        pr[0] = load_phase(tfirst);
        for (int tb = tfirst; tb <= tlast; tb += NP) {
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const int t = tb + u;
                if (t > tlast) break;  // uniform per wavefront
                Row<R, SPL> it = nt, ib = nbm;
                if (t < tlast) {
                    load_psi(t + 1, nt, nbm);
                    pr[(u + 1) % NP] = load_phase(t + 1);
                }
                pipeline_step<S, K, R, SPL, PT>(ht, hb, it, ib, a,
                                                [&](int k) { return pr[(u - 1 - k + 2 * NP) % NP]; });
                store_out(t - K, it, ib);
            }
        }
    } else {
        PhasePair<PT, SPL> pn = load_phase(tfirst);  // next pair's phase, in flight
        PT* ring = &lring[LDS ? wave : 0][0][0][0][lane];
        constexpr int SLOT = 2 * SPL * kWaveSize;  // PT elements per slot
        int wslot = 0;                             // slot of pair t
        for (int t = tfirst; t <= tlast; ++t) {
            Row<R, SPL> it = nt, ib = nbm;
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                ring[wslot * SLOT + i * kWaveSize] = pn.top[i];
                ring[wslot * SLOT + (SPL + i) * kWaveSize] = pn.bot[i];
            }
            if (t < tlast) {
                load_psi(t + 1, nt, nbm);
                pn = load_phase(t + 1);
            }
            pipeline_step<S, K, R, SPL, PT>(ht, hb, it, ib, a, [&](int k) {
                int slot = wslot - 1 - k;
                if (slot < 0) slot += NL;
                PhasePair<PT, SPL> ph;
#pragma unroll
                for (int i = 0; i < SPL; ++i) {
                    ph.top[i] = ring[slot * SLOT + i * kWaveSize];
                    ph.bot[i] = ring[slot * SLOT + (SPL + i) * kWaveSize];
                }
                return ph;
            });
            store_out(t - K, it, ib);
            wslot = (wslot + 1 == NL) ? 0 : wslot + 1;
        }
    }
}

// ------------------------------------------------------------------ phase table (row a0)

__global__ void phase_table_c128(const double* __restrict__ V, double2* __restrict__ P,
                                 long long n, double dt, double eps0, double hbar) {
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (long long)gridDim.x * blockDim.x) {
        double phi = dt * (V[l] + eps0) / hbar;
        double s, c;
        sincos(phi, &s, &c);
        P[l] = make_double2(c, -s);
    }
}

__global__ void phase_table_c64(const double* __restrict__ V, float4* __restrict__ P,
                                long long n, double dt, double eps0, double hbar) {
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (long long)gridDim.x * blockDim.x) {
        double phi = dt * (V[l] + eps0) / hbar;
        double s, c;
        sincos(phi, &s, &c);
        float hr = (float)c, hi = (float)(-s);
        float lr = (float)(c - (double)hr), li = (float)(-s - (double)hi);
        P[l] = make_float4(hr, hi, lr, li);
    }
}

// ------------------------------------------------------------------ observables (row a7)

__device__ __forceinline__ void load_site(const void* psi, long long l, double& re, double& im, C128) {
    double2 v = reinterpret_cast<const double2*>(psi)[l];
    re = v.x;
    im = v.y;
}
__device__ __forceinline__ void load_site(const void* psi, long long l, double& re, double& im, C64) {
    float2 v = reinterpret_cast<const float2*>(psi)[l];
    re = (double)v.x;
    im = (double)v.y;
}

template <class T>
__global__ void __launch_bounds__(kReduceThreads)
observables_partial(const void* __restrict__ psi, const double* __restrict__ V, int nx, int ny,
                    double Jx, double Jy, double eps0, double* __restrict__ partial) {
    __shared__ double sn[kReduceThreads], se[kReduceThreads];
    double an = 0.0, ae = 0.0;
    for (int y = blockIdx.x; y < ny; y += gridDim.x) {
        const int yp = (y + 1 == ny) ? 0 : y + 1;
        const int ym = (y == 0) ? ny - 1 : y - 1;
        const long long row = (long long)y * nx;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const int xp = (x + 1 == nx) ? 0 : x + 1;
            const int xm = (x == 0) ? nx - 1 : x - 1;
            double r, i, r1, i1, r2, i2, r3, i3, r4, i4;
            load_site(psi, row + x, r, i, T());
            load_site(psi, row + xp, r1, i1, T());
            load_site(psi, row + xm, r2, i2, T());
            load_site(psi, (long long)yp * nx + x, r3, i3, T());
            load_site(psi, (long long)ym * nx + x, r4, i4, T());
            const double diag = V[row + x] + eps0;
            const double hr = diag * r - Jx * (r1 + r2) - Jy * (r3 + r4);
            const double hi = diag * i - Jx * (i1 + i2) - Jy * (i3 + i4);
            an += r * r + i * i;
            ae += r * hr + i * hi;
        }
    }
    sn[threadIdx.x] = an;
    se[threadIdx.x] = ae;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sn[threadIdx.x] += sn[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sn[0];
        partial[2 * blockIdx.x + 1] = se[0];
    }
}

__global__ void __launch_bounds__(kReduceThreads)
observables_final(const double* __restrict__ partial, int nblocks, double* __restrict__ result) {
    __shared__ double sn[kReduceThreads], se[kReduceThreads];
    double an = 0.0, ae = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        an += partial[2 * b];
        ae += partial[2 * b + 1];
    }
    sn[threadIdx.x] = an;
    se[threadIdx.x] = ae;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sn[threadIdx.x] += sn[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        result[0] = sn[0];
        result[1] = sn[0] > 0.0 ? se[0] / sn[0] : 0.0;
    }
}

// ------------------------------------------------------------------ launch dispatch

template <class R>
MarchArgs<R> make_args(const PassDesc& d, const MarchGeometry& g) {
    MarchArgs<R> a;
    a.src = d.src;
    a.dst = d.dst;
    a.ptab = d.ptab;
    a.nx = d.nx;
    a.ny = d.ny;
    a.strip_sites = g.strip_sites;
    a.seg_rows = d.seg_rows;
    a.nstrips = g.nstrips;
    a.nsegs = g.nsegs;
    const Coef64& ox1 = d.first ? d.oxh : d.ox2;
    const Coef64& oy1 = d.first ? d.oyh : d.oy2;
    a.o1xs = (R)ox1.s; a.o1xd = (R)ox1.d; a.o1ys = (R)oy1.s; a.o1yd = (R)oy1.d;
    a.o2xs = (R)d.ox2.s; a.o2xd = (R)d.ox2.d; a.o2ys = (R)d.oy2.s; a.o2yd = (R)d.oy2.d;
    a.ehxs = (R)d.oxh.s; a.ehxd = (R)d.oxh.d; a.ehys = (R)d.oyh.s; a.ehyd = (R)d.oyh.d;
    return a;
}

template <class T, int S, bool LAST, int PPL, bool LDS>
const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&march_kernel<T, S, LAST, PPL, LDS>);
}

// Instances: register ring for 1..4 steps per pass (1 or 2 pairs per lane),
// LDS ring for 1..kMaxSteps steps per pass (1 pair per lane).
template <class T, bool LAST, int PPL, bool LDS, int... Ss>
const void* pick_steps(int steps, std::integer_sequence<int, Ss...>) {
    const void* f = nullptr;
    ((steps == Ss + 1 ? (f = kernel_ptr<T, Ss + 1, LAST, PPL, LDS>(), 0) : 0), ...);
    return f;
}

template <class T, bool LAST>
const void* pick_variant(int steps, int ppl, bool lds) {
    if (lds) {
        if (ppl != 1) return nullptr;
        return pick_steps<T, LAST, 1, true>(steps, std::make_integer_sequence<int, kMaxSteps>());
    }
    if (ppl == 2)
        return pick_steps<T, LAST, 2, false>(steps, std::make_integer_sequence<int, kMaxRegSteps>());
    return pick_steps<T, LAST, 1, false>(steps, std::make_integer_sequence<int, kMaxRegSteps>());
}

template <class T>
const void* pick_kernel(int steps, bool last, int ppl, bool lds) {
    return last ? pick_variant<T, true>(steps, ppl, lds) : pick_variant<T, false>(steps, ppl, lds);
}

const void* march_kernel_ptr(int dtype, int steps, bool last, int ppl, bool lds) {
    return dtype == 1 ? pick_kernel<C128>(steps, last, ppl, lds)
                      : pick_kernel<C64>(steps, last, ppl, lds);
}

template <class R>
hipError_t launch_with(const void* f, const PassDesc& d, hipStream_t s) {
    const MarchGeometry g = march_geometry(d.nx, d.ny, d.steps, d.last, d.pairs_per_lane, d.seg_rows);
    MarchArgs<R> a = make_args<R>(d, g);
    void* params[] = {&a};
    return hipLaunchKernel(f, dim3(g.blocks), dim3(kWaveSize * kWavesPerBlock), params, 0, s);
}

}  // namespace

MarchGeometry march_geometry(int nx, int ny, int steps, bool last, int pairs_per_lane,
                             int seg_rows) {
    MarchGeometry g;
    const int K = steps + (last ? 1 : 0);
    g.halo_lanes = (K + pairs_per_lane - 1) / pairs_per_lane;
    g.strip_sites = (kWaveSize - 2 * g.halo_lanes) * 2 * pairs_per_lane;
    g.nstrips = (nx + g.strip_sites - 1) / g.strip_sites;
    g.nsegs = (ny + seg_rows - 1) / seg_rows;
    g.tiles = (long long)g.nstrips * g.nsegs;
    g.blocks = (int)((g.tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    return g;
}

hipError_t launch_phase_table(int dtype, const double* V, void* ptab, long long sites,
                              double dt, double eps0, double hbar, hipStream_t s) {
    const int threads = 256;
    long long want = (sites + threads - 1) / threads;
    const int blocks = (int)(want < 8192 ? want : 8192);
    if (dtype == 1)
        hipLaunchKernelGGL(phase_table_c128, dim3(blocks), dim3(threads), 0, s, V,
                           reinterpret_cast<double2*>(ptab), sites, dt, eps0, hbar);
    else
        hipLaunchKernelGGL(phase_table_c64, dim3(blocks), dim3(threads), 0, s, V,
                           reinterpret_cast<float4*>(ptab), sites, dt, eps0, hbar);
    return hipGetLastError();
}

bool march_variant_exists(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds) {
    return march_kernel_ptr(dtype, steps, last, pairs_per_lane, phase_lds) != nullptr;
}

int march_blocks_per_cu(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds) {
    const void* f = march_kernel_ptr(dtype, steps, last, pairs_per_lane, phase_lds);
    if (!f) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kWaveSize * kWavesPerBlock, 0) !=
        hipSuccess)
        return 0;
    return n;
}

hipError_t launch_pass(int dtype, const PassDesc& d, hipStream_t s) {
    const void* f = march_kernel_ptr(dtype, d.steps, d.last, d.pairs_per_lane, d.phase_lds);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = dtype == 1 ? launch_with<double>(f, d, s) : launch_with<float>(f, d, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_observables(int dtype, const void* psi, const double* V, int nx, int ny,
                              double Jx, double Jy, double eps0, double* partial, int nblocks,
                              double* result, hipStream_t s) {
    if (dtype == 1)
        hipLaunchKernelGGL(observables_partial<C128>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, Jx, Jy, eps0, partial);
    else
        hipLaunchKernelGGL(observables_partial<C64>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, Jx, Jy, eps0, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(observables_final, dim3(1), dim3(kReduceThreads), 0, s, partial, nblocks,
                       result);
    return hipGetLastError();
}

}  // namespace tsq
