// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>

#include <cmath>
#include <stdint.h>

#include "../../include/tsq.h"

namespace tsq {

// Coefficients of one 2x2 block exponential [[c, i s], [i s, c]], held as
// s = sin(al) and d = 1 - c = 2 sin^2(al/2), and its angle al.
struct Coef64 {
    double s, d;
    double al;
};

// Launch description of one fused pass of `steps` time steps over the mesh.
struct PassDesc {
    const void* src;      // psi before the pass
    void* dst;            // psi after the pass (a different buffer)
    const void* ptab;     // phase table
    int nx, ny;
    int steps;            // time steps fused in this pass (1..kMaxSteps)
    bool first;           // the pass starts the evolution: its first odd factor is O(h)
    bool last;            // the pass ends the evolution: it appends the final O(h)
    int seg_rows;         // rows per wavefront segment (even)
    int pairs_per_lane;   // 1 or 2 x-pairs held by each lane
    bool phase_lds;       // phase ring in LDS (else registers)
    bool closed = false;  // hard walls instead of periodic wrap
    bool td = false;      // time-dependent potential: the table holds (theta0, w)
    const double* f = nullptr;  // td: modulation f_n of this pass's steps (host, `steps` values)
    Coef64 oxh, oyh;      // tau = dt/2 along x, y
    Coef64 ox2, oy2;      // tau = dt along x, y
    // fourth order in one pass per step (periodic): sub-steps p, p, m, p, p;
    // the fields above are those of the p sub-step, these of the m sub-step
    bool u4 = false;
    const void* ptab2 = nullptr;  // phase table of the m sub-step; td: the kTurns factors
    Coef64 mxh, myh;              // m sub-step, tau = its dt / 2
    double log_table_p = 0.0, log_table_m = 0.0;  // -2 log of each table's scale
};

constexpr int kMaxSteps = 8;     // deepest fusion (phase ring in LDS)
constexpr int kMaxRegSteps = 6;  // deepest fusion with the phase ring in registers
constexpr int kMaxRegSteps2 = 4; // ... with two x-pairs per lane
constexpr int kMaxTdSteps = 6;   // deepest fusion with a time-dependent potential
constexpr int kTurns = 2048;     // time-dependent phase: factors exp(-i j pi/1024), j mod 2048
constexpr int kWaveSize = 64;
constexpr int kWavesPerBlock = 4;

// Geometry the march kernel uses (shared by host-side launch arithmetic).
struct MarchGeometry {
    int halo_lanes;    // lanes per side whose results are discarded
    int strip_sites;   // x-sites stored per wavefront
    int nstrips, nsegs;
    long long tiles;
    int blocks;
};
MarchGeometry march_geometry(int nx, int ny, int steps, bool last, int pairs_per_lane,
                             int seg_rows);

// Kernel arguments of one pass over one problem (also the job record of the
// batched kernel, uploaded to device memory).  R = double (complex128) or
// float (complex64).
//
// Two forms of the rotations: the delta form a' = a + (i s b - d a) (4
// multiply-adds per site) and the tangent form (a, b) <- (a + i t b,
// b + i t a), t = tan(al), which is sec(al) times the block exponential (2
// multiply-adds per site).
// Closed meshes apply the odd factors in the delta form and the four even
// factors of a step in the tangent form.  Between the first and the last even
// factor of a step the only other operators are even y (even x) factors, which act
// within columns (rows), and the diagonal phase; so the cosines the even
// factors leave out, per site the product over the factors that pair it
// (a site of the last column of an odd-width mesh has no even x partner, one
// of the last row of an odd-height mesh no even y partner), come back exactly
// as a per-site scale of the phase table (time-dependent potentials: the
// shared factors carry the interior's scale and the march multiplies the
// last odd column's and row's factors by kxw, kyw).
// Periodic meshes use the tangent form throughout; every site of a periodic
// mesh meets each of a step's factors, so the dropped cosines multiply every
// site alike and are restored elsewhere:
//   * time-independent potentials: the phase table holds exp(-i phi) times the
//     product g of a whole step's cosines (see phase_scale); stage 0 of a pass
//     applies its odd x factor in the delta form with s' = t, d' = 0 (the
//     tangent form, to the bit) or, in the first pass, with the coefficients of
//     the opening half factor and the ratio of its cosines to those of g; the
//     closing stage's odd x factor carries its own cosines;
//   * time-dependent potentials (the phase formed in the march): every stage's
//     odd x factor carries that stage's cosines.
// Coefficients s' = m sin(al_x), d' = 1 - m cos(al_x) of an odd x factor in
// the delta form with modulus m come from the rounded tangents, so every step
// is unitary up to the rounding of s', d' and the table.  Field use
// (periodic):
//   o1x* (s', d')  stage 0 odd x         o1ys  stage 0 odd y tangent
//   o2xs tangent / (s', d') (td)         o2ys  odd y tangent
//   c1x* (s', d')  closing odd x         c1ys  closing odd y tangent
//   ehxs, ehys     even tangents
// Per-stage coefficients of the fourth-order pass (stages 0..4, closing 5):
// odd x (s', d') and odd y tangent per stage; even tangents per sub-step kind
// (0 = p, 1 = m).
template <class R>
struct Order4Coefs {
    R xs[6], xd[6], yt[6];
    R ext[2], eyt[2];
};

template <class R>
struct MarchArgs {
    const void* src;
    void* dst;
    const void* ptab;
    const void* ptab2;  // fourth order: the m sub-step's table; time-dependent: the kTurns factors
    int nx, ny, strip_sites, seg_rows, nstrips, nsegs;
    R o1xs, o1xd, o1ys, o1yd;  // odd factors opening the pass: tau = dt/2 (first pass) or dt
    R o2xs, o2xd, o2ys, o2yd;  // odd factors between steps, tau = dt
    R ehxs, ehxd, ehys, ehyd;  // even factors, tau = dt/2
    R c1xs, c1xd, c1ys, c1yd;  // odd factors closing the evolution, tau = dt/2
    double g[kMaxSteps];       // time-dependent potential: f_n of step k of the pass
    double kxw, kyw;           // closed, time-dependent: scale of the last odd column, row
    Order4Coefs<R> u4;         // fourth order in one pass per step
};

// Tangent-form coefficients (periodic meshes), rounded to R.
template <class R>
R tangent(const Coef64& c) {
    return (R)std::tan(c.al);
}
// log(1 + t^2): log of the squared modulus a tangent factor multiplies by
template <class R>
double log_sec2(R t) {
    return std::log1p((double)t * (double)t);
}
// Odd x factor in the delta form, angle al, squared modulus exp(-L):
// s' = m sin(al), 1 - d' = sqrt(m^2 - s'^2) with s' rounded first.
template <class R>
void delta_odd_x(double al, double L, R& xs, R& xd) {
    const double m2 = std::exp(-L);
    xs = (R)(std::sqrt(m2) * std::sin(al));
    const double s2 = (double)xs * (double)xs;
    const double one_minus_x = -std::expm1(-L) + s2;  // 1 - (m^2 - s'^2)
    xd = (R)(one_minus_x / (1.0 + std::sqrt(m2 - s2)));
}
// Log of the squared modulus a steady step's tangent factors multiply every
// site by (odd x and y at tau = dt, two even x and two even y at dt/2); the
// phase table of a periodic mesh holds exp(-i phi) * exp(-L/2).  A closed
// mesh's table holds exp(-i phi) times the cosines of the even factors that
// pair the site (log_sec2 of the even tangents).
template <class R>
double step_log_sec2(const Coef64& oxh, const Coef64& oyh, const Coef64& ox2,
                     const Coef64& oy2) {
    return log_sec2(tangent<R>(ox2)) + log_sec2(tangent<R>(oy2)) +
           2.0 * log_sec2(tangent<R>(oxh)) + 2.0 * log_sec2(tangent<R>(oyh));
}

template <class R>
MarchArgs<R> make_march_args(const PassDesc& d, const MarchGeometry& g) {
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
    if (d.closed) {
        a.o1xs = (R)ox1.s; a.o1xd = (R)ox1.d; a.o1ys = (R)oy1.s; a.o1yd = (R)oy1.d;
        a.o2xs = (R)d.ox2.s; a.o2xd = (R)d.ox2.d; a.o2ys = (R)d.oy2.s; a.o2yd = (R)d.oy2.d;
        a.c1xs = (R)d.oxh.s; a.c1xd = (R)d.oxh.d; a.c1ys = (R)d.oyh.s; a.c1yd = (R)d.oyh.d;
        a.ehxs = tangent<R>(d.oxh);
        a.ehys = tangent<R>(d.oyh);
        a.ehxd = a.ehyd = R(0);
        // the last column (row) of an odd width (height) has no even x (y)
        // partner: 1 / cos^2 of that factor over the interior's scale
        a.kxw = std::exp(log_sec2(a.ehxs));
        a.kyw = std::exp(log_sec2(a.ehys));
    } else {
        a.kxw = a.kyw = 1.0;
        const R tex = tangent<R>(d.oxh), tey = tangent<R>(d.oyh);
        const double Le = 2.0 * log_sec2(tex) + 2.0 * log_sec2(tey);  // four even factors
        a.ehxs = tex;
        a.ehys = tey;
        a.o1ys = tangent<R>(oy1);
        a.o2ys = tangent<R>(d.oy2);
        a.c1ys = tangent<R>(d.oyh);
        a.o1yd = a.o2yd = a.c1yd = a.ehxd = a.ehyd = R(0);
        // closing stage: odd x and y at dt/2, no table
        delta_odd_x<R>(d.oxh.al, log_sec2(a.c1ys), a.c1xs, a.c1xd);
        // the phase factor (table or, time-dependent, the turns) restores a
        // steady step's cosines (L_step); stage 0 of the first pass restores
        // the rest of its own
        a.o2xs = tangent<R>(d.ox2);
        a.o2xd = R(0);
        if (d.first) {
            const double L_step = step_log_sec2<R>(d.oxh, d.oyh, d.ox2, d.oy2);
            delta_odd_x<R>(ox1.al, Le + log_sec2(a.o1ys) - L_step, a.o1xs, a.o1xd);
        } else {
            a.o1xs = a.o2xs;
            a.o1xd = R(0);
        }
    }
    for (int k = 0; k < kMaxSteps; ++k) a.g[k] = (d.td && d.f && k < d.steps) ? d.f[k] : 0.0;
    a.ptab2 = d.ptab2;
    a.u4 = Order4Coefs<R>{};
    if (d.u4) {
        // sub-step kinds p, p, m, p, p; the odd factor ahead of sub-step k
        // merges the half factors of sub-steps k-1 and k (Eq. "fourthorder"
        // as consecutive second-order steps), or opens the evolution
        const Coef64* hx[2] = {&d.oxh, &d.mxh};
        const Coef64* hy[2] = {&d.oyh, &d.myh};
        const int kind[5] = {0, 0, 1, 0, 0};
        const double Ltab[2] = {d.log_table_p, d.log_table_m};
        for (int q = 0; q < 2; ++q) {
            a.u4.ext[q] = tangent<R>(*hx[q]);
            a.u4.eyt[q] = tangent<R>(*hy[q]);
        }
        for (int k = 0; k <= 5; ++k) {
            const int cur = k < 5 ? kind[k] : 0, prev = k > 0 ? kind[k - 1] : 0;
            const bool open = k == 0 && d.first, close = k == 5;
            const double alx = (open ? 0.0 : hx[prev]->al) + (close ? 0.0 : hx[cur]->al);
            const double aly = (open ? 0.0 : hy[prev]->al) + (close ? 0.0 : hy[cur]->al);
            a.u4.yt[k] = (R)std::tan(aly);
            double L = log_sec2(a.u4.yt[k]);
            if (!close)
                L += 2.0 * log_sec2(a.u4.ext[cur]) + 2.0 * log_sec2(a.u4.eyt[cur]) - Ltab[cur];
            delta_odd_x<R>(alx, L, a.u4.xs[k], a.u4.xd[k]);
        }
    }
    return a;
}

// One entry of the batched kernel's work list.
struct BatchTile {
    int job;    // index into the launch's MarchArgs array
    int strip;
    int seg;
    int rows;   // rows the tile marches (host-side sort key)
};

// Resident blocks per compute unit of one march kernel instance (0 if the
// query fails); used to size segments so a pass is one round of resident waves.
int march_blocks_per_cu(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                        bool batch = false, bool closed = false, bool td = false, bool u4 = false);
bool march_variant_exists(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                          bool closed = false, bool td = false);

// All launchers return hipSuccess or the launch error.
// exp(-i dt (V + eps0) / hbar) times `scale` per site.
// Per-site scale of the phase table: g, or on a closed mesh gx on the last
// column (column wx >= 0: an odd width leaves it without an even x partner),
// gy on the last row (from site wy0 >= 0: an odd height), gxy on both.
struct TableScale {
    double g = 1.0, gx = 1.0, gy = 1.0, gxy = 1.0;
    long long nx = 1, wx = -1, wy0 = -1;
};
hipError_t launch_phase_table(int dtype, const double* V, void* ptab, long long sites,
                              double dt, double eps0, double hbar, const TableScale& scale,
                              hipStream_t s);
// Table of the time-dependent potential V0 + f(t) W: per site the phase angle
// theta0 = dt (V0 + eps0) / hbar and its modulation w = dt W / hbar, as a
// double2 (16 B/site, both dtypes); step n's phase is exp(-i (theta0 + f_n w)).
// `turns` receives the kTurns factors scale * exp(-i j pi/1024) (double2) the
// march composes each step's factor from.
hipError_t launch_td_table(const double* V0, const double* W, void* table, void* turns,
                           long long sites, double dt, double eps0, double hbar, double scale,
                           hipStream_t s);
hipError_t launch_pass(int dtype, const PassDesc& d, hipStream_t s);
// Second stage of the FP64 reductions: sum the `nblocks` (norm, energy) partials
// in a fixed order into result[0] = norm, result[1] = energy / norm.
hipError_t launch_observables_final(const double* partial, int nblocks, double* result,
                                    hipStream_t s);
// Batched pass: `nwaves` wavefronts walk `ntiles` tiles of `jobs` (device
// MarchArgs<double> for complex128, MarchArgs<float> for complex64).
hipError_t launch_batch(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                        const void* jobs, const BatchTile* tiles, int ntiles, int nwaves,
                        hipStream_t s);
hipError_t launch_observables(int dtype, const void* psi, const double* V, int nx, int ny,
                              double Jx, double Jy, double eps0, bool closed, double* partial,
                              int nblocks, double* result, hipStream_t s);

constexpr int kReduceBlocks = 8192;  // partial sums of the norm and energy reductions

// Bytes of the library-held device array of tsq_batch_evolve_noalloc (per GPU).
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;

// Record `fmt` as the calling thread's last error and return `code`.
int set_error(int code, const char* fmt, ...);

// Build the batch of tsq_batch_create, copy its work lists to `bws` (at most
// `bws_bytes`) and enqueue every pass on `stream`; `need` (if not null)
// receives the work lists' size in bytes.  Shared by tsq_batch_evolve and its
// workspace-free variant.
int batch_evolve_into(tsq_plan* const* plans, void* const* psi, void* const* ws,
                      const int64_t* steps, int32_t n, const tsq_schedule* schedule, void* bws,
                      size_t bws_bytes, void* stream, size_t* need);
constexpr int kReduceThreads = 256;

}  // namespace tsq
