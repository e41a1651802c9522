// Three-dimensional march: the second-order step on a (nz, ny, nx) mesh, one
// time step per pass.  Sec. 2 splits the 2D mesh Hamiltonian into five parts
// (the diagonal and the even and odd pairs of each axis); this march extends
// that split to three axes, seven parts (Sec. 5 names three dimensions as
// future work).  Per step, first factor first:
//   Ox Oy Oz Ex Ey Ez P Ez Ey Ex Oz Oy Ox   (kinetic factors for dt/2)
// with consecutive steps sharing their odd factors as in the 2D march; a
// closing pass after the last step applies its final Oz Oy Ox.
//
// Tiling: a block of kWaves3 wavefronts owns an x-strip of 64 lanes (two
// x-sites per lane) times a slab of kWaves3 row pairs (wavefront w holds row
// pair w: each lane keeps rows a = 2m and b = 2m+1 of its two x-sites), and it
// marches along z over a segment of plane pairs with the 2D march's pipeline
// (planes in place of rows, F/G named by the direction of travel).  x-pairs
// are exchanged across lanes by DPP shifts; even y-pairs sit in a lane; odd
// y-pairs join row b of wavefront w with row a of wavefront w+1 through LDS,
// one block barrier per exchange; z-pairs sit in a lane.  The lanes and
// wavefronts at the tile edges are halo whose results are discarded (one pair
// per side, like the 2D halo).
#pragma once

#include "tsq_internal3.h"
#include "tsq_march.hpp"

namespace tsq {
namespace {

// A plane pair held by one lane: planes F and G, each with rows a and b of the
// lane's row pair ([0] = a, [1] = b), two x-sites per row.
template <class R>
struct PlanePair {
    Row<R, 2> f[2], g[2];
};

template <class PT>
struct PlanePhase {
    PT f[2][2], g[2][2];  // [row][site]
};

// LDS area of one block for the odd y exchange: [buffer][wavefront][plane]
// [row][component][lane]; components re0, im0, re1, im1 of the two sites.
template <class R>
struct Exchange3 {
    R v[2][kWaves3][2][2][4][kWaveSize];
};

// Wait for this wavefront's LDS writes, then meet the block at the barrier;
// global loads in flight are not waited for.
__device__ __forceinline__ void block_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <class R>
__device__ __forceinline__ void put_row(Exchange3<R>& x, int buf, int w, int plane, int row,
                                        int lane, const Row<R, 2>& r) {
    x.v[buf][w][plane][row][0][lane] = r.re[0];
    x.v[buf][w][plane][row][1][lane] = r.im[0];
    x.v[buf][w][plane][row][2][lane] = r.re[1];
    x.v[buf][w][plane][row][3][lane] = r.im[1];
}

template <class R>
__device__ __forceinline__ Row<R, 2> get_row(const Exchange3<R>& x, int buf, int w, int plane,
                                             int row, int lane) {
    Row<R, 2> r;
    r.re[0] = x.v[buf][w][plane][row][0][lane];
    r.im[0] = x.v[buf][w][plane][row][1][lane];
    r.re[1] = x.v[buf][w][plane][row][2][lane];
    r.im[1] = x.v[buf][w][plane][row][3][lane];
    return r;
}

// Odd y-pairs of two planes p and q: row b of wavefront w with row a of
// wavefront w+1.  Every wavefront publishes its rows, the block meets once,
// and each wavefront rotates its own rows with its neighbours' published
// (pre-factor) values; the wavefronts at the slab edges have no partner in the
// block (halo) and rotate with zeros.  Buffers alternate, so one barrier per
// exchange suffices: a buffer is written again only after every wavefront has
// passed the barrier of the exchange in between, hence finished reading it.
template <class R>
__device__ __forceinline__ void odd_y3(Row<R, 2> (&p)[2], Row<R, 2> (&q)[2], R s, R d,
                                       Exchange3<R>& x, int& buf, int w, int lane) {
    put_row(x, buf, w, 0, 0, lane, p[0]);
    put_row(x, buf, w, 0, 1, lane, p[1]);
    put_row(x, buf, w, 1, 0, lane, q[0]);
    put_row(x, buf, w, 1, 1, lane, q[1]);
    block_sync_lds();
    Row<R, 2> pb, pa, qb, qa;  // partners of p[1], p[0], q[1], q[0]
#pragma unroll
    for (int i = 0; i < 2; ++i) pb.re[i] = pb.im[i] = pa.re[i] = pa.im[i] = R(0);
    qb = pb;
    qa = pb;
    if (w + 1 < kWaves3) {
        pb = get_row(x, buf, w + 1, 0, 0, lane);
        qb = get_row(x, buf, w + 1, 1, 0, lane);
    }
    if (w > 0) {
        pa = get_row(x, buf, w - 1, 0, 1, lane);
        qa = get_row(x, buf, w - 1, 1, 1, lane);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        rot_site(p[1].re[i], p[1].im[i], pb.re[i], pb.im[i], s, d);
        rot_site(p[0].re[i], p[0].im[i], pa.re[i], pa.im[i], s, d);
        rot_site(q[1].re[i], q[1].im[i], qb.re[i], qb.im[i], s, d);
        rot_site(q[0].re[i], q[0].im[i], qa.re[i], qa.im[i], s, d);
    }
    buf ^= 1;
}

// The single stage of a pass.  o is the older plane pair, n the newer one; the
// odd factors act on the boundary planes (o.g, n.f), then the even factors
// and the phase on o.  A closing pass (CLOSE, after the last step) applies
// only the closing odd factors, for dt/2.
template <bool CLOSE, class R, class PT>
__device__ __forceinline__ void stage3(PlanePair<R>& o, PlanePair<R>& n,
                                       const March3Args<R>& a, const XPairs<1, false>& xm,
                                       const PlanePhase<PT>& ph, Exchange3<R>& x, int& buf,
                                       int w, int lane) {
    const R oxs = CLOSE ? a.ehs[0] : a.o1s[0], oxd = CLOSE ? a.ehd[0] : a.o1d[0];
    const R oys = CLOSE ? a.ehs[1] : a.o1s[1], oyd = CLOSE ? a.ehd[1] : a.o1d[1];
    const R ozs = CLOSE ? a.ehs[2] : a.o1s[2], ozd = CLOSE ? a.ehd[2] : a.o1d[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        odd_x<false>(o.g[r], oxs, oxd, xm);
        odd_x<false>(n.f[r], oxs, oxd, xm);
    }
    odd_y3(o.g, n.f, oys, oyd, x, buf, w, lane);
#pragma unroll
    for (int r = 0; r < 2; ++r) pair_y(o.g[r], n.f[r], ozs, ozd);
    if constexpr (!CLOSE) {
        const R es[3] = {a.ehs[0], a.ehs[1], a.ehs[2]};
        const R ed[3] = {a.ehd[0], a.ehd[1], a.ehd[2]};
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            even_x<false>(o.f[r], es[0], ed[0], xm);
            even_x<false>(o.g[r], es[0], ed[0], xm);
        }
        pair_y(o.f[0], o.f[1], es[1], ed[1]);
        pair_y(o.g[0], o.g[1], es[1], ed[1]);
#pragma unroll
        for (int r = 0; r < 2; ++r) pair_y(o.f[r], o.g[r], es[2], ed[2]);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            phase_row(o.f[r], ph.f[r]);
            phase_row(o.g[r], ph.g[r]);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) pair_y(o.f[r], o.g[r], es[2], ed[2]);
        pair_y(o.f[0], o.f[1], es[1], ed[1]);
        pair_y(o.g[0], o.g[1], es[1], ed[1]);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            even_x<false>(o.f[r], es[0], ed[0], xm);
            even_x<false>(o.g[r], es[0], ed[0], xm);
        }
    }
}

// One run of plane pairs [q0, q1) of one column (strip, slab) of one pass;
// wavefront w of the block.
// Register homes as in the 2D march: the plane pair entering in iteration j
// stays in home j mod 3 until stored one iteration later.  The phase of the
// pair stage 0 completes is loaded one iteration ahead into one register
// home, right after the stage has used the previous one: the phase of pair j
// is loaded in iteration j and used in iteration j+1.
template <class T, bool CLOSE>
__device__ __forceinline__ void march3_tile(const March3Args<typename T::R>& a, int strip,
                                            int slab, int q0, int q1, bool rev, int w, int lane,
                                            Exchange3<typename T::R>& x, int& buf) {
    using R = typename T::R;
    using PT = typename T::PT;
    constexpr int K = 1;           // one stage: one step, or the closing odd factors
    constexpr int HL = K;          // halo lanes (x) and halo wavefronts (y) per side
    constexpr int NH = K + 2;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long plane = (long long)nx * ny;

    // x: the lane's x-pair (wrapped) and whether it is stored
    const long long xu = (long long)strip * a.strip_sites + (long long)(lane - HL) * 2;
    const int col = wrap(xu, nx);
    const bool x_keep = lane >= HL && lane < kWaveSize - HL && xu < nx;
    // y: the wavefront's row pair (wrapped) and whether it is stored
    const long long yu = (long long)slab * a.slab_pairs + (w - HL);  // unwrapped row pair
    const int ya = wrap(2 * yu, ny);
    const bool y_keep = w >= HL && w < kWaves3 - HL && 2 * yu < ny;
    const bool keep = x_keep && y_keep;
    const long long rowa = (long long)ya * nx + col, rowb = (long long)(ya + 1) * nx + col;
    const XPairs<1, false> xm{};

    // z: output plane pairs [q0, q1), input [q0 - K, q1 - 1 + K], marched up
    // (rev) or down; rz* are the first planes of the next pairs to load.
    const int nit = (q1 - q0) + 2 * K;
    const int tstart = rev ? q1 - 1 + K : q0 - K;
    const int fo = rev ? 1 : 0;
    const int zstep = rev ? -2 : 2;
    int rz = wrap(2LL * tstart, nz);
    int rzp = rz;  // phase
    int qout = rev ? q1 - 1 + 2 * K : q0 - 2 * K;

    auto step_z = [&](int& z) {
        z += zstep;
        z = z < 0 ? z + nz : z;
        z = z >= nz ? z - nz : z;
    };
    auto load_plane = [&](int z, Row<R, 2> (&rows)[2]) {
        load_pair(a.src, z * plane + rowa, rows[0], 0);
        load_pair(a.src, z * plane + rowb, rows[1], 0);
    };
    auto load_psi = [&](PlanePair<R>& h) {
        load_plane(rz + fo, h.f);
        load_plane(rz + 1 - fo, h.g);
        step_z(rz);
    };
    auto load_phase_plane = [&](int z, PT (&v)[2][2]) {
        const typename T::TT* P = reinterpret_cast<const typename T::TT*>(a.ptab);
        v[0][0] = decode_phase(P[z * plane + rowa]);
        v[0][1] = decode_phase(P[z * plane + rowa + 1]);
        v[1][0] = decode_phase(P[z * plane + rowb]);
        v[1][1] = decode_phase(P[z * plane + rowb + 1]);
    };
    auto load_phase = [&](PlanePhase<PT>& ph) {
        load_phase_plane(rzp + fo, ph.f);
        load_phase_plane(rzp + 1 - fo, ph.g);
        step_z(rzp);
    };
    auto store_out = [&](const PlanePair<R>& h) {
        const int qo = qout;
        qout += rev ? -1 : 1;
        if (rev ? (qo >= q1) : (qo < q0)) return;  // warming up (wavefront-uniform)
        if (!keep) return;
        const long long zf = 2LL * qo + fo, zg = 2LL * qo + 1 - fo;
        store_pair(a.dst, zf * plane + rowa, h.f[0], 0);
        store_pair(a.dst, zf * plane + rowb, h.f[1], 0);
        store_pair(a.dst, zg * plane + rowa, h.g[0], 0);
        store_pair(a.dst, zg * plane + rowb, h.g[1], 0);
    };

    PlanePair<R> home[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                home[h].f[r].re[i] = home[h].f[r].im[i] = R(0);
                home[h].g[r].re[i] = home[h].g[r].im[i] = R(0);
            }
    PlanePhase<PT> ph;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int i = 0; i < 2; ++i) ph.f[r][i] = ph.g[r][i] = zero_phase<PT>();

    int q = rev ? tstart + 1 : tstart - 1;     // pair stage 0 completes this iteration
    const int qend = rev ? q - nit : q + nit;  // one past the last iteration
    load_psi(home[0]);
    auto iteration = [&](auto U) {
        constexpr int u = decltype(U)::value;
        load_psi(home[(u + 1) % NH]);  // the last iteration loads one pair more than it uses
        stage3<CLOSE>(home[(u - 1 + NH) % NH], home[u % NH], a, xm, ph, x, buf, w, lane);
        if constexpr (!CLOSE) load_phase(ph);  // the phase of the pair completed next
        store_out(home[(u - K + 2 * NH) % NH]);
        q += rev ? -1 : 1;
        return q != qend;
    };
    // no phase before the loop: iteration 0 completes a pair of the zero
    // warm-up (before the march start) and then loads the phase of pair 0
    while (static_all<NH>(iteration)) {
    }
}

template <class T, bool CLOSE>
__global__ void __launch_bounds__(kWaveSize * kWaves3)
march3_kernel(const March3Args<typename T::R> a) {
    __shared__ Exchange3<typename T::R> xch;
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    // XCD-aware block order, as in the 2D march.  Tiles are dealt segment
    // fastest; the same segment of neighbouring columns marches the same
    // planes at the same time, so the halo rows two slabs share meet in L2.
    const int nb = gridDim.x;
    const int full = nb & ~7;
    const int b = blockIdx.x;
    const int lb = (b < full) ? ((b & 7) * (full >> 3) + (b >> 3)) : b;
    const long long ntiles = (long long)a.nstrips * a.nslabs * a.nsegs;
    if (lb >= ntiles) return;  // uniform per block
    const int seg = (int)(lb % a.nsegs);
    const long long rest = lb / a.nsegs;
    const int slab = (int)(rest % a.nslabs);
    const int strip = (int)(rest / a.nslabs);
    const int q0 = seg * a.seg_pairs;
    const int q1 = min(q0 + a.seg_pairs, a.nz >> 1);
    int buf = 0;
    march3_tile<T, CLOSE>(a, strip, slab, q0, q1, seg & 1, w, lane, xch, buf);
}

template <class T>
const void* pick_kernel3(bool close) {
    return close ? reinterpret_cast<const void*>(&march3_kernel<T, true>)
                 : reinterpret_cast<const void*>(&march3_kernel<T, false>);
}

}  // namespace
}  // namespace tsq
