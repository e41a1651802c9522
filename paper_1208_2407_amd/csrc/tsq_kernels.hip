// HIP kernels for gfx950 of the second-order Trotter-Suzuki step
// (Wittek & Cucchietti, Sec. 2): the phase table of the diagonal part H0, the
// FP64 norm and energy of the mesh Hamiltonian, and the launchers of the fused
// step march (the product U2 of Eq. "secondorder") whose templates live in
// tsq_march.hpp.

#include <utility>

#include "tsq_internal.h"

namespace tsq {

// Kernel pointer of one march instance, from the translation unit that holds
// it (march_<dtype>_<variant>.hip); nullptr if no such instance is built.
const void* march_ptr_c128_single(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c64_single(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c128_batch(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c64_batch(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c128_closed(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c64_closed(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c128_td(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c64_td(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c128_closedtd(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c64_closedtd(int steps, bool last, int ppl, bool lds);

namespace {

struct C128 {};
struct C64 {};

enum class Variant { Single, Batch, Closed, TimeDep, ClosedTimeDep };

const void* march_kernel_ptr(int dtype, int steps, bool last, int ppl, bool lds, Variant v) {
    const bool d = dtype == 1;
    switch (v) {
        case Variant::Single:
            return d ? march_ptr_c128_single(steps, last, ppl, lds) : march_ptr_c64_single(steps, last, ppl, lds);
        case Variant::Batch:
            return d ? march_ptr_c128_batch(steps, last, ppl, lds) : march_ptr_c64_batch(steps, last, ppl, lds);
        case Variant::Closed:
            return d ? march_ptr_c128_closed(steps, last, ppl, lds) : march_ptr_c64_closed(steps, last, ppl, lds);
        case Variant::TimeDep:
            return d ? march_ptr_c128_td(steps, last, ppl, lds) : march_ptr_c64_td(steps, last, ppl, lds);
        case Variant::ClosedTimeDep:
            return d ? march_ptr_c128_closedtd(steps, last, ppl, lds)
                     : march_ptr_c64_closedtd(steps, last, ppl, lds);
    }
    return nullptr;
}

Variant variant_of(bool batch, bool closed, bool td) {
    if (batch) return Variant::Batch;
    if (td) return closed ? Variant::ClosedTimeDep : Variant::TimeDep;
    return closed ? Variant::Closed : Variant::Single;
}

// ------------------------------------------------------------------ phase table of H0 (Sec. 2)

// `g` scales every entry (the product of a step's cosines on periodic meshes,
// else 1).
__global__ void phase_table_c128(const double* __restrict__ V, double2* __restrict__ P,
                                 long long n, double dt, double eps0, double hbar, double g) {
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (long long)gridDim.x * blockDim.x) {
        double phi = dt * (V[l] + eps0) / hbar;
        double s, c;
        sincos(phi, &s, &c);
        P[l] = make_double2(g * c, -(g * s));
    }
}

// complex64: cos(phi) and -sin(phi) as 32-bit fixed point, value * 2^30
// rounded to nearest (|value| <= 1, so 2^30 fits; error <= 2^-31 per part).
__global__ void phase_table_c64(const double* __restrict__ V, int2* __restrict__ P,
                                long long n, double dt, double eps0, double hbar, double g) {
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (long long)gridDim.x * blockDim.x) {
        double phi = dt * (V[l] + eps0) / hbar;
        double s, c;
        sincos(phi, &s, &c);
        P[l] = make_int2(__double2int_rn(g * c * 0x1p30), __double2int_rn(-(g * s) * 0x1p30));
    }
}

// Time-dependent potential V0 + f(t) W: per site theta0 = dt (V0 + eps0) / hbar
// and w = dt W / hbar; step n's phase is exp(-i (theta0 + f_n w)), formed in
// the march.
__global__ void td_table(const double* __restrict__ V0, const double* __restrict__ W,
                         double2* __restrict__ T, long long n, double dt, double eps0, double hbar) {
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < n;
         l += (long long)gridDim.x * blockDim.x)
        T[l] = make_double2(dt * (V0[l] + eps0) / hbar, dt * W[l] / hbar);
}

// ------------------------------------------------------------------ norm and energy (Sec. 2)

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

// Block b sums |psi|^2 and Re(conj(psi) (H psi)) over its share of the mesh:
// work items (column chunk of kReduceThreads columns, band of `band` rows),
// items b, b + gridDim.x, ...; each thread walks its column down the band with
// the rows above and below the current one in registers, so every psi and V
// value is read once from device memory (the x-neighbours come from the cache
// lines the wavefront has just read).  Fixed item order and a fixed in-block
// tree: the result is bitwise reproducible.
template <class T>
__global__ void __launch_bounds__(kReduceThreads)
observables_partial(const void* __restrict__ psi, const double* __restrict__ V, int nx, int ny,
                    double Jx, double Jy, double eps0, int closed, int band,
                    double* __restrict__ partial) {
    __shared__ double sn[kReduceThreads], se[kReduceThreads];
    double an = 0.0, ae = 0.0;
    const int chunks = (nx + kReduceThreads - 1) / kReduceThreads;
    const int bands = (ny + band - 1) / band;
    const long long items = (long long)chunks * bands;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const int x = (int)(it % chunks) * kReduceThreads + (int)threadIdx.x;
        const int y0 = (int)(it / chunks) * band;
        const int y1 = min(y0 + band, ny);
        if (x >= nx) continue;
        // neighbours wrap on periodic meshes and are absent beyond closed walls
        const bool has_xp = !closed || x + 1 < nx, has_xm = !closed || x > 0;
        const int xp = (x + 1 == nx) ? 0 : x + 1;
        const int xm = (x == 0) ? nx - 1 : x - 1;
        double ur = 0, ui = 0, cr, ci;  // row above, current row
        if (!closed || y0 > 0)
            load_site(psi, (long long)(y0 == 0 ? ny - 1 : y0 - 1) * nx + x, ur, ui, T());
        load_site(psi, (long long)y0 * nx + x, cr, ci, T());
        for (int y = y0; y < y1; ++y) {
            double dr = 0, di = 0;  // row below
            if (!closed || y + 1 < ny)
                load_site(psi, (long long)(y + 1 == ny ? 0 : y + 1) * nx + x, dr, di, T());
            const long long row = (long long)y * nx;
            double r1 = 0, i1 = 0, r2 = 0, i2 = 0;
            if (has_xp) load_site(psi, row + xp, r1, i1, T());
            if (has_xm) load_site(psi, row + xm, r2, i2, T());
            const double diag = V[row + x] + eps0;
            const double hr = diag * cr - Jx * (r1 + r2) - Jy * (dr + ur);
            const double hi = diag * ci - Jx * (i1 + i2) - Jy * (di + ui);
            an += cr * cr + ci * ci;
            ae += cr * hr + ci * hi;
            ur = cr; ui = ci;
            cr = dr; ci = di;
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
hipError_t launch_with(const void* f, const PassDesc& d, hipStream_t s) {
    const MarchGeometry g = march_geometry(d.nx, d.ny, d.steps, d.last, d.pairs_per_lane, d.seg_rows);
    MarchArgs<R> a = make_march_args<R>(d, g);
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
    // one block per segment of kWavesPerBlock neighbouring strips
    g.blocks = (int)((long long)((g.nstrips + kWavesPerBlock - 1) / kWavesPerBlock) * g.nsegs);
    return g;
}

hipError_t launch_phase_table(int dtype, const double* V, void* ptab, long long sites,
                              double dt, double eps0, double hbar, double scale, hipStream_t s) {
    const int threads = 256;
    long long want = (sites + threads - 1) / threads;
    const int blocks = (int)(want < 8192 ? want : 8192);
    if (dtype == 1)
        hipLaunchKernelGGL(phase_table_c128, dim3(blocks), dim3(threads), 0, s, V,
                           reinterpret_cast<double2*>(ptab), sites, dt, eps0, hbar, scale);
    else
        hipLaunchKernelGGL(phase_table_c64, dim3(blocks), dim3(threads), 0, s, V,
                           reinterpret_cast<int2*>(ptab), sites, dt, eps0, hbar, scale);
    return hipGetLastError();
}

hipError_t launch_td_table(const double* V0, const double* W, void* table, long long sites,
                           double dt, double eps0, double hbar, hipStream_t s) {
    const int threads = 256;
    long long want = (sites + threads - 1) / threads;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(td_table, dim3(blocks), dim3(threads), 0, s, V0, W,
                       reinterpret_cast<double2*>(table), sites, dt, eps0, hbar);
    return hipGetLastError();
}

bool march_variant_exists(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                          bool closed, bool td) {
    return march_kernel_ptr(dtype, steps, last, pairs_per_lane, phase_lds,
                            variant_of(false, closed, td)) != nullptr;
}

int march_blocks_per_cu(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                        bool batch, bool closed, bool td) {
    const void* f = march_kernel_ptr(dtype, steps, last, pairs_per_lane, phase_lds,
                                     variant_of(batch, closed, td));
    if (!f) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kWaveSize * kWavesPerBlock, 0) !=
        hipSuccess)
        return 0;
    return n;
}

hipError_t launch_batch(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                        const void* jobs, const BatchTile* tiles, int ntiles, int nwaves,
                        hipStream_t s) {
    const void* f = march_kernel_ptr(dtype, steps, last, pairs_per_lane, phase_lds, Variant::Batch);
    if (!f || ntiles <= 0 || nwaves <= 0) return hipErrorInvalidValue;
    const int blocks = (nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    void* params[] = {&jobs, &tiles, &ntiles};
    hipError_t e = hipLaunchKernel(f, dim3(blocks), dim3(kWaveSize * kWavesPerBlock), params, 0, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_pass(int dtype, const PassDesc& d, hipStream_t s) {
    const void* f = march_kernel_ptr(dtype, d.steps, d.last, d.pairs_per_lane, d.phase_lds,
                                     variant_of(false, d.closed, d.td));
    if (!f) return hipErrorInvalidValue;
    hipError_t e = dtype == 1 ? launch_with<double>(f, d, s) : launch_with<float>(f, d, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_observables_final(const double* partial, int nblocks, double* result,
                                    hipStream_t s) {
    hipLaunchKernelGGL(observables_final, dim3(1), dim3(kReduceThreads), 0, s, partial, nblocks,
                       result);
    return hipGetLastError();
}

hipError_t launch_observables(int dtype, const void* psi, const double* V, int nx, int ny,
                              double Jx, double Jy, double eps0, bool closed, double* partial,
                              int nblocks, double* result, hipStream_t s) {
    const int cl = closed ? 1 : 0;
    // bands of rows sized so the work items fill `nblocks` blocks once
    const long long chunks = (nx + kReduceThreads - 1) / kReduceThreads;
    long long bands = nblocks / chunks;
    if (bands < 1) bands = 1;
    if (bands > ny) bands = ny;
    const int band = (int)((ny + bands - 1) / bands);
    const long long items = chunks * ((ny + band - 1) / band);
    if (items < nblocks) nblocks = (int)items;
    if (dtype == 1)
        hipLaunchKernelGGL(observables_partial<C128>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, Jx, Jy, eps0, cl, band, partial);
    else
        hipLaunchKernelGGL(observables_partial<C64>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, Jx, Jy, eps0, cl, band, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(observables_final, dim3(1), dim3(kReduceThreads), 0, s, partial, nblocks,
                       result);
    return hipGetLastError();
}

}  // namespace tsq
