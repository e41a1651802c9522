// HIP launch code of the three-dimensional march (the extension to three
// dimensions of Sec. 5) and its FP64 observables.

#include <algorithm>

#include "tsq_internal3.h"

namespace tsq {

const void* march3_ptr_c128(bool close);
const void* march3_ptr_c64(bool close);

namespace {

struct C128 {};
struct C64 {};

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

// Three-dimensional meshes: rows r = z ny + y of the (nz, ny, nx) mesh, six
// neighbours wrapping periodically.
template <class T>
__global__ void __launch_bounds__(kReduceThreads)
observables3_partial(const void* __restrict__ psi, const double* __restrict__ V, int nx, int ny,
                     int nz, double Jx, double Jy, double Jz, double eps0,
                     double* __restrict__ partial) {
    __shared__ double sn[kReduceThreads], se[kReduceThreads];
    double an = 0.0, ae = 0.0;
    const long long plane = (long long)nx * ny;
    for (long long rr = blockIdx.x; rr < (long long)ny * nz; rr += gridDim.x) {
        const int z = (int)(rr / ny), y = (int)(rr - (long long)z * ny);
        const int yp = (y + 1 == ny) ? 0 : y + 1, ym = (y == 0) ? ny - 1 : y - 1;
        const int zp = (z + 1 == nz) ? 0 : z + 1, zm = (z == 0) ? nz - 1 : z - 1;
        const long long row = rr * nx;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const int xp = (x + 1 == nx) ? 0 : x + 1, xm = (x == 0) ? nx - 1 : x - 1;
            double r, i, r1, i1, r2, i2, r3, i3, r4, i4, r5, i5, r6, i6;
            load_site(psi, row + x, r, i, T());
            load_site(psi, row + xp, r1, i1, T());
            load_site(psi, row + xm, r2, i2, T());
            load_site(psi, (long long)z * plane + (long long)yp * nx + x, r3, i3, T());
            load_site(psi, (long long)z * plane + (long long)ym * nx + x, r4, i4, T());
            load_site(psi, (long long)zp * plane + (long long)y * nx + x, r5, i5, T());
            load_site(psi, (long long)zm * plane + (long long)y * nx + x, r6, i6, T());
            const double diag = V[row + x] + eps0;
            const double hr = diag * r - Jx * (r1 + r2) - Jy * (r3 + r4) - Jz * (r5 + r6);
            const double hi = diag * i - Jx * (i1 + i2) - Jy * (i3 + i4) - Jz * (i5 + i6);
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

}  // namespace

hipError_t launch_observables3(int dtype, const void* psi, const double* V, int nx, int ny, int nz,
                               double Jx, double Jy, double Jz, double eps0, double* partial,
                               int nblocks, double* result, hipStream_t s) {
    if (dtype == 1)
        hipLaunchKernelGGL(observables3_partial<C128>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, nz, Jx, Jy, Jz, eps0, partial);
    else
        hipLaunchKernelGGL(observables3_partial<C64>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, nz, Jx, Jy, Jz, eps0, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_observables_final(partial, nblocks, result, s);
}

template <class R>
static hipError_t launch3_with(const void* f, const Pass3Desc& d, hipStream_t s) {
    const int K = 1;
    March3Args<R> a;
    a.src = d.src;
    a.dst = d.dst;
    a.ptab = d.ptab;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.strip_sites = (kWaveSize - 2 * K) * 2;
    a.slab_pairs = kWaves3 - 2 * K;
    a.seg_pairs = d.seg_pairs;
    a.nstrips = (d.nx + a.strip_sites - 1) / a.strip_sites;
    a.nslabs = (d.ny / 2 + a.slab_pairs - 1) / a.slab_pairs;
    a.nsegs = (d.nz / 2 + d.seg_pairs - 1) / d.seg_pairs;
    for (int ax = 0; ax < 3; ++ax) {
        const Coef64& o1 = d.first ? d.oh[ax] : d.o2[ax];
        a.o1s[ax] = (R)o1.s;
        a.o1d[ax] = (R)o1.d;
        a.ehs[ax] = (R)d.oh[ax].s;
        a.ehd[ax] = (R)d.oh[ax].d;
    }
    const long long tiles = (long long)a.nstrips * a.nslabs * a.nsegs;
    if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    void* params[] = {&a};
    return hipLaunchKernel(f, dim3((unsigned)tiles), dim3(kWaveSize * kWaves3), params, 0, s);
}

hipError_t launch_pass3(int dtype, const Pass3Desc& d, hipStream_t s) {
    const void* f = dtype == 1 ? march3_ptr_c128(d.close) : march3_ptr_c64(d.close);
    if (!f || d.seg_pairs < 1) return hipErrorInvalidValue;
    hipError_t e = dtype == 1 ? launch3_with<double>(f, d, s) : launch3_with<float>(f, d, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace tsq
