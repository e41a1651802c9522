// HIP kernels for gfx950 around the step march (Wittek & Cucchietti, Sec. 2):
// the phase table of the diagonal part H0 (and the table of a time-dependent
// potential), and the FP64 norm and energy of the mesh Hamiltonian.

#include "tsq_internal.h"

namespace tsq {
namespace {

struct C128 {};
struct C64 {};

// ------------------------------------------------------------------ phase table of H0 (Sec. 2)

// exp(-i phi_l) times the site's scale (the cosines the march's tangent-form
// factors leave out; see TableScale) for sites l = i, i + n/4... of each
// thread's four-site groups: the four loads of V are issued before the four
// sines and cosines.
__device__ __forceinline__ double site_scale(const TableScale& sc, long long l) {
    if (sc.wx < 0 && sc.wy0 < 0) return sc.g;
    const bool x = sc.wx >= 0 && l % sc.nx == sc.wx;
    const bool y = sc.wy0 >= 0 && l >= sc.wy0;
    return x ? (y ? sc.gxy : sc.gx) : (y ? sc.gy : sc.g);
}
template <class Store>
__device__ __forceinline__ void phase_sites(const double* __restrict__ V, long long n, double dt,
                                            double eps0, double hbar, Store&& store) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; l + 3 * stride < n; l += 4 * stride) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = V[l + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double s, c;
            sincos(dt * (v[k] + eps0) / hbar, &s, &c);
            store(l + k * stride, c, s);
        }
    }
    for (; l < n; l += stride) {
        double s, c;
        sincos(dt * (V[l] + eps0) / hbar, &s, &c);
        store(l, c, s);
    }
}

__global__ void phase_table_c128(const double* __restrict__ V, double2* __restrict__ P,
                                 long long n, double dt, double eps0, double hbar, TableScale sc) {
    phase_sites(V, n, dt, eps0, hbar, [&](long long l, double c, double s) {
        const double g = site_scale(sc, l);
        P[l] = make_double2(g * c, -(g * s));
    });
}

// complex64: cos(phi) and -sin(phi) as 32-bit fixed point, value * 2^30
// rounded to nearest (|value| <= 1, so 2^30 fits; error <= 2^-31 per part).
__global__ void phase_table_c64(const double* __restrict__ V, int2* __restrict__ P,
                                long long n, double dt, double eps0, double hbar, TableScale sc) {
    phase_sites(V, n, dt, eps0, hbar, [&](long long l, double c, double s) {
        const double g = site_scale(sc, l);
        P[l] = make_int2(__double2int_rn(g * c * 0x1p30), __double2int_rn(-(g * s) * 0x1p30));
    });
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

// The march's factors scale * exp(-i j pi/1024), j = 0 .. kTurns-1 (j / 1024
// is exact, so sincospi sees the angle without rounding).
__global__ void td_turns(double2* __restrict__ U, double scale) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kTurns) return;
    double sn, cs;
    sincospi((double)j / 1024.0, &sn, &cs);
    U[j] = make_double2(scale * cs, -(scale * sn));
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
// lines the wavefront has just read).  Rows go four at a time, their loads
// issued together.  Fixed item order, fixed row order per thread and a fixed
// in-block tree: the result is bitwise reproducible.
template <class T>
__device__ __forceinline__ void site_energy(double cr, double ci, double ur, double ui, double dr,
                                            double di, double r1, double i1, double r2, double i2,
                                            double v, double Jx, double Jy, double eps0,
                                            double& an, double& ae) {
    const double diag = v + eps0;
    const double hr = diag * cr - Jx * (r1 + r2) - Jy * (dr + ur);
    const double hi = diag * ci - Jx * (i1 + i2) - Jy * (di + ui);
    an += cr * cr + ci * ci;
    ae += cr * hr + ci * hi;
}

template <class T>
__global__ void __launch_bounds__(kReduceThreads)
observables_partial(const void* __restrict__ psi, const double* __restrict__ V, int nx, int ny,
                    double Jx, double Jy, double eps0, int closed, int band,
                    double* __restrict__ partial) {
    __shared__ double sn[kReduceThreads], se[kReduceThreads];
    constexpr int U = 4;  // rows per step of the walk
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
        auto load_row = [&](int y, double& dr, double& di, double& r1, double& i1, double& r2,
                            double& i2, double& v) {
            // row below y, the x-neighbours on row y, V on row y
            dr = di = r1 = i1 = r2 = i2 = 0.0;
            if (!closed || y + 1 < ny)
                load_site(psi, (long long)(y + 1 == ny ? 0 : y + 1) * nx + x, dr, di, T());
            const long long row = (long long)y * nx;
            if (has_xp) load_site(psi, row + xp, r1, i1, T());
            if (has_xm) load_site(psi, row + xm, r2, i2, T());
            v = V[row + x];
        };
        double ur = 0, ui = 0, cr, ci;  // row above, current row
        if (!closed || y0 > 0)
            load_site(psi, (long long)(y0 == 0 ? ny - 1 : y0 - 1) * nx + x, ur, ui, T());
        load_site(psi, (long long)y0 * nx + x, cr, ci, T());
        int y = y0;
        for (; y + U <= y1; y += U) {
            double dr[U], di[U], r1[U], i1[U], r2[U], i2[U], v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) load_row(y + k, dr[k], di[k], r1[k], i1[k], r2[k], i2[k], v[k]);
#pragma unroll
            for (int k = 0; k < U; ++k) {
                site_energy<T>(cr, ci, ur, ui, dr[k], di[k], r1[k], i1[k], r2[k], i2[k], v[k], Jx,
                               Jy, eps0, an, ae);
                ur = cr; ui = ci;
                cr = dr[k]; ci = di[k];
            }
        }
        for (; y < y1; ++y) {
            double dr, di, r1, i1, r2, i2, v;
            load_row(y, dr, di, r1, i1, r2, i2, v);
            site_energy<T>(cr, ci, ur, ui, dr, di, r1, i1, r2, i2, v, Jx, Jy, eps0, an, ae);
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

// Periodic meshes with an even number of columns: each lane owns two
// neighbouring columns (16-byte loads of psi and V per row, as the march
// issues), and the x-neighbours outside its pair come from the lanes beside
// it by a DPP wavefront shift; only the first and last lanes of a wavefront
// (and the last lane holding columns when the row ends inside the wavefront)
// load theirs.  Work items are (chunk of 2 * kReduceThreads columns, band of
// rows), walked as in observables_partial; fixed order, bitwise reproducible.
__device__ __forceinline__ double lane_from_left(double v) {
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_from_right(double v) {
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// psi of sites l and l+1 (l even): complex128 two 16-byte loads, complex64 one.
__device__ __forceinline__ void load_pair2(const void* psi, long long l, double (&re)[2],
                                           double (&im)[2], C128) {
    const double2* q = reinterpret_cast<const double2*>(psi) + l;
    const double2 a = q[0], b = q[1];
    re[0] = a.x; im[0] = a.y; re[1] = b.x; im[1] = b.y;
}
__device__ __forceinline__ void load_pair2(const void* psi, long long l, double (&re)[2],
                                           double (&im)[2], C64) {
    const float4 a = *reinterpret_cast<const float4*>(reinterpret_cast<const float2*>(psi) + l);
    re[0] = a.x; im[0] = a.y; re[1] = a.z; im[1] = a.w;
}

template <class T>
__global__ void __launch_bounds__(kReduceThreads)
observables_pairs(const void* __restrict__ psi, const double* __restrict__ V, int nx, int ny,
                  double Jx, double Jy, double eps0, int band, double* __restrict__ partial) {
    __shared__ double sn[kReduceThreads], se[kReduceThreads];
    constexpr int U = 4;  // rows per step of the walk
    constexpr int W = 2 * kReduceThreads;  // columns per chunk
    double an = 0.0, ae = 0.0;
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int chunks = (nx + W - 1) / W;
    const int bands = (ny + band - 1) / band;
    const long long items = (long long)chunks * bands;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const int x0 = (int)(it % chunks) * W + 2 * (int)threadIdx.x;
        const int y0 = (int)(it / chunks) * band;
        const int y1 = min(y0 + band, ny);
        // every lane takes part in the shifts; lanes past the row load nothing
        const bool live = x0 < nx;
        const bool edge_l = lane == 0;
        const bool edge_r = lane == kWaveSize - 1 || x0 + 2 >= nx;
        const int xl = x0 == 0 ? nx - 1 : x0 - 1;
        const int xr = x0 + 2 >= nx ? 0 : x0 + 2;
        const int xc = live ? x0 : 0;
        auto load_pairs = [&](int y, double (&re)[2], double (&im)[2]) {
            re[0] = re[1] = im[0] = im[1] = 0.0;
            if (live) load_pair2(psi, (long long)y * nx + xc, re, im, T());
        };
        double ur[2], ui[2], cr[2], ci[2];
        load_pairs(y0 == 0 ? ny - 1 : y0 - 1, ur, ui);
        load_pairs(y0, cr, ci);
        // one row: the row below is loaded by the caller, V and the edge
        // neighbours of row y here
        auto row = [&](int y, const double (&dr)[2], const double (&di)[2], double2 v) {
            double lr = lane_from_left(cr[1]), li = lane_from_left(ci[1]);
            double rr = lane_from_right(cr[0]), ri = lane_from_right(ci[0]);
            if (live && edge_l) load_site(psi, (long long)y * nx + xl, lr, li, T());
            if (live && edge_r) load_site(psi, (long long)y * nx + xr, rr, ri, T());
            if (live) {
                site_energy<T>(cr[0], ci[0], ur[0], ui[0], dr[0], di[0], cr[1], ci[1], lr, li, v.x,
                               Jx, Jy, eps0, an, ae);
                site_energy<T>(cr[1], ci[1], ur[1], ui[1], dr[1], di[1], rr, ri, cr[0], ci[0], v.y,
                               Jx, Jy, eps0, an, ae);
            }
        };
        auto load_v = [&](int y) {
            return live ? *reinterpret_cast<const double2*>(V + (long long)y * nx + xc)
                        : make_double2(0.0, 0.0);
        };
        int y = y0;
        for (; y + U <= y1; y += U) {
            double dr[U][2], di[U][2];
            double2 v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                load_pairs(y + k + 1 == ny ? 0 : y + k + 1, dr[k], di[k]);
                v[k] = load_v(y + k);
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                row(y + k, dr[k], di[k], v[k]);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    ur[i] = cr[i]; ui[i] = ci[i];
                    cr[i] = dr[k][i]; ci[i] = di[k][i];
                }
            }
        }
        for (; y < y1; ++y) {
            double dr[2], di[2];
            load_pairs(y + 1 == ny ? 0 : y + 1, dr, di);
            row(y, dr, di, load_v(y));
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ur[i] = cr[i]; ui[i] = ci[i];
                cr[i] = dr[i]; ci[i] = di[i];
            }
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

}  // namespace

hipError_t launch_phase_table(int dtype, const double* V, void* ptab, long long sites,
                              double dt, double eps0, double hbar, const TableScale& scale,
                              hipStream_t s) {
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

hipError_t launch_td_table(const double* V0, const double* W, void* table, void* turns,
                           long long sites, double dt, double eps0, double hbar, double scale,
                           hipStream_t s) {
    const int threads = 256;
    long long want = (sites + threads - 1) / threads;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(td_table, dim3(blocks), dim3(threads), 0, s, V0, W,
                       reinterpret_cast<double2*>(table), sites, dt, eps0, hbar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(td_turns, dim3((kTurns + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<double2*>(turns), scale);
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
    // periodic meshes (even sides) with 16-byte aligned psi and V take the
    // two-column kernel
    const bool aligned = reinterpret_cast<uintptr_t>(psi) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(V) % 16 == 0;
    const bool pairs = !closed && (nx % 2) == 0 && aligned;
    const int width = pairs ? 2 * kReduceThreads : kReduceThreads;
    // bands of rows sized so the work items fill `nblocks` blocks once
    const long long chunks = (nx + width - 1) / width;
    long long bands = nblocks / chunks;
    if (bands < 1) bands = 1;
    if (bands > ny) bands = ny;
    const int band = (int)((ny + bands - 1) / bands);
    const long long items = chunks * ((ny + band - 1) / band);
    if (items < nblocks) nblocks = (int)items;
    if (pairs && dtype == 1)
        hipLaunchKernelGGL(observables_pairs<C128>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, Jx, Jy, eps0, band, partial);
    else if (pairs)
        hipLaunchKernelGGL(observables_pairs<C64>, dim3(nblocks), dim3(kReduceThreads), 0, s,
                           psi, V, nx, ny, Jx, Jy, eps0, band, partial);
    else if (dtype == 1)
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
