// Internal interface of the three-dimensional march (host launch code and
// kernels).
#pragma once

#include "tsq_internal.h"

namespace tsq {

// Kernel arguments of one pass of the three-dimensional march (one step per
// pass): mesh (nz, ny, nx), tiles of an x-strip x a slab of row pairs x a
// segment of plane pairs, and the rotation coefficients per axis.
template <class R>
struct March3Args {
    const void* src;
    void* dst;
    const void* ptab;
    int nx, ny, nz;
    int strip_sites, slab_pairs, seg_pairs;  // stored x-sites, row pairs, plane pairs per tile
    int nstrips, nslabs, nsegs;
    R o1s[3], o1d[3];  // odd factors opening the pass (tau = dt/2 first pass, else dt), x y z
    R ehs[3], ehd[3];  // even factors and the closing odd factors, tau = dt/2, x y z
};

constexpr int kWaves3 = 8;  // wavefronts per block of the 3D march (one row pair each)

struct Pass3Desc {
    const void* src;
    void* dst;
    const void* ptab;
    int nx, ny, nz;
    bool first;           // opening odd factors for dt/2 (else dt)
    bool close;           // a closing pass: only the final odd factors, dt/2
    int seg_pairs;        // plane pairs per tile
    Coef64 oh[3], o2[3];  // tau = dt/2 and tau = dt, per axis
};

hipError_t launch_pass3(int dtype, const Pass3Desc& d, hipStream_t s);
hipError_t launch_observables3(int dtype, const void* psi, const double* V, int nx, int ny, int nz,
                               double Jx, double Jy, double Jz, double eps0, double* partial,
                               int nblocks, double* result, hipStream_t s);

}  // namespace tsq
