// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tsq {

// Coefficients of one 2x2 block exponential [[c, i s], [i s, c]], held as
// s = sin(al) and d = 1 - c = 2 sin^2(al/2).
struct Coef64 {
    double s, d;
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
    Coef64 oxh, oyh;      // tau = dt/2 along x, y
    Coef64 ox2, oy2;      // tau = dt along x, y
};

constexpr int kMaxSteps = 8;     // deepest fusion (phase ring in LDS)
constexpr int kMaxRegSteps = 4;  // deepest fusion with the phase ring in registers
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

// Resident blocks per compute unit of one march kernel instance (0 if the
// query fails); used to size segments so a pass is one round of resident waves.
int march_blocks_per_cu(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds);
bool march_variant_exists(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds);

// All launchers return hipSuccess or the launch error.
hipError_t launch_phase_table(int dtype, const double* V, void* ptab, long long sites,
                              double dt, double eps0, double hbar, hipStream_t s);
hipError_t launch_pass(int dtype, const PassDesc& d, hipStream_t s);
hipError_t launch_observables(int dtype, const void* psi, const double* V, int nx, int ny,
                              double Jx, double Jy, double eps0, double* partial,
                              int nblocks, double* result, hipStream_t s);

constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

}  // namespace tsq
