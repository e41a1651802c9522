// Launchers of the fused step march of gfx950 (the product U2 of
// Eq. "secondorder", Wittek & Cucchietti, Sec. 2) whose templates live in
// tsq_march.hpp: instance lookup, launch geometry, occupancy queries.  The
// phase tables and the norm and energy live in tsq_tables.hip.

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
const void* march_ptr_c128_order4(int steps, bool last, int ppl, bool lds);
const void* march_ptr_c64_order4(int steps, bool last, int ppl, bool lds);

namespace {

enum class Variant { Single, Batch, Closed, TimeDep, ClosedTimeDep, Order4 };

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
        case Variant::Order4:
            return d ? march_ptr_c128_order4(steps, last, ppl, lds) : march_ptr_c64_order4(steps, last, ppl, lds);
    }
    return nullptr;
}

Variant variant_of(bool batch, bool closed, bool td, bool u4 = false) {
    if (u4) return Variant::Order4;
    if (batch) return Variant::Batch;
    if (td) return closed ? Variant::ClosedTimeDep : Variant::TimeDep;
    return closed ? Variant::Closed : Variant::Single;
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

bool march_variant_exists(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                          bool closed, bool td) {
    return march_kernel_ptr(dtype, steps, last, pairs_per_lane, phase_lds,
                            variant_of(false, closed, td)) != nullptr;
}

int march_blocks_per_cu(int dtype, int steps, bool last, int pairs_per_lane, bool phase_lds,
                        bool batch, bool closed, bool td, bool u4) {
    const void* f = march_kernel_ptr(dtype, steps, last, pairs_per_lane, phase_lds,
                                     variant_of(batch, closed, td, u4));
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
                                     variant_of(false, d.closed, d.td, d.u4));
    if (!f) return hipErrorInvalidValue;
    hipError_t e = dtype == 1 ? launch_with<double>(f, d, s) : launch_with<float>(f, d, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace tsq
