// March kernel instances: complex128, time-dependent potential between closed walls.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c128_closedtd(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C128, Variant::ClosedTimeDep>(steps, last, ppl, lds);
}

}  // namespace tsq
