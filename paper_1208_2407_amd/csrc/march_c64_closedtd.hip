// March kernel instances: complex64, time-dependent potential between closed walls.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c64_closedtd(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C64, Variant::ClosedTimeDep>(steps, last, ppl, lds);
}

}  // namespace tsq
