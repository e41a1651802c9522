// March kernel instances: complex64, time-dependent potential variant.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c64_td(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C64, Variant::TimeDep>(steps, last, ppl, lds);
}

}  // namespace tsq
