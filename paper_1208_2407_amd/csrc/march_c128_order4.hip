// March kernel instances: complex128, fourth order in one pass per step.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c128_order4(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C128, Variant::Order4>(steps, last, ppl, lds);
}

}  // namespace tsq
