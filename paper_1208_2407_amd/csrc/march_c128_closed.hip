// March kernel instances: complex128, closed variant.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c128_closed(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C128, Variant::Closed>(steps, last, ppl, lds);
}

}  // namespace tsq
