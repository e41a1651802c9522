// March kernel instances: complex64, closed variant.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c64_closed(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C64, Variant::Closed>(steps, last, ppl, lds);
}

}  // namespace tsq
