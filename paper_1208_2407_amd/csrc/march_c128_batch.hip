// March kernel instances: complex128, batch variant.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c128_batch(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C128, Variant::Batch>(steps, last, ppl, lds);
}

}  // namespace tsq
