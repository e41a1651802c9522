// March kernel instances: complex64, batch variant.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c64_batch(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C64, Variant::Batch>(steps, last, ppl, lds);
}

}  // namespace tsq
