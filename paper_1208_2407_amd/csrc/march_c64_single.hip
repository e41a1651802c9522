// March kernel instances: complex64, single variant.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c64_single(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C64, Variant::Single>(steps, last, ppl, lds);
}

}  // namespace tsq
