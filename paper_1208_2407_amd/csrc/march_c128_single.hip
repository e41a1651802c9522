// March kernel instances: complex128, single variant.
#include "tsq_march.hpp"

namespace tsq {

const void* march_ptr_c128_single(int steps, bool last, int ppl, bool lds) {
    return pick_kernel<C128, Variant::Single>(steps, last, ppl, lds);
}

}  // namespace tsq
