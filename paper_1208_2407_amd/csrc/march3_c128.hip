// March kernel instances: complex128, three-dimensional meshes.
#include "tsq_march3.hpp"

namespace tsq {

const void* march3_ptr_c128(bool close) { return pick_kernel3<C128>(close); }

}  // namespace tsq
