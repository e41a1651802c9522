// March kernel instances: complex64, three-dimensional meshes.
#include "tsq_march3.hpp"

namespace tsq {

const void* march3_ptr_c64(bool close) { return pick_kernel3<C64>(close); }

}  // namespace tsq
