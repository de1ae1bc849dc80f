// In-plane preconditioner kernel instantiations: F64, vector engine.
#include "wvl_xy_impl.h"

namespace wvl {
template void helm_launch_v<F64>(const HelmArgs&, int, int, size_t, hipStream_t);
}  // namespace wvl
