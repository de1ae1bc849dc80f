// In-plane preconditioner kernel instantiations: F32C, vector engine.
#include "wvl_xy_impl.h"

namespace wvl {
template void helm_launch_v<F32C>(const HelmArgs&, int, int, size_t, hipStream_t);
}  // namespace wvl
