// In-plane kernel instantiations: F32C, vector engine, shared potential.
#include "wvl_xy_impl.h"

namespace wvl {
template void xy_launch_v<F32C, true>(const XyArgs&, int, int, size_t, hipStream_t);
}  // namespace wvl
