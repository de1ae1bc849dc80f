// In-plane kernel instantiations: F64, vector engine, shared potential.
#include "wvl_xy_impl.h"

namespace wvl {
template void xy_launch_v<F64, true>(const XyArgs&, int, int, size_t, hipStream_t);
}  // namespace wvl
