// In-plane kernel instantiations: float64 matrix-core engine, shared potential.
#include "wvl_xy_impl.h"

namespace wvl {
template void xy_launch_m<true>(const XyArgs&, int, int, size_t, hipStream_t);
}  // namespace wvl
