// In-plane preconditioner kernel instantiations: float64 matrix-core engine.
#include "wvl_xy_impl.h"

namespace wvl {
void helm_launch_mf(const HelmArgs& a, int mt, int nblocks, size_t lds, hipStream_t st) {
  helm_launch_m(a, mt, nblocks, lds, st);
}
}  // namespace wvl
