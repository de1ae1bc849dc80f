// 1D pass kernels instantiated for F32.
#include "wvl_passes_impl.h"

namespace wvl {
template hipError_t launch_op<F32>(int, int, const PassGeom&, int, const void*, void*, const void*,
                                  int64_t, double, double*, hipStream_t);
template hipError_t zfinal_p<F32>(const PassGeom&, int, const void*, const void*, const void*, void*,
                                 int64_t, double, double*, hipStream_t);
}  // namespace wvl
