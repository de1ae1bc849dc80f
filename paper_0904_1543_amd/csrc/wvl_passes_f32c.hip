// 1D pass kernels instantiated for F32C.
#include "wvl_passes_impl.h"

namespace wvl {
template hipError_t launch_op<F32C>(int, int, const PassGeom&, int, const void*, void*, const void*,
                                  int64_t, double, double*, hipStream_t);
template hipError_t zfinal_p<F32C>(const PassGeom&, int, const void*, const void*, const void*, void*,
                                 int64_t, double, double*, hipStream_t);
}  // namespace wvl
