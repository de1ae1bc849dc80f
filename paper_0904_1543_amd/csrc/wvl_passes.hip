// Dispatch of the 1D pass kernels by precision (the device code is in
// wvl_passes_impl.h, instantiated per precision by wvl_passes_<prec>.hip).

#include "wvl_kernels.h"

namespace wvl {

template <int P>
hipError_t launch_op(int op, int axis, const PassGeom& g, int ntiles, const void* in, void* out,
                     const void* k0, int64_t plane, double kmul, double* epart, hipStream_t st);
template <int P>
hipError_t zfinal_p(const PassGeom& g, int ntiles, const void* t, const void* c, const void* kxy,
                    void* out, int64_t plane, double kmul, double* epart, hipStream_t st);

hipError_t launch_zfinal(int prec, const PassGeom& g, int ntiles, const void* t, const void* c,
                         const void* kxy, void* out, int64_t plane, double kmul, double* epart,
                         hipStream_t st) {
  switch (prec) {
    case F64: return zfinal_p<F64>(g, ntiles, t, c, kxy, out, plane, kmul, epart, st);
    case F32: return zfinal_p<F32>(g, ntiles, t, c, kxy, out, plane, kmul, epart, st);
    default:  return zfinal_p<F32C>(g, ntiles, t, c, kxy, out, plane, kmul, epart, st);
  }
}

hipError_t launch_pass(int prec, int op, int axis, const PassGeom& g, int ntiles, const void* in,
                       void* out, const void* k0, int64_t plane, double kmul, double* epart,
                       hipStream_t st) {
  switch (prec) {
    case F64: return launch_op<F64>(op, axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    case F32: return launch_op<F32>(op, axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    default:  return launch_op<F32C>(op, axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
  }
}

}  // namespace wvl
