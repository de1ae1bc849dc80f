// Pointwise stages and float64 reductions, gfx950.
//
//  * density rho = sum_i f_i psi_i^2 (Sec. 2, Eq. "density"; Sec. 2.5) and the
//    potential product y = V psi (Sec. 2.4 step 3b).  The density is always
//    accumulated in float64 and in a fixed orbital order (one thread owns one
//    grid point and walks the orbitals), so results are bitwise reproducible;
//  * energies as float64 reductions (the paper calls BLAS for them, Sec. 4.1):
//    fixed-order two-stage sums, no floating-point atomics.

#include <algorithm>

#include "wvl_kernels.h"

namespace wvl {

template <int P, bool WRITE_Y, bool ORB_E>
__global__ __launch_bounds__(kThreads) void k_pot_shared(const OrbDev* __restrict__ orbs, int norb,
                                                         int64_t M, const void* psi, void* y,
                                                         const double* __restrict__ V,
                                                         double pot_scale, int64_t plane,
                                                         double* rho, int rho_acc,
                                                         double* __restrict__ rvpart,
                                                         double* __restrict__ ppart) {
  using T = Prec<P>;
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool act = r < M;
  const double v = (act && V) ? V[r] : 0.0;
  const double vs = v * pot_scale;
  double acc = 0.0;
  for (int b = 0; b < norb; ++b) {
    const int64_t off = orbs[b].off;
    double pd = 0.0;
    if (act) {
      const typename T::V p = T::ldc(psi, off + r, plane);
      pd = T::d(p);
      acc = __builtin_fma(orbs[b].occ * pd, pd, acc);
      if (WRITE_Y) T::st(y, off + r, plane, T::scale(p, vs));
    }
    if (ORB_E) block_sum_store(v * pd * pd, ppart + (int64_t)b * gridDim.x + blockIdx.x);
  }
  if (rho && act) rho[r] = rho_acc ? rho[r] + acc : acc;
  if (rvpart) block_sum_store(v * acc, rvpart + blockIdx.x);
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_pot_orb(PassGeom g, const void* psi, void* y,
                                                      const double* __restrict__ V,
                                                      double pot_scale, int64_t plane,
                                                      double* __restrict__ ppart) {
  using T = Prec<P>;
  for_each_tile(g, [&](int b, int t, int slot) {
    const OrbDev od = g.orbs[b];
    const int64_t M = (int64_t)od.m[0] * od.m[1] * od.m[2];
    const int64_t r = (int64_t)t * kThreads + threadIdx.x;
    double e = 0.0;
    if (r < M) {
      const double v = V[od.voff + r];
      const typename T::V p = T::ldc(psi, od.off + r, plane);
      const double pd = T::d(p);
      e = v * pd * pd;
      if (y) T::st(y, od.off + r, plane, T::scale(p, v * pot_scale));
    }
    if (ppart) block_sum_store(e, ppart + slot);
  });
}

// x_b <- mul * f_b * x_b for every orbital b (the occupation weights of the
// energy gradient 2 f_b H c_b)
template <int P>
__global__ __launch_bounds__(kThreads) void k_scale_occ(PassGeom g, void* x, double mul,
                                                        int64_t plane) {
  using T = Prec<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const int64_t M = (int64_t)od.m[0] * od.m[1] * od.m[2];
  const int64_t r = (int64_t)t * kThreads + threadIdx.x;
  if (r < M) T::st(x, od.off + r, plane, T::scale(T::ldc(x, od.off + r, plane), mul * od.occ));
}

__device__ double block_sum_all(double v) {
  __shared__ double red[kThreads / 64];
  #pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  #pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kThreads) void k_orb_sums(const OrbDev* orbs, int norb,
                                                       const int32_t* pz, const int32_t* py,
                                                       const int32_t* px, const double* ez,
                                                       const double* ey, const double* ex,
                                                       const double* ppart, int pot_mode,
                                                       const int32_t* pp, int nblk, double* eorb) {
  const int b = blockIdx.x;
  double k = 0.0;
  if (ez) for (int i = pz[b] + threadIdx.x; i < pz[b + 1]; i += kThreads) k += ez[i];
  if (ey) for (int i = py[b] + threadIdx.x; i < py[b + 1]; i += kThreads) k += ey[i];
  if (ex) for (int i = px[b] + threadIdx.x; i < px[b + 1]; i += kThreads) k += ex[i];
  double p = 0.0;
  if (pot_mode == 1) {
    for (int i = pp[b] + threadIdx.x; i < pp[b + 1]; i += kThreads) p += ppart[i];
  } else if (pot_mode == 2) {
    for (int i = threadIdx.x; i < nblk; i += kThreads) p += ppart[(int64_t)b * nblk + i];
  }
  const double ks = block_sum_all(k);
  const double ps = block_sum_all(p);
  if (threadIdx.x == 0) {
    eorb[b] = ps;
    eorb[norb + b] = ks;
  }
  (void)orbs;
}

__global__ __launch_bounds__(kThreads) void k_totals(const OrbDev* orbs, int norb,
                                                     const double* eorb, const double* rvpart,
                                                     int nrv, double* e_loc, double* e_kin) {
  double k = 0.0, l = 0.0;
  for (int b = threadIdx.x; b < norb; b += kThreads) {
    k += orbs[b].occ * eorb[norb + b];
    if (nrv == 0) l += orbs[b].occ * eorb[b];
  }
  if (nrv > 0)
    for (int i = threadIdx.x; i < nrv; i += kThreads) l += rvpart[i];
  const double ks = block_sum_all(k);
  const double ls = block_sum_all(l);
  if (threadIdx.x == 0) {
    if (e_kin) *e_kin = ks;
    if (e_loc) *e_loc = ls;
  }
}

// ---------------------------------------------------------------------------
__global__ void k_convert(const void* src, int sp, void* dst, int dp, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double x;
    if (sp == F64) x = ((const double*)src)[i];
    else if (sp == F32) x = (double)((const float*)src)[i];
    else x = (double)((const float*)src)[i] + (double)((const float*)src)[n + i];
    if (dp == F64) ((double*)dst)[i] = x;
    else if (dp == F32) ((float*)dst)[i] = (float)x;
    else {
      const float h = (float)x;
      ((float*)dst)[i] = h;
      ((float*)dst)[n + i] = (float)(x - (double)h);
    }
  }
}

__global__ void k_fill(double* dst, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

// work-queue counters: a kernel (not a memset) so it can sit in a captured graph
__global__ void k_fill_int(int32_t* dst, int n) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
template <int P>
static hipError_t pot_shared_p(const OrbDev* orbs, int norb, int64_t M, const void* psi, void* y,
                               const double* V, double pot_scale, int64_t plane, double* rho,
                               int rho_acc, double* rvpart, double* ppart, hipStream_t st) {
  const int nblk = (int)((M + kThreads - 1) / kThreads);
#define WVL_L(KERN) hipLaunchKernelGGL((KERN), dim3(nblk), dim3(kThreads), 0, st, orbs, norb, M, psi, y, V, pot_scale, plane, rho, rho_acc, rvpart, ppart)
  if (y) { if (ppart) WVL_L((k_pot_shared<P, true, true>)); else WVL_L((k_pot_shared<P, true, false>)); }
  else   { if (ppart) WVL_L((k_pot_shared<P, false, true>)); else WVL_L((k_pot_shared<P, false, false>)); }
#undef WVL_L
  return hipGetLastError();
}

hipError_t launch_pot_shared(int prec, const OrbDev* orbs, int norb, int64_t M, const void* psi,
                             void* y, const double* V, double pot_scale, int64_t plane,
                             double* rho, int rho_acc, double* rvpart, double* ppart,
                             hipStream_t st) {
  if (M == 0) return hipSuccess;
  switch (prec) {
    case F64: return pot_shared_p<F64>(orbs, norb, M, psi, y, V, pot_scale, plane, rho, rho_acc, rvpart, ppart, st);
    case F32: return pot_shared_p<F32>(orbs, norb, M, psi, y, V, pot_scale, plane, rho, rho_acc, rvpart, ppart, st);
    default:  return pot_shared_p<F32C>(orbs, norb, M, psi, y, V, pot_scale, plane, rho, rho_acc, rvpart, ppart, st);
  }
}

hipError_t launch_pot_orb(int prec, const PassGeom& g, int ntiles, const void* psi, void* y,
                          const double* V, double pot_scale, int64_t plane, double* ppart,
                          hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  dim3 grid(g.queue ? std::min(ntiles, g.grid) : ntiles), block(kThreads);
  switch (prec) {
    case F64: hipLaunchKernelGGL((k_pot_orb<F64>), grid, block, 0, st, g, psi, y, V, pot_scale, plane, ppart); break;
    case F32: hipLaunchKernelGGL((k_pot_orb<F32>), grid, block, 0, st, g, psi, y, V, pot_scale, plane, ppart); break;
    default:  hipLaunchKernelGGL((k_pot_orb<F32C>), grid, block, 0, st, g, psi, y, V, pot_scale, plane, ppart); break;
  }
  return hipGetLastError();
}

hipError_t launch_scale_occ(int prec, const PassGeom& g, int ntiles, void* x, double mul,
                           int64_t plane, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  dim3 grid(ntiles), block(kThreads);
  switch (prec) {
    case F64: hipLaunchKernelGGL((k_scale_occ<F64>), grid, block, 0, st, g, x, mul, plane); break;
    case F32: hipLaunchKernelGGL((k_scale_occ<F32>), grid, block, 0, st, g, x, mul, plane); break;
    default:  hipLaunchKernelGGL((k_scale_occ<F32C>), grid, block, 0, st, g, x, mul, plane); break;
  }
  return hipGetLastError();
}

hipError_t launch_orb_sums(const OrbDev* orbs, int norb, const int32_t* pz, const int32_t* py,
                           const int32_t* px, const double* ez, const double* ey, const double* ex,
                           const double* ppart, int pot_mode, const int32_t* pp, int nblk,
                           double* eorb, hipStream_t st) {
  if (norb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_orb_sums, dim3(norb), dim3(kThreads), 0, st, orbs, norb, pz, py, px, ez, ey,
                     ex, ppart, pot_mode, pp, nblk, eorb);
  return hipGetLastError();
}

hipError_t launch_totals(const OrbDev* orbs, int norb, const double* eorb, const double* rvpart,
                         int nrv, double* e_loc, double* e_kin, hipStream_t st) {
  hipLaunchKernelGGL(k_totals, dim3(1), dim3(kThreads), 0, st, orbs, norb, eorb, rvpart, nrv, e_loc,
                     e_kin);
  return hipGetLastError();
}

hipError_t launch_convert(const void* src, int sp, void* dst, int dp, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, st, src, sp, dst, dp, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* dst, int64_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, dst, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_int(int32_t* dst, int n, hipStream_t st) {
  if (n <= 0 || n > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(256), 0, st, dst, n);
  return hipGetLastError();
}

}  // namespace wvl
