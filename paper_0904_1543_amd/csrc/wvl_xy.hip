// Host dispatch of the in-plane kernel (the device code is in wvl_xy_impl.h,
// instantiated per precision and engine by the wvl_xy_<form>.hip files).

#include <stdlib.h>

#include "wvl_plane.h"

namespace wvl {

template <int P, bool SH>
void xy_launch_v(const XyArgs& a, int mi, int nblocks, size_t lds, hipStream_t st);
template <bool SH>
void xy_launch_m(const XyArgs& a, int mt, int nblocks, size_t lds, hipStream_t st);
template <int P>
void helm_launch_v(const HelmArgs& a, int mi, int nblocks, size_t lds, hipStream_t st);
void helm_launch_mf(const HelmArgs& a, int mt, int nblocks, size_t lds, hipStream_t st);

// rho[r] = sum_g rho_part[g][r] (group order), and per-block sums of V rho
__global__ __launch_bounds__(kThreads) void k_rho_reduce(const double* __restrict__ part, int ngroups,
                                                         int64_t M, const double* __restrict__ V,
                                                         double* rho, double* __restrict__ rvpart) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double s = 0.0;
  if (r < M)
    for (int g = 0; g < ngroups; ++g) s += part[(int64_t)g * M + r];
  if (rho && r < M) rho[r] = s;
  if (rvpart) block_sum_store(r < M ? V[r] * s : 0.0, rvpart + blockIdx.x);
}

static int xy_items(int m1, int m2) {
  const int ix = ((m1 + kU - 1) / kU) * m2, iy = ((m2 + kU - 1) / kU) * m1;
  const int it = ix > iy ? ix : iy;
  return (it + kXyThreads - 1) / kXyThreads;
}
static int xy_tiles(int m1, int m2) {
  const int nt = ((m1 + 15) / 16) * ((m2 + 15) / 16);
  return (nt + kXyWaves - 1) / kXyWaves;
}
static int mf_pitch(int m1) { return m1 + ((36 - (m1 & 31)) & 31); }

bool xy_matrix_engine(int prec, int m1, int m2) {
  return prec == F64 && xy_tiles(m1, m2) <= 8 && (size_t)m2 * mf_pitch(m1) * 8 <= 160 * 1024;
}

size_t xy_lds_bytes(int prec, int m1, int m2, bool engine) {
  if (engine) return (size_t)m2 * mf_pitch(m1) * 8;
  return (size_t)m2 * (m1 + 1) * (prec == F32 ? 4 : 8);
}

bool xy_supported(int prec, int m1, int m2, bool engine) {
  if (engine) return xy_matrix_engine(prec, m1, m2);
  return xy_items(m1, m2) <= kMaxItems && xy_lds_bytes(prec, m1, m2, false) <= 160 * 1024;
}

hipError_t launch_xy(int prec, const XyArgs& a, int m1, int m2, int nblocks, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  const bool sh = a.shared != 0;
  const bool mx = a.engine != 0;
  if (mx && !xy_matrix_engine(prec, m1, m2)) return hipErrorInvalidValue;
  const size_t lds = xy_lds_bytes(prec, m1, m2, mx);
  if (mx) {
    const int mt = xy_tiles(m1, m2);
    // one workgroup per CU anyway at 2 waves per SIMD: keep the group's
    // density plane in LDS beside the plane (same pitch) when both fit
    XyArgs b = a;
    b.rho_lds = sh && a.occupancy == 2 && 2 * lds <= 160 * 1024 && !getenv("WVL_NO_RHO_LDS");
    const size_t l = b.rho_lds ? 2 * lds : lds;
    sh ? xy_launch_m<true>(b, mt, nblocks, l, st) : xy_launch_m<false>(b, mt, nblocks, l, st);
    return hipGetLastError();
  }
  const int mi = xy_items(m1, m2);
  switch (prec) {
    case F64: sh ? xy_launch_v<F64, true>(a, mi, nblocks, lds, st) : xy_launch_v<F64, false>(a, mi, nblocks, lds, st); break;
    case F32: sh ? xy_launch_v<F32, true>(a, mi, nblocks, lds, st) : xy_launch_v<F32, false>(a, mi, nblocks, lds, st); break;
    default:  sh ? xy_launch_v<F32C, true>(a, mi, nblocks, lds, st) : xy_launch_v<F32C, false>(a, mi, nblocks, lds, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_helm_xy(int prec, const HelmArgs& a, int m1, int m2, int nblocks, bool engine,
                          hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  if (engine && !xy_matrix_engine(prec, m1, m2)) return hipErrorInvalidValue;
  const size_t lds = xy_lds_bytes(prec, m1, m2, engine);
  if (engine) {
    helm_launch_mf(a, xy_tiles(m1, m2), nblocks, lds, st);
    return hipGetLastError();
  }
  const int mi = xy_items(m1, m2);
  switch (prec) {
    case F64: helm_launch_v<F64>(a, mi, nblocks, lds, st); break;
    case F32: helm_launch_v<F32>(a, mi, nblocks, lds, st); break;
    default:  helm_launch_v<F32C>(a, mi, nblocks, lds, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_rho_reduce(const double* part, int ngroups, int64_t M, const double* V,
                             double* rho, double* rvpart, hipStream_t st) {
  const int nblk = (int)((M + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_rho_reduce, dim3(nblk), dim3(kThreads), 0, st, part, ngroups, M, V, rho,
                     rvpart);
  return hipGetLastError();
}

}  // namespace wvl
