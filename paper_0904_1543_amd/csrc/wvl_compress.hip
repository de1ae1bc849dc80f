// Compressed storage of the orbitals: unpack onto the whole grid and pack
// back (steps 1 and 7 of the local Hamiltonian, Sec. 2.4), gfx950.
//
// Sec. 2.1: an orbital stores its scaling coefficient only at the coarse
// points of the low-resolution region and its seven wavelet coefficients only
// at the points of the high-resolution region.  The compressed vector of one
// orbital is [coarse-region scaling coefficients][7 per fine-region point];
// regions are given as segments of consecutive points along axis 1.  Both
// kernels are gathers, so every store is coalesced:
//  * decompress: one thread per element of the full interleaved grid; the
//    element's coarse point and component mu = b1 + 2 b2 + 4 b3 select the
//    compressed index through a per-point map (-1: not stored, value 0);
//  * compress: one thread per compressed element; the region's point list
//    gives the full-grid position to read.

#include "wvl_kernels.h"

namespace wvl {

template <int P>
__global__ __launch_bounds__(kThreads) void k_decompress(const OrbDev* __restrict__ orbs, int norb,
                                                         const int32_t* __restrict__ map_c,
                                                         const int32_t* __restrict__ map_f,
                                                         int64_t nvc, int64_t L, const void* in,
                                                         int64_t plane_in, void* out,
                                                         int64_t plane_out) {
  using T = Prec<P>;
  const OrbDev o0 = orbs[0];
  const int m1 = o0.m[0], m2 = o0.m[1], m3 = o0.m[2];
  const int n1 = m1 >> 1, n2 = m2 >> 1;
  const uint32_t M = (uint32_t)m1 * m2 * m3;
  const int64_t total = (int64_t)M * norb;
  for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * kThreads) {
    const int b = (int)(g / M);
    const uint32_t e = (uint32_t)(g - (int64_t)b * M);
    const uint32_t row = e / (uint32_t)m1;
    const int x = (int)(e - row * (uint32_t)m1);
    const int y = (int)(row % (uint32_t)m2), z = (int)(row / (uint32_t)m2);
    const int pnt = (x >> 1) + n1 * ((y >> 1) + n2 * (z >> 1));
    const int mu = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
    const int64_t src = (int64_t)b * L;
    typename T::V v = T::from_d(0.0);
    if (mu == 0) {
      const int k = map_c[pnt];
      if (k >= 0) v = T::ldc(in, src + k, plane_in);
    } else {
      const int k = map_f[pnt];
      if (k >= 0) v = T::ldc(in, src + nvc + 7 * (int64_t)k + mu - 1, plane_in);
    }
    T::st(out, orbs[b].off + e, plane_out, v);
  }
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_compress(const OrbDev* __restrict__ orbs, int norb,
                                                       const int32_t* __restrict__ list_c,
                                                       const int32_t* __restrict__ list_f,
                                                       int64_t nvc, int64_t L, const void* in,
                                                       int64_t plane_in, void* out,
                                                       int64_t plane_out) {
  using T = Prec<P>;
  const OrbDev o0 = orbs[0];
  const int m1 = o0.m[0], m2 = o0.m[1];
  const int n1 = m1 >> 1, n2 = m2 >> 1;
  const int64_t total = L * norb;
  for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * kThreads) {
    const int b = (int)(g / L);
    const int64_t j = g - (int64_t)b * L;
    int pnt, mu;
    if (j < nvc) {
      pnt = list_c[j];
      mu = 0;
    } else {
      const int64_t k = (j - nvc) / 7;
      mu = (int)(j - nvc - 7 * k) + 1;
      pnt = list_f[k];
    }
    const int i1 = pnt % n1, r = pnt / n1;
    const int i2 = r % n2, i3 = r / n2;
    const int64_t e = ((int64_t)(2 * i3 + ((mu >> 2) & 1)) * m2 + (2 * i2 + ((mu >> 1) & 1))) * m1 +
                      2 * i1 + (mu & 1);
    T::st(out, g, plane_out, T::ldc(in, orbs[b].off + e, plane_in));
  }
}

static unsigned grid_for(int64_t n) {
  int64_t blocks = (n + kThreads - 1) / kThreads;
  return (unsigned)(blocks > 65536 ? 65536 : (blocks < 1 ? 1 : blocks));
}

hipError_t launch_decompress(int prec, const OrbDev* orbs, int norb, int64_t M,
                             const int32_t* map_c, const int32_t* map_f, int64_t nvc, int64_t L,
                             const void* in, int64_t plane_in, void* out, int64_t plane_out,
                             hipStream_t st) {
  const dim3 g(grid_for(M * norb)), b(kThreads);
  switch (prec) {
    case F64: hipLaunchKernelGGL((k_decompress<F64>), g, b, 0, st, orbs, norb, map_c, map_f, nvc, L, in, plane_in, out, plane_out); break;
    case F32: hipLaunchKernelGGL((k_decompress<F32>), g, b, 0, st, orbs, norb, map_c, map_f, nvc, L, in, plane_in, out, plane_out); break;
    default:  hipLaunchKernelGGL((k_decompress<F32C>), g, b, 0, st, orbs, norb, map_c, map_f, nvc, L, in, plane_in, out, plane_out); break;
  }
  return hipGetLastError();
}

hipError_t launch_compress(int prec, const OrbDev* orbs, int norb, const int32_t* list_c,
                           const int32_t* list_f, int64_t nvc, int64_t L, const void* in,
                           int64_t plane_in, void* out, int64_t plane_out, hipStream_t st) {
  if (L == 0) return hipSuccess;
  const dim3 g(grid_for(L * norb)), b(kThreads);
  switch (prec) {
    case F64: hipLaunchKernelGGL((k_compress<F64>), g, b, 0, st, orbs, norb, list_c, list_f, nvc, L, in, plane_in, out, plane_out); break;
    case F32: hipLaunchKernelGGL((k_compress<F32>), g, b, 0, st, orbs, norb, list_c, list_f, nvc, L, in, plane_in, out, plane_out); break;
    default:  hipLaunchKernelGGL((k_compress<F32C>), g, b, 0, st, orbs, norb, list_c, list_f, nvc, L, in, plane_in, out, plane_out); break;
  }
  return hipGetLastError();
}

}  // namespace wvl
