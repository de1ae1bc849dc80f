// Vector stages of the preconditioner's conjugate-gradient iteration, gfx950.
//
// The preconditioned gradient solves (-1/2 nabla^2 - eps_b) x = g for every
// orbital b (Sec. 2, Eq. "precon") by preconditioned conjugate gradients.  The
// operator application is the kinetic recursion with K_0 = -eps s (Sec. 3.4,
// last sentence), run by the 1D pass kernels; this file holds everything
// else, for a whole batch at once:
//   init     r = g, p = z = r / diag, x = 0
//   alpha    per orbital: alpha = (r.z) / (p.q), with p.q = p.Kin p - eps p.p
//   update1  x += alpha p, r -= alpha q, z = r / diag
//   beta     per orbital: beta = (r.z)_new / (r.z)_old
//   update2  p = z + beta p
// The Jacobi preconditioner diag is the diagonal of the operator in the
// wavelet basis: per axis one value for scaling and one for wavelet
// coefficients (OrbDev::kdiag), minus eps.  Every element kernel reads and
// writes the plan's storage precision and computes in float64; dot products
// are block partial sums (one per tile of 2048 points), summed per orbital in a
// fixed order by one workgroup, so results are deterministic.

#include "wvl_kernels.h"

namespace wvl {

struct CgScal { double alpha, beta, rz, pad; };

// Tiles of the element kernels: kCgTile consecutive elements of one orbital,
// in chunks of kCgPer per thread at a stride of kThreads (coalesced); the
// loads of a chunk are issued before any is used, and a tile is long enough
// to amortise the lookup of its orbital.  Each thread walks its elements with
// the (x, y, z) position stepped incrementally, so the diagonal needs no
// division per element.
constexpr int kCgPer = 8;                      // elements per thread and chunk
constexpr int kCgChunks = 4;                   // chunks per tile
constexpr int kCgTile = kThreads * kCgPer * kCgChunks;

struct CgPos {
  int x, y, z, dx, dy, dz, m1, m2;
  __device__ CgPos(const OrbDev& od, uint32_t e0) : m1(od.m[0]), m2(od.m[1]) {
    const uint32_t row = e0 / (uint32_t)m1;
    x = (int)(e0 - row * (uint32_t)m1);
    y = (int)(row % (uint32_t)m2);
    z = (int)(row / (uint32_t)m2);
    dx = kThreads % m1;
    const int rows = kThreads / m1;
    dy = rows % m2;
    dz = rows / m2;
  }
  __device__ void next() {
    x += dx;
    int cy = dy;
    if (x >= m1) { x -= m1; ++cy; }
    y += cy;
    int cz = dz;
    while (y >= m2) { y -= m2; ++cz; }
    z += cz;
  }
  __device__ double diag(const OrbDev& od, double eps) const {
    return od.kdiag[0][x & 1] + od.kdiag[1][y & 1] + od.kdiag[2][z & 1] - eps;
  }
};

template <int P>
__global__ __launch_bounds__(kThreads) void k_cg_init(PassGeom g, const void* gin, void* x, void* r,
                                                      void* p, const double* __restrict__ eps,
                                                      int64_t plane, double* prz, double* ppp,
                                                      double* prr) {
  using T = Prec<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const uint32_t M = (uint32_t)od.m[0] * od.m[1] * od.m[2];
  const uint32_t e0 = (uint32_t)t * kCgTile + threadIdx.x;
  const double ep = eps[b];
  double rz = 0.0, pp = 0.0, rr = 0.0;
  CgPos pos(od, e0);
  #pragma unroll 1
  for (int k = 0; k < kCgPer * kCgChunks; ++k) {
    const uint32_t e = e0 + (uint32_t)k * kThreads;
    if (e < M) {
      const int64_t i = od.off + e;
      const double rv = T::d(T::ldc(gin, i, plane));
      const double z = rv / pos.diag(od, ep);
      T::st(r, i, plane, T::from_d(rv));
      T::st(p, i, plane, T::from_d(z));
      T::st(x, i, plane, T::from_d(0.0));
      rz += rv * z;
      pp += z * z;
      rr += rv * rv;
    }
    pos.next();
  }
  block_sum_store(rz, prz + blockIdx.x);
  block_sum_store(pp, ppp + blockIdx.x);
  block_sum_store(rr, prr + blockIdx.x);
}

__device__ double cg_block_sum(double v) {
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

// sum of the tiles [pre[b], pre[b+1]) of a partial array (nullable: 0)
__device__ __forceinline__ double orb_sum(const double* part, const int32_t* pre, int b) {
  double s = 0.0;
  if (part)
    for (int i = pre[b] + threadIdx.x; i < pre[b + 1]; i += kThreads) s += part[i];
  return cg_block_sum(s);
}

// one workgroup per orbital: p.q = (kinetic partials of the passes) - eps p.p
__global__ __launch_bounds__(kThreads) void k_cg_alpha(const int32_t* pz, const int32_t* py,
                                                       const int32_t* px, const int32_t* pp,
                                                       const double* ez, const double* ey,
                                                       const double* ex, const double* prz,
                                                       const double* ppp, const double* eps,
                                                       CgScal* sc) {
  const int b = blockIdx.x;
  const double kin = orb_sum(ez, pz, b) + orb_sum(ey, py, b) + orb_sum(ex, px, b);
  const double rz = orb_sum(prz, pp, b);
  const double pn = orb_sum(ppp, pp, b);
  if (threadIdx.x == 0) {
    const double pq = kin - eps[b] * pn;
    sc[b].alpha = (pq > 0.0 && rz > 0.0) ? rz / pq : 0.0;
    sc[b].rz = rz;
  }
}

// x += alpha p; r -= alpha (q - shift eps p); z = r / diag; partials of r.z, r.r
template <int P>
__global__ __launch_bounds__(kThreads) void k_cg_update1(PassGeom g, void* x, void* r, const void* p,
                                                         const void* q, const double* __restrict__ eps,
                                                         int shift, const CgScal* __restrict__ sc,
                                                         int64_t plane, double* prz, double* prr) {
  using T = Prec<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const uint32_t M = (uint32_t)od.m[0] * od.m[1] * od.m[2];
  const uint32_t e0 = (uint32_t)t * kCgTile + threadIdx.x;
  const double a = sc[b].alpha, ep = eps[b];
  const double sh = shift ? ep : 0.0;
  double rz = 0.0, rr = 0.0;
  CgPos pos(od, e0);
  #pragma unroll 1
  for (int ch = 0; ch < kCgChunks; ++ch) {
  const uint32_t c0 = e0 + (uint32_t)(ch * kCgPer) * kThreads;
  // every load of the chunk is issued before the first use
  double pv[kCgPer], qv[kCgPer], xv[kCgPer], rv[kCgPer];
  #pragma unroll
  for (int k = 0; k < kCgPer; ++k) {
    const uint32_t e = c0 + (uint32_t)k * kThreads;
    pv[k] = qv[k] = xv[k] = rv[k] = 0.0;
    if (e < M) {
      const int64_t i = od.off + e;
      pv[k] = T::d(T::ldc(p, i, plane));
      qv[k] = T::d(T::ldc(q, i, plane));
      xv[k] = T::d(T::ldc(x, i, plane));
      rv[k] = T::d(T::ldc(r, i, plane));
    }
  }
  #pragma unroll
  for (int k = 0; k < kCgPer; ++k) {
    const uint32_t e = c0 + (uint32_t)k * kThreads;
    if (e < M) {
      const int64_t i = od.off + e;
      const double qs = qv[k] - sh * pv[k];
      const double xn = xv[k] + a * pv[k];
      const double rn = rv[k] - a * qs;
      T::st(x, i, plane, T::from_d(xn));
      T::st(r, i, plane, T::from_d(rn));
      rz += rn * (rn / pos.diag(od, ep));
      rr += rn * rn;
    }
    pos.next();
  }
  }
  block_sum_store(rz, prz + blockIdx.x);
  block_sum_store(rr, prr + blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_cg_beta(const int32_t* pp, const double* prz,
                                                      CgScal* sc) {
  const int b = blockIdx.x;
  const double rz = orb_sum(prz, pp, b);
  if (threadIdx.x == 0) {
    const double old = sc[b].rz;
    sc[b].beta = old > 0.0 ? rz / old : 0.0;
    sc[b].rz = rz;
  }
}

// p = r / diag + beta p; partials of p.p
template <int P>
__global__ __launch_bounds__(kThreads) void k_cg_update2(PassGeom g, const void* r, void* p,
                                                         const double* __restrict__ eps,
                                                         const CgScal* __restrict__ sc,
                                                         int64_t plane, double* ppp) {
  using T = Prec<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const uint32_t M = (uint32_t)od.m[0] * od.m[1] * od.m[2];
  const uint32_t e0 = (uint32_t)t * kCgTile + threadIdx.x;
  const double beta = sc[b].beta, ep = eps[b];
  double pp = 0.0;
  CgPos pos(od, e0);
  #pragma unroll 1
  for (int ch = 0; ch < kCgChunks; ++ch) {
  const uint32_t c0 = e0 + (uint32_t)(ch * kCgPer) * kThreads;
  double rv[kCgPer], pv[kCgPer];
  #pragma unroll
  for (int k = 0; k < kCgPer; ++k) {
    const uint32_t e = c0 + (uint32_t)k * kThreads;
    rv[k] = pv[k] = 0.0;
    if (e < M) {
      const int64_t i = od.off + e;
      rv[k] = T::d(T::ldc(r, i, plane));
      pv[k] = T::d(T::ldc(p, i, plane));
    }
  }
  #pragma unroll
  for (int k = 0; k < kCgPer; ++k) {
    const uint32_t e = c0 + (uint32_t)k * kThreads;
    if (e < M) {
      const int64_t i = od.off + e;
      const double pn = rv[k] / pos.diag(od, ep) + beta * pv[k];
      T::st(p, i, plane, T::from_d(pn));
      pp += pn * pn;
    }
    pos.next();
  }
  }
  block_sum_store(pp, ppp + blockIdx.x);
}

// K_0 = -eps_b s (the initial value of the kinetic recursion, Sec. 3.4)
template <int P>
__global__ __launch_bounds__(kThreads) void k_cg_shift(PassGeom g, const void* s, void* k0,
                                                       const double* __restrict__ eps,
                                                       int64_t plane) {
  using T = Prec<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const uint32_t M = (uint32_t)od.m[0] * od.m[1] * od.m[2];
  const double f = -eps[b];
  #pragma unroll 4
  for (int k = 0; k < kCgPer * kCgChunks; ++k) {
    const uint32_t e = (uint32_t)t * kCgTile + (uint32_t)k * kThreads + threadIdx.x;
    if (e < M) {
      const int64_t i = od.off + e;
      T::st(k0, i, plane, T::scale(T::ldc(s, i, plane), f));
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_res(const int32_t* pp, const double* prr,
                                                     double* res) {
  const int b = blockIdx.x;
  const double rr = orb_sum(prr, pp, b);
  if (threadIdx.x == 0) res[b] = sqrt(rr);
}

// ---------------------------------------------------------------------------
#define WVL_PREC_SWITCH(prec, KERN, ...)                                               \
  switch (prec) {                                                                      \
    case F64: hipLaunchKernelGGL((KERN<F64>), __VA_ARGS__); break;                     \
    case F32: hipLaunchKernelGGL((KERN<F32>), __VA_ARGS__); break;                     \
    default:  hipLaunchKernelGGL((KERN<F32C>), __VA_ARGS__); break;                    \
  }

hipError_t launch_cg_init(int prec, const PassGeom& g, int ntiles, const void* gin, void* x,
                          void* r, void* p, const double* eps, int64_t plane, double* prz,
                          double* ppp, double* prr, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  WVL_PREC_SWITCH(prec, k_cg_init, dim3(ntiles), dim3(kThreads), 0, st, g, gin, x, r, p, eps, plane,
                  prz, ppp, prr);
  return hipGetLastError();
}

hipError_t launch_cg_alpha(int norb, const int32_t* pz, const int32_t* py, const int32_t* px,
                           const int32_t* pp, const double* ez, const double* ey, const double* ex,
                           const double* prz, const double* ppp, const double* eps, void* sc,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(norb), dim3(kThreads), 0, st, pz, py, px, pp, ez, ey, ex, prz,
                     ppp, eps, (CgScal*)sc);
  return hipGetLastError();
}

hipError_t launch_cg_update1(int prec, const PassGeom& g, int ntiles, void* x, void* r,
                             const void* p, const void* q, const double* eps, int shift,
                             const void* sc, int64_t plane, double* prz, double* prr,
                             hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  WVL_PREC_SWITCH(prec, k_cg_update1, dim3(ntiles), dim3(kThreads), 0, st, g, x, r, p, q, eps, shift,
                  (const CgScal*)sc, plane, prz, prr);
  return hipGetLastError();
}

hipError_t launch_cg_beta(int norb, const int32_t* pp, const double* prz, void* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta, dim3(norb), dim3(kThreads), 0, st, pp, prz, (CgScal*)sc);
  return hipGetLastError();
}

hipError_t launch_cg_update2(int prec, const PassGeom& g, int ntiles, const void* r, void* p,
                             const double* eps, const void* sc, int64_t plane, double* ppp,
                             hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  WVL_PREC_SWITCH(prec, k_cg_update2, dim3(ntiles), dim3(kThreads), 0, st, g, r, p, eps,
                  (const CgScal*)sc, plane, ppp);
  return hipGetLastError();
}

hipError_t launch_cg_shift(int prec, const PassGeom& g, int ntiles, const void* s, void* k0,
                           const double* eps, int64_t plane, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  WVL_PREC_SWITCH(prec, k_cg_shift, dim3(ntiles), dim3(kThreads), 0, st, g, s, k0, eps, plane);
  return hipGetLastError();
}

hipError_t launch_cg_res(int norb, const int32_t* pp, const double* prr, double* res,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_cg_res, dim3(norb), dim3(kThreads), 0, st, pp, prr, res);
  return hipGetLastError();
}

size_t cg_scalar_bytes() { return sizeof(CgScal); }
int cg_tile_elems() { return kCgTile; }

}  // namespace wvl
