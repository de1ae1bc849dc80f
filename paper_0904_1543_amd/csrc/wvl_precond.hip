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
// are block partial sums (one per tile of 8192 points), summed per orbital in a
// fixed order by one workgroup, so results are deterministic.

#include "wvl_kernels.h"

namespace wvl {

struct CgScal { double alpha, beta, rz, pad; };

// Tiles of the element kernels: kCgTile consecutive elements of one orbital.
// A thread moves groups of four consecutive elements (one 16-byte access per
// plane, two in float64): orbital offsets and the plane length are multiples
// of 8 elements (m1 m2 m3 = 8 n1 n2 n3) and batch arrays start on 16-byte
// boundaries, so a group is aligned and never straddles two orbitals.  The
// groups of a thread lie kThreads groups apart (coalesced), kCgG of them per
// chunk with every load of the chunk issued before the first use.  Each
// thread walks its groups with the (x, y, z) position stepped incrementally,
// so the diagonal needs no division per element.
constexpr int kCgG = 2;                        // groups per thread and chunk
constexpr int kCgPer = 4 * kCgG;               // elements per thread and chunk
constexpr int kCgChunks = 4;                   // chunks per tile
constexpr int kCgTile = kThreads * kCgPer * kCgChunks;
constexpr uint32_t kCgStep = 4 * kThreads;     // elements between a thread's groups

// position of the first element of a thread's group
struct CgPos {
  int x, y, z, dx, dy, dz, m1, m2;
  __device__ CgPos(const OrbDev& od, uint32_t e0, uint32_t step) : m1(od.m[0]), m2(od.m[1]) {
    const uint32_t row = e0 / (uint32_t)m1;
    x = (int)(e0 - row * (uint32_t)m1);
    y = (int)(row % (uint32_t)m2);
    z = (int)(row / (uint32_t)m2);
    dx = (int)(step % (uint32_t)m1);
    const int rows = (int)(step / (uint32_t)m1);
    dy = rows % m2;
    dz = rows / m2;
  }
  __device__ void next() {
    x += dx;
    int cy = dy;
    if (x >= m1) { x -= m1; ++cy; }
    y += cy;
    int cz = dz;
    if (y >= m2) { y -= m2; ++cz; }
    z += cz;
  }
};

// 1 / diag per parity class (x, y, z mod 2) of one orbital: diag is the
// kinetic diagonal of the wavelet basis, one value per axis for scaling and
// one for wavelet coefficients, minus eps.
struct CgInv {
  double v[8];   // index (z & 1) << 2 | (y & 1) << 1 | (x & 1)
  __device__ CgInv(const OrbDev& od, double eps) {
    #pragma unroll
    for (int k = 0; k < 8; ++k)
      v[k] = 1.0 / (od.kdiag[0][k & 1] + od.kdiag[1][(k >> 1) & 1] + od.kdiag[2][k >> 2] - eps);
  }
  // the four elements of the group at p: x is even (the group starts at a
  // multiple of 4 and m1 is even), so element j has x parity j & 1; elements
  // 2 and 3 move to the next row when x = m1 - 2 (m2 even: the parity of y
  // + 1 is right also where it wraps to 0, and z advances with it)
  __device__ void group(const CgPos& p, double (&w)[4]) const {
    const int wrap = p.x + 2 >= p.m1 ? 1 : 0;
    const int y1 = p.y + wrap;
    const int z1 = p.z + (y1 == p.m2 ? 1 : 0);
    pair(p.y & 1, p.z & 1, w[0], w[1]);
    pair(y1 & 1, z1 & 1, w[2], w[3]);
  }
  __device__ void pair(int py, int pz, double& a0, double& a1) const {
    a0 = pz ? (py ? v[6] : v[4]) : (py ? v[2] : v[0]);
    a1 = pz ? (py ? v[7] : v[5]) : (py ? v[3] : v[1]);
  }
};

// loads and stores of one group in the plan's storage precision, as float64
template <int P> struct G4;
template <> struct G4<F64> {
  __device__ static void ld(const void* p, int64_t i, int64_t, double (&v)[4]) {
    const double2* q = reinterpret_cast<const double2*>((const double*)p + i);
    const double2 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
  __device__ static void st(void* p, int64_t i, int64_t, const double (&v)[4]) {
    double2* q = reinterpret_cast<double2*>((double*)p + i);
    q[0] = make_double2(v[0], v[1]);
    q[1] = make_double2(v[2], v[3]);
  }
};
template <> struct G4<F32> {
  __device__ static void ld(const void* p, int64_t i, int64_t, double (&v)[4]) {
    const float4 a = *reinterpret_cast<const float4*>((const float*)p + i);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
  __device__ static void st(void* p, int64_t i, int64_t, const double (&v)[4]) {
    *reinterpret_cast<float4*>((float*)p + i) =
        make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  }
};
template <> struct G4<F32C> {
  __device__ static void ld(const void* p, int64_t i, int64_t plane, double (&v)[4]) {
    const float* f = (const float*)p;
    const float4 h = *reinterpret_cast<const float4*>(f + i);
    const float4 l = *reinterpret_cast<const float4*>(f + plane + i);
    v[0] = (double)h.x + (double)l.x;
    v[1] = (double)h.y + (double)l.y;
    v[2] = (double)h.z + (double)l.z;
    v[3] = (double)h.w + (double)l.w;
  }
  __device__ static void st(void* p, int64_t i, int64_t plane, const double (&v)[4]) {
    float h[4], l[4];
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      h[k] = (float)v[k];
      l[k] = (float)(v[k] - (double)h[k]);
    }
    float* f = (float*)p;
    *reinterpret_cast<float4*>(f + i) = make_float4(h[0], h[1], h[2], h[3]);
    *reinterpret_cast<float4*>(f + plane + i) = make_float4(l[0], l[1], l[2], l[3]);
  }
};

template <int P>
__global__ __launch_bounds__(kThreads) void k_cg_init(PassGeom g, const void* gin, void* x, void* r,
                                                      void* p, const double* __restrict__ eps,
                                                      int64_t plane, double* prz, double* ppp,
                                                      double* prr) {
  using L = G4<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const uint32_t M = (uint32_t)od.m[0] * od.m[1] * od.m[2];
  const uint32_t e0 = (uint32_t)t * kCgTile + 4 * threadIdx.x;
  const CgInv inv(od, eps[b]);
  double rz = 0.0, pp = 0.0, rr = 0.0;
  CgPos pos(od, e0, kCgStep);
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  #pragma unroll 1
  for (int k = 0; k < kCgG * kCgChunks; ++k) {
    const uint32_t e = e0 + (uint32_t)k * kCgStep;
    if (e < M) {
      const int64_t i = od.off + e;
      double rv[4], zv[4], w[4];
      L::ld(gin, i, plane, rv);
      inv.group(pos, w);
      #pragma unroll
      for (int j = 0; j < 4; ++j) {
        zv[j] = rv[j] * w[j];
        rz += rv[j] * zv[j];
        pp += zv[j] * zv[j];
        rr += rv[j] * rv[j];
      }
      L::st(r, i, plane, rv);
      L::st(p, i, plane, zv);
      L::st(x, i, plane, zero);
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
  using L = G4<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const uint32_t M = (uint32_t)od.m[0] * od.m[1] * od.m[2];
  const uint32_t e0 = (uint32_t)t * kCgTile + 4 * threadIdx.x;
  const double a = sc[b].alpha, ep = eps[b];
  const double sh = shift ? ep : 0.0;
  const CgInv inv(od, ep);
  double rz = 0.0, rr = 0.0;
  CgPos pos(od, e0, kCgStep);
  #pragma unroll 1
  for (int ch = 0; ch < kCgChunks; ++ch) {
    const uint32_t c0 = e0 + (uint32_t)(ch * kCgG) * kCgStep;
    // every load of the chunk is issued before the first use
    double pv[kCgG][4], qv[kCgG][4], xv[kCgG][4], rv[kCgG][4];
    #pragma unroll
    for (int k = 0; k < kCgG; ++k) {
      const uint32_t e = c0 + (uint32_t)k * kCgStep;
      if (e < M) {
        const int64_t i = od.off + e;
        L::ld(p, i, plane, pv[k]);
        L::ld(q, i, plane, qv[k]);
        L::ld(x, i, plane, xv[k]);
        L::ld(r, i, plane, rv[k]);
      }
    }
    #pragma unroll
    for (int k = 0; k < kCgG; ++k) {
      const uint32_t e = c0 + (uint32_t)k * kCgStep;
      if (e < M) {
        const int64_t i = od.off + e;
        double w[4], xn[4], rn[4];
        inv.group(pos, w);
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double qs = qv[k][j] - sh * pv[k][j];
          xn[j] = xv[k][j] + a * pv[k][j];
          rn[j] = rv[k][j] - a * qs;
          rz += rn[j] * (rn[j] * w[j]);
          rr += rn[j] * rn[j];
        }
        L::st(x, i, plane, xn);
        L::st(r, i, plane, rn);
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
  using L = G4<P>;
  int b, t;
  find_tile(g.prefix, g.norb, blockIdx.x, b, t);
  const OrbDev od = g.orbs[b];
  const uint32_t M = (uint32_t)od.m[0] * od.m[1] * od.m[2];
  const uint32_t e0 = (uint32_t)t * kCgTile + 4 * threadIdx.x;
  const double beta = sc[b].beta;
  const CgInv inv(od, eps[b]);
  double pp = 0.0;
  CgPos pos(od, e0, kCgStep);
  #pragma unroll 1
  for (int ch = 0; ch < kCgChunks; ++ch) {
    const uint32_t c0 = e0 + (uint32_t)(ch * kCgG) * kCgStep;
    double rv[kCgG][4], pv[kCgG][4];
    #pragma unroll
    for (int k = 0; k < kCgG; ++k) {
      const uint32_t e = c0 + (uint32_t)k * kCgStep;
      if (e < M) {
        const int64_t i = od.off + e;
        L::ld(r, i, plane, rv[k]);
        L::ld(p, i, plane, pv[k]);
      }
    }
    #pragma unroll
    for (int k = 0; k < kCgG; ++k) {
      const uint32_t e = c0 + (uint32_t)k * kCgStep;
      if (e < M) {
        const int64_t i = od.off + e;
        double w[4], pn[4];
        inv.group(pos, w);
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
          pn[j] = rv[k][j] * w[j] + beta * pv[k][j];
          pp += pn[j] * pn[j];
        }
        L::st(p, i, plane, pn);
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
