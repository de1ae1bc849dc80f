// The in-plane part of the local Hamiltonian, one z-plane per workgroup, gfx950.
//
// The 3D operators are tensor products of 1D operators (Sec. 3.1), so the
// local Hamiltonian of one orbital factorises along z:
//     psi = W_x W_y u,            u  = W_z c            (W = magic filter o synthesis)
//     Hc  = W_z^T t + K_z c + kxy, t = W_y^T W_x^T (V psi), kxy = (K_x + K_y) c
// with W^T = analysis o transposed magic filter and K = analysis o kinetic o
// synthesis (the combined filters of Sec. 2.4, last paragraph; the kinetic
// part uses A_a S_a = I on the other axes).  This kernel does everything that
// stays inside one z-plane: it holds the plane in LDS (up to 128 x 129 values,
// 160 KB per workgroup on gfx950) and applies the four W / W^T passes, the
// pointwise stage (density rho += f psi^2 in float64, e_pot, y = V psi) and the
// two in-plane kinetic passes, so a plane crosses HBM once in and twice out
// (t, kxy) instead of once per 1D pass.
//
// Every work item computes U = 4 consecutive outputs of one line, applying
// the filter in chunks of 16 taps from a register window read from LDS.  The
// passes run in place: outputs stay in registers until every thread has read
// its inputs.  One plane buffer (74 KB at 96 x 96 in float64) lets two
// workgroups share a CU, so one workgroup's HBM transfers overlap the other's
// arithmetic.  Rows have an odd pitch (m1 + 1 values) so that the x-passes,
// whose lanes walk down a column of rows, hit distinct banks.  The density of
// a shared potential is accumulated per group of orbitals, in orbital order,
// in a partial array that the group's workgroup owns (no atomics).

#include "wvl_kernels.h"

namespace wvl {

constexpr int kXyThreads = 512;
constexpr int kU = 4;             // outputs per work item
constexpr int kCh = 16;           // taps per chunk
constexpr int kMaxItems = 8;      // work items per thread and pass (m <= 128)

// Work items of a pass: item i = threadIdx.x + it * kXyThreads covers line
// i % mo, outputs [U (i / mo), U (i / mo) + U); (line, segment) are stepped
// incrementally, without a division per item.
struct ItemIter {
  int line, seg, dl, ds, mo;
  __device__ ItemIter(int mo_) : mo(mo_) {
    line = threadIdx.x % mo_;
    seg = threadIdx.x / mo_;
    dl = kXyThreads % mo_;
    ds = kXyThreads / mo_;
  }
  __device__ void next() {
    line += dl;
    seg += ds;
    if (line >= mo) { line -= mo; ++seg; }
  }
};

// One 1D pass of operator OP over the plane in LDS.  AX = 1: along rows (x),
// AX = 2: along columns (y).  Outputs go to `res` (written back by the caller).
template <int OP, int P, int AX, int MI>
__device__ __forceinline__ void plane_conv(typename Prec<P>::V* buf, int m1, int m2, int pitch,
                                           typename Prec<P>::V (&res)[MI][kU],
                                           int& nitems) {
  using T = Prec<P>;
  using V = typename T::V;
  constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI;
  constexpr int NCH = (OHI - OLO + kCh) / kCh;
  constexpr int WMAX = kU + kCh - 1;
  const int mc = AX == 1 ? m1 : m2;          // conv length
  const int mo = AX == 1 ? m2 : m1;          // number of lines
  const int nseg = (mc + kU - 1) / kU;
  const bool onewrap = mc >= WMAX;           // a window wraps at most once
  const int estride = AX == 1 ? 1 : pitch;   // LDS elements between neighbours
  ItemIter itr(mo);
  nitems = 0;
  #pragma unroll
  for (int it = 0; it < MI; ++it) {
    if (itr.seg >= nseg) break;
    nitems = it + 1;
    const int k0 = itr.seg * kU;
    const V* lp = AX == 1 ? buf + itr.line * pitch : buf + itr.line;
    typename T::Acc acc[kU];
    #pragma unroll
    for (int u = 0; u < kU; ++u) acc[u] = T::zero();
    #pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int olo = OLO + ch * kCh;
      const int ohi = (OLO + ch * kCh + kCh - 1) < OHI ? (OLO + ch * kCh + kCh - 1) : OHI;
      // window: win[w] = x[k0 - ohi + w], w < kU + ohi - olo
      V win[WMAX];
      const int s0 = wrapi(k0 - ohi, mc);
      #pragma unroll
      for (int w = 0; w < WMAX; ++w) {
        if (w < kU + ohi - olo) {
          int idx = s0 + w;
          if (onewrap) idx = idx >= mc ? idx - mc : idx;
          else idx = wrapi(idx, mc);
          win[w] = lp[idx * estride];
        }
      }
      #pragma unroll
      for (int u = 0; u < kU; ++u) {
        #pragma unroll
        for (int oo = 0; oo < kCh; ++oo) {
          const int o = OLO + ch * kCh + oo;
          if (o <= OHI && coef<OP>(u & 1, o, 0) != 0.0)
            T::template add<OP>(acc[u], u & 1, o, win[u + ohi - o]);
        }
      }
      // keep one window live at a time (the scheduler would otherwise hoist
      // the next chunk's loads and run out of registers)
      __builtin_amdgcn_sched_barrier(0);
    }
    #pragma unroll
    for (int u = 0; u < kU; ++u) res[it][u] = T::fin(acc[u]);
    __builtin_amdgcn_sched_barrier(0);
    itr.next();
  }
}

// write back the results of plane_conv (same mapping), skipping k >= mc
template <int P, int AX, int MI>
__device__ __forceinline__ void plane_store(typename Prec<P>::V* buf, int m1, int m2, int pitch,
                                            const typename Prec<P>::V (&res)[MI][kU],
                                            int nitems, bool add) {
  using T = Prec<P>;
  const int mc = AX == 1 ? m1 : m2;
  const int mo = AX == 1 ? m2 : m1;
  ItemIter itr(mo);
  #pragma unroll
  for (int it = 0; it < MI; ++it) {
    if (it >= nitems) break;
    #pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = itr.seg * kU + u;
      if (k < mc) {
        const int pos = AX == 1 ? itr.line * pitch + k : k * pitch + itr.line;
        buf[pos] = add ? T::plus(buf[pos], res[it][u]) : res[it][u];
      }
    }
    itr.next();
  }
}

template <int OP, int P, int AX, int MI>
__device__ __forceinline__ void plane_pass(typename Prec<P>::V* buf, int m1, int m2, int pitch) {
  typename Prec<P>::V res[MI][kU];
  int n = 0;
  plane_conv<OP, P, AX, MI>(buf, m1, m2, pitch, res, n);
  __syncthreads();
  plane_store<P, AX, MI>(buf, m1, m2, pitch, res, n, false);
  __syncthreads();
}

// sum over the plane of x * scale * y for the kinetic energy: x from LDS at the
// output positions of the item mapping (before they are overwritten)
template <int P, int AX, int MI>
__device__ __forceinline__ double plane_dot(const typename Prec<P>::V* buf, int m1, int m2,
                                            int pitch, const typename Prec<P>::V (&res)[MI][kU],
                                            int nitems) {
  using T = Prec<P>;
  const int mc = AX == 1 ? m1 : m2;
  const int mo = AX == 1 ? m2 : m1;
  double e = 0.0;
  ItemIter itr(mo);
  #pragma unroll
  for (int it = 0; it < MI; ++it) {
    if (it >= nitems) break;
    #pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = itr.seg * kU + u;
      if (k < mc) {
        const int pos = AX == 1 ? itr.line * pitch + k : k * pitch + itr.line;
        e += T::d(buf[pos]) * T::d(res[it][u]);
      }
    }
    itr.next();
  }
  return e;
}

// Points of the plane owned by this thread: e = threadIdx.x + k * kXyThreads,
// with its LDS position y * pitch + x stepped incrementally.
struct PtIter {
  int e, x, y, dx, dy, m1;
  __device__ PtIter(int m1_) : m1(m1_) {
    e = threadIdx.x;
    x = threadIdx.x % m1_;
    y = threadIdx.x / m1_;
    dx = kXyThreads % m1_;
    dy = kXyThreads / m1_;
  }
  __device__ int pos(int pitch) const { return y * pitch + x; }
  __device__ void next() {
    e += kXyThreads;
    x += dx;
    y += dy;
    if (x >= m1) { x -= m1; ++y; }
  }
};

__device__ __forceinline__ double xy_block_sum(double v) {
  __shared__ double red[kXyThreads / 64];
  #pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  #pragma unroll
  for (int w = 0; w < kXyThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Grid: shared-potential batches (SHARED): blockIdx.x = z * ngroups + g
// (orbitals g*G .. g*G+G-1), the group's density accumulated in LDS after the
// plane; otherwise one (orbital, plane) per block via the plane prefix pq.
// Slot of (b, z) in the per-plane energy arrays: pq[b] + z.  MI: work items
// per thread and pass (planes up to 96 x 96: 3, up to 128 x 128: 4).
// One (orbital, plane): everything the kernel does for orbital b at plane z.
template <int P, int MI, bool SHARED>
__device__ __forceinline__ void xy_orbital_plane(const XyArgs& a, int b, int z, int g,
                                                           int bi) {
  using T = Prec<P>;
  using V = typename T::V;
  extern __shared__ __align__(16) unsigned char xy_lds[];
  V* buf = reinterpret_cast<V*>(xy_lds);
    // every orbital of a group has the same plane; taking the sizes from the
    // orbital's own descriptor keeps the index arithmetic inside the loop
    const OrbDev od = a.orbs[b];
    const int m1 = od.m[0], m2 = od.m[1];
    const int pitch = m1 + 1;
    const int npl = m1 * m2;
    const double ks1 = od.kscale[0], ks2 = od.kscale[1];
    const int64_t gp = od.off + (int64_t)z * npl;     // plane start in the batch buffers
    // ---- psi = W_x W_y u
    for (PtIter q(m1); q.e < npl; q.next()) buf[q.pos(pitch)] = T::ldc(a.u, gp + q.e, a.plane);
    __syncthreads();
    plane_pass<OP_CW, P, 2, MI>(buf, m1, m2, pitch);
    plane_pass<OP_CW, P, 1, MI>(buf, m1, m2, pitch);
    // ---- pointwise stage: rho (group partial, fixed orbital order), e_pot,
    //      y = pot_scale V psi
    double ep = 0.0;
    const double* Vp = a.V + od.voff + (int64_t)z * npl;
    double* rp = SHARED ? a.rho_part + (int64_t)g * a.M + (int64_t)z * npl : nullptr;
    for (PtIter q(m1); q.e < npl; q.next()) {
      const int pos = q.pos(pitch), e = q.e;
      const V psi = buf[pos];
      const double pd = T::d(psi);
      const double v = Vp[e];
      if (SHARED && rp) rp[e] = bi == 0 ? od.occ * pd * pd : __builtin_fma(od.occ * pd, pd, rp[e]);
      ep = __builtin_fma(v * pd, pd, ep);
      buf[pos] = T::scale(psi, v * a.pot_scale);
    }
    __syncthreads();
    // ---- t = W_y^T W_x^T y
    plane_pass<OP_CWT, P, 1, MI>(buf, m1, m2, pitch);
    plane_pass<OP_CWT, P, 2, MI>(buf, m1, m2, pitch);
    for (PtIter q(m1); q.e < npl; q.next()) T::st(a.t, gp + q.e, a.plane, buf[q.pos(pitch)]);
    __syncthreads();
    // ---- kxy = (K_x + K_y) c, and <c, (K_x + K_y) c> for the kinetic energy:
    //      K_y c goes straight to kxy (lanes along x: coalesced), K_x c through
    //      LDS once c is no longer needed, then kxy += the LDS plane
    for (PtIter q(m1); q.e < npl; q.next()) buf[q.pos(pitch)] = T::ldc(a.c, gp + q.e, a.plane);
    __syncthreads();
    double ek = 0.0;
    {
      V r[MI][kU];
      int n = 0;
      plane_conv<OP_CK, P, 2, MI>(buf, m1, m2, pitch, r, n);
      #pragma unroll
      for (int it = 0; it < MI; ++it)
        #pragma unroll
        for (int u = 0; u < kU; ++u) r[it][u] = T::scale(r[it][u], ks2);
      ek += plane_dot<P, 2, MI>(buf, m1, m2, pitch, r, n);
      ItemIter itr(m1);
      #pragma unroll
      for (int it = 0; it < MI; ++it) {
        if (it >= n) break;
        #pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int y = itr.seg * kU + u;
          if (y < m2) {
            const V val = a.kin_mul != 1.0 ? T::scale(r[it][u], a.kin_mul) : r[it][u];
            T::st(a.kxy, gp + (int64_t)y * m1 + itr.line, a.plane, val);
          }
        }
        itr.next();
      }
    }
    {
      V r[MI][kU];
      int n = 0;
      plane_conv<OP_CK, P, 1, MI>(buf, m1, m2, pitch, r, n);
      #pragma unroll
      for (int it = 0; it < MI; ++it)
        #pragma unroll
        for (int u = 0; u < kU; ++u) r[it][u] = T::scale(r[it][u], ks1);
      ek += plane_dot<P, 1, MI>(buf, m1, m2, pitch, r, n);
      if (a.kin_mul != 1.0) {
        #pragma unroll
        for (int it = 0; it < MI; ++it)
          #pragma unroll
          for (int u = 0; u < kU; ++u) r[it][u] = T::scale(r[it][u], a.kin_mul);
      }
      __syncthreads();
      plane_store<P, 1, MI>(buf, m1, m2, pitch, r, n, false);
    }
    __syncthreads();
    for (PtIter q(m1); q.e < npl; q.next()) {
      const V kx = buf[q.pos(pitch)];
      T::st(a.kxy, gp + q.e, a.plane, T::plus(T::ldc(a.kxy, gp + q.e, a.plane), kx));
    }
    // ---- per-(orbital, plane) energies (the block sums end with a barrier)
    const double sp = xy_block_sum(ep);
    const double sk = xy_block_sum(ek);
    if (threadIdx.x == 0) {
      a.epot[a.pq[b] + z] = sp;
      a.ekin[a.pq[b] + z] = sk;
    }
}

// Grid: shared-potential batches (SHARED): blockIdx.x = z * ngroups + g and
// the orbital is g * G + slot (one launch per slot, in slot order, so the
// group's density partial is accumulated in orbital order); otherwise one
// (orbital, plane) per block via the plane prefix pq.
template <int P, int MI, bool SHARED, int WPE>
__global__ __launch_bounds__(kXyThreads) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_xy(XyArgs a) {
  int b, z, g = 0;
  if (SHARED) {
    g = blockIdx.x % a.ngroups;
    z = blockIdx.x / a.ngroups;
    b = g * a.G + a.slot;
    if (b >= a.norb) return;
  } else {
    find_tile(a.pq, a.norb, blockIdx.x, b, z);
  }
  xy_orbital_plane<P, MI, SHARED>(a, b, z, g, a.slot);
}

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

size_t xy_lds_bytes(int prec, int m1, int m2, bool shared) {
  (void)shared;
  return (size_t)m2 * (m1 + 1) * (prec == F32 ? 4 : 8);
}

bool xy_supported(int prec, int m1, int m2, bool shared) {
  return xy_items(m1, m2) <= kMaxItems && xy_lds_bytes(prec, m1, m2, shared) <= 160 * 1024;
}

template <int P, bool SH, int WPE>
static void xy_launch_w(const XyArgs& a, int mi, int nblocks, size_t lds, hipStream_t st) {
  const dim3 g(nblocks), b(kXyThreads);
  if (mi <= 3) hipLaunchKernelGGL((k_xy<P, 3, SH, WPE>), g, b, lds, st, a);
  else if (mi <= 5) hipLaunchKernelGGL((k_xy<P, 5, SH, WPE>), g, b, lds, st, a);
  else hipLaunchKernelGGL((k_xy<P, 8, SH, WPE>), g, b, lds, st, a);
}

template <int P, bool SH>
static void xy_launch_p(const XyArgs& a, int mi, int nblocks, size_t lds, hipStream_t st) {
  // occupancy target: 4 waves per SIMD (two workgroups per CU, <= 128
  // registers) or 2 (one workgroup per CU, <= 256 registers)
  if (a.occupancy == 2) xy_launch_w<P, SH, 2>(a, mi, nblocks, lds, st);
  else xy_launch_w<P, SH, 4>(a, mi, nblocks, lds, st);
}

hipError_t launch_xy(int prec, const XyArgs& a, int m1, int m2, int nblocks, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  const int mi = xy_items(m1, m2);
  const bool sh = a.shared != 0;
  const size_t lds = xy_lds_bytes(prec, m1, m2, sh);
  switch (prec) {
    case F64: sh ? xy_launch_p<F64, true>(a, mi, nblocks, lds, st) : xy_launch_p<F64, false>(a, mi, nblocks, lds, st); break;
    case F32: sh ? xy_launch_p<F32, true>(a, mi, nblocks, lds, st) : xy_launch_p<F32, false>(a, mi, nblocks, lds, st); break;
    default:  sh ? xy_launch_p<F32C, true>(a, mi, nblocks, lds, st) : xy_launch_p<F32C, false>(a, mi, nblocks, lds, st); break;
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
