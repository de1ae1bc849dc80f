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
//
// Device code of the in-plane kernel (templates); wvl_xy.hip holds the host
// dispatch, and each wvl_xy_<form>.hip instantiates one precision/engine so
// that the instantiations compile in parallel.
#pragma once

#include "wvl_plane.h"

namespace wvl {

constexpr int kCh = 16;           // taps per chunk

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
      // window: win[w] = x[k0 - ohi + w], w < kU + ohi - olo.  Away from the
      // ends of the line the window is contiguous (constant offsets from one
      // base); near them it wraps, stepped one index at a time.
      const int len = kU + ohi - olo;
      V win[WMAX];
      int s0 = k0 - ohi;
      if (s0 >= 0 && s0 + len <= mc) {
        const V* p = lp + s0 * estride;
        #pragma unroll
        for (int w = 0; w < WMAX; ++w)
          if (w < len) win[w] = p[w * estride];
      } else {
        while (s0 < 0) s0 += mc;
        while (s0 >= mc) s0 -= mc;
        int off = s0 * estride;
        const int end = mc * estride;
        #pragma unroll
        for (int w = 0; w < WMAX; ++w) {
          if (w < len) {
            win[w] = lp[off];
            off += estride;
            off = off == end ? 0 : off;
          }
        }
      }
      // taps outer, outputs inner: kU independent accumulation chains
      #pragma unroll
      for (int oo = 0; oo < kCh; ++oo) {
        const int o = OLO + ch * kCh + oo;
        #pragma unroll
        for (int u = 0; u < kU; ++u) {
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

// ---------------------------------------------------------------------------
// Engines: how one 1D pass over the plane in LDS is computed.  conv<OP, AX>
// leaves the pass's outputs in registers (Res); store writes them back in
// place (after a barrier: every input must have been read first), dot sums
// x * result over the output positions (x: the pass's input there), and
// store_global_y writes the results of an AX = 2 pass to a plane in memory.

// Vector FMA engine (every precision): work items of U outputs of one line.
template <int P, int MI>
struct VecEngine {
  using T = Prec<P>;
  using V = typename T::V;
  struct Res { V r[MI][kU]; int n; };
  static constexpr bool kGroupLoop = false;   // one launch per slot
  static constexpr bool kFusedK = false;      // in-plane kinetic passes through memory
  __device__ __forceinline__ static int pitch(int m1) { return m1 + 1; }
  template <int OP, int AX>
  __device__ __forceinline__ static void conv(V* buf, int m1, int m2, int pitch, Res& r) {
    plane_conv<OP, P, AX, MI>(buf, m1, m2, pitch, r.r, r.n);
  }
  template <int AX>
  __device__ __forceinline__ static void store(V* buf, int m1, int m2, int pitch, const Res& r) {
    plane_store<P, AX, MI>(buf, m1, m2, pitch, r.r, r.n, false);
  }
  template <int AX>
  __device__ __forceinline__ static double dot(const V* buf, int m1, int m2, int pitch, const Res& r) {
    return plane_dot<P, AX, MI>(buf, m1, m2, pitch, r.r, r.n);
  }
  __device__ __forceinline__ static void scale(Res& r, double s) {
    #pragma unroll
    for (int it = 0; it < MI; ++it)
      #pragma unroll
      for (int u = 0; u < kU; ++u) r.r[it][u] = T::scale(r.r[it][u], s);
  }
  __device__ __forceinline__ static void store_global_y(void* dst, int64_t gp, int64_t plane, int m1, int m2,
                                        const Res& r) {
    ItemIter itr(m1);
    #pragma unroll
    for (int it = 0; it < MI; ++it) {
      if (it >= r.n) break;
      #pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int y = itr.seg * kU + u;
        if (y < m2) T::st(dst, gp + (int64_t)y * m1 + itr.line, plane, r.r[it][u]);
      }
      itr.next();
    }
  }
  // dst += the results of an AX = 2 pass
  __device__ __forceinline__ static void add_global_y(void* dst, int64_t gp, int64_t plane, int m1,
                                                      int m2, const Res& r) {
    ItemIter itr(m1);
    #pragma unroll
    for (int it = 0; it < MI; ++it) {
      if (it >= r.n) break;
      #pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int y = itr.seg * kU + u;
        if (y < m2) {
          const int64_t i = gp + (int64_t)y * m1 + itr.line;
          T::st(dst, i, plane, T::plus(T::ldc(dst, i, plane), r.r[it][u]));
        }
      }
      itr.next();
    }
  }
};

// Matrix-core engine (float64): a pass is a product with a banded circulant
// matrix, F[k][j] = F_{k mod 2}(k - j) (mod m), applied to the plane from the
// left (y) or the right (x).  It is cut into 16 x 16 output tiles; a tile
// needs 16 + OHI - OLO inputs along the pass, i.e. S steps of the
// 16 x 16 x 4 float64 matrix instruction, whose filter operand is the same
// for every tile (k0 is a multiple of 16, so the output parity is that of the
// row in the tile).  For step s, lane l = n + 16 kk holds F at tap
// o = n - kk + OHI - 4 s (zero outside the window): as the B operand of an
// x-pass (B[kk][n]) and as the A operand of a y-pass (A[n][kk]).
typedef double d4 __attribute__((ext_vector_type(4)));

template <int OP>
struct Frag {
  static constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI;
  static constexpr int S = (16 + OHI - OLO + 3) / 4;
  double v[S][64];
  constexpr Frag() : v() {
    for (int s = 0; s < S; ++s)
      for (int l = 0; l < 64; ++l) {
        const int n = l & 15, kk = l >> 4;
        v[s][l] = coef<OP>(n & 1, n - kk + OHI - 4 * s, 0);
      }
  }
};
static __device__ const Frag<OP_CW> kFragCW = Frag<OP_CW>();
static __device__ const Frag<OP_CWT> kFragCWT = Frag<OP_CWT>();
static __device__ const Frag<OP_CK> kFragCK = Frag<OP_CK>();
template <int OP> __device__ __forceinline__ const double* frag_tab() {
  return OP == OP_CW ? &kFragCW.v[0][0] : OP == OP_CWT ? &kFragCWT.v[0][0] : &kFragCK.v[0][0];
}


template <int MT>
struct MfEngine {
  using T = Prec<F64>;
  using V = double;
  struct Res { d4 r[MT]; int n; };
  static constexpr bool kGroupLoop = true;    // a group's orbitals in one workgroup
  // (K_x + K_y) c summed in the accumulators: both passes enumerate their
  // tiles by (y block, x block), so a lane holds the same plane element in
  // the y-pass and the x-pass result (element (i, n) of a tile: y offset i,
  // x offset n in both), and the x pass starts from the y pass's sums
  static constexpr bool kFusedK = true;
  // rows of 4 (mod 32) doubles: the x-pass operand (16 rows x 4 columns) and
  // the tile stores fall on distinct banks
  __device__ __forceinline__ static int pitch(int m1) { return m1 + ((36 - (m1 & 31)) & 31); }
  // The tiles of this wave, tile = wave + t kXyWaves = a n + b, stepped
  // without a division per tile; the wave index is uniform, so this is
  // scalar work.  Order (a, b) = (output block k0 along the pass, line block
  // o0) with n = line blocks, or (y block, x block) with n = x blocks.
  struct Walk {
    int a, b, n, da, db;
    __device__ __forceinline__ explicit Walk(int n_) : n(n_) {
      const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
      a = wv / n;
      b = wv - a * n;
      da = kXyWaves / n;
      db = kXyWaves - da * n;
    }
    __device__ __forceinline__ void next() {
      b += db;
      a += da;
      if (b >= n) { b -= n; ++a; }
    }
  };
  __device__ __forceinline__ static int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  }
  // One pass.  YX: tiles in (y block, x block) order; ACC: accumulate onto
  // r (the other pass's sums of the same elements); fscale multiplies the
  // filter (the kinetic factor -1/(2 h^2) of the pass's axis).
  template <int OP, int AX, bool YX = false, bool ACC = false>
  __device__ __forceinline__ static void conv(V* buf, int m1, int m2, int pitch, Res& r,
                                              double fscale = 1.0) {
    constexpr int S = Frag<OP>::S, OHI = Frag<OP>::OHI;
    const int lane = threadIdx.x & 63, li = lane & 15, q = lane >> 4;
    const int mc = AX == 1 ? m1 : m2, mo = AX == 1 ? m2 : m1;
    const int nbo = (mo + 15) >> 4, nt = ((mc + 15) >> 4) * nbo;
    const int es = AX == 1 ? 1 : pitch;
    double fc[S];
    const double* ft = frag_tab<OP>();
    // opaque to the optimiser: the table is re-read per pass instead of being
    // hoisted (and kept live in registers) across a loop over orbitals
    asm volatile("" : "+s"(ft));
    #pragma unroll
    for (int s = 0; s < S; ++s) fc[s] = ft[s * 64 + lane] * fscale;
    if (!ACC) r.n = 0;
    const int wv = wave_id();
    Walk wk(YX ? (m1 + 15) >> 4 : nbo);
    #pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (wv + t * kXyWaves >= nt) break;
      if (!ACC) r.n = t + 1;
      const int k0 = (YX && AX == 1 ? wk.b : wk.a) * 16;
      const int o0 = (YX && AX == 1 ? wk.a : wk.b) * 16;
      wk.next();
      const int line = min(o0 + li, mo - 1);      // rows/columns past the end: unused outputs
      const V* lp = AX == 1 ? buf + line * pitch : buf + line;
      // input index of step s: (k0 - OHI + 4 s + q) mod mc.  The window's
      // start jb is uniform; a window that does not reach the end of the line
      // is read at fixed strides, otherwise with a wrap per step (lines are
      // at least 4 long, so a step wraps at most once)
      int jb = k0 - OHI;
      while (jb < 0) jb += mc;
      double x[S];
      if (jb + 4 * S <= mc) {
        const V* p0 = lp + (jb + q) * es;
        #pragma unroll
        for (int s = 0; s < S; ++s) x[s] = p0[4 * s * es];
      } else {
        int j = jb + q;
        j = j >= mc ? j - mc : j;
        #pragma unroll
        for (int s = 0; s < S; ++s) {
          x[s] = lp[__mul24(j, es)];
          j += 4;
          j = j >= mc ? j - mc : j;
        }
      }
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      if (ACC) acc = r.r[t];
      #pragma unroll
      for (int s = 0; s < S; ++s)
        acc = AX == 1 ? __builtin_amdgcn_mfma_f64_16x16x4f64(x[s], fc[s], acc, 0, 0, 0)
                      : __builtin_amdgcn_mfma_f64_16x16x4f64(fc[s], x[s], acc, 0, 0, 0);
      r.r[t] = acc;
    }
  }
  // output element (i, n) of a tile is in lane n + 16 (i mod 4), register i / 4
  template <int AX, typename F>
  __device__ __forceinline__ static void each(int m1, int m2, const Res& r, F&& f) {
    const int lane = threadIdx.x & 63, li = lane & 15, q = lane >> 4;
    const int mc = AX == 1 ? m1 : m2, mo = AX == 1 ? m2 : m1;
    const int nbo = (mo + 15) >> 4;
    Walk wk(nbo);
    #pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (t >= r.n) break;
      const int k0 = wk.a * 16, o0 = wk.b * 16;
      wk.next();
      #pragma unroll
      for (int v = 0; v < 4; ++v) {
        // x-pass: row o0 + i, column k0 + n;  y-pass: row k0 + i, column o0 + n
        const int i = q + 4 * v;
        const int k = AX == 1 ? k0 + li : k0 + i;
        const int o = AX == 1 ? o0 + i : o0 + li;
        if (k < mc && o < mo) f(AX == 1 ? o : k, AX == 1 ? k : o, r.r[t][v]);
      }
    }
  }
  template <int AX>
  __device__ __forceinline__ static void store(V* buf, int m1, int m2, int pitch, const Res& r) {
    each<AX>(m1, m2, r, [&](int y, int x, double val) { buf[y * pitch + x] = val; });
  }
  template <int AX>
  __device__ __forceinline__ static double dot(const V* buf, int m1, int m2, int pitch, const Res& r) {
    double e = 0.0;
    each<AX>(m1, m2, r, [&](int y, int x, double val) { e += buf[y * pitch + x] * val; });
    return e;
  }
  __device__ __forceinline__ static void scale(Res& r, double s) {
    #pragma unroll
    for (int t = 0; t < MT; ++t) r.r[t] *= s;
  }
  __device__ __forceinline__ static void store_global_y(void* dst, int64_t gp, int64_t plane, int m1, int m2,
                                        const Res& r) {
    each<2>(m1, m2, r, [&](int y, int x, double val) {
      T::st(dst, gp + (int64_t)y * m1 + x, plane, val);
    });
  }
  __device__ __forceinline__ static void add_global_y(void* dst, int64_t gp, int64_t plane, int m1,
                                                      int m2, const Res& r) {
    each<2>(m1, m2, r, [&](int y, int x, double val) {
      const int64_t i = gp + (int64_t)y * m1 + x;
      T::st(dst, i, plane, T::ldc(dst, i, plane) + val);
    });
  }
};

template <typename E, int OP, int AX>
__device__ __forceinline__ void eng_pass(typename E::V* buf, int m1, int m2, int pitch) {
  typename E::Res r;
  E::template conv<OP, AX>(buf, m1, m2, pitch, r);
  __syncthreads();
  E::template store<AX>(buf, m1, m2, pitch, r);
  __syncthreads();
}

// One (orbital, plane): everything the kernel does for orbital b at plane z.
// RL: the group's density plane is kept in LDS after the plane buffer (same
// pitch) across the group's orbitals and written once by k_xy
template <int P, typename E, bool SHARED, bool RL = false>
__device__ __forceinline__ void xy_orbital_plane(const XyArgs& a, int b, int z, int g, int bi) {
  using T = Prec<P>;
  using V = typename T::V;
  extern __shared__ __align__(16) unsigned char xy_lds[];
  V* buf = reinterpret_cast<V*>(xy_lds);
  const OrbDev od = a.orbs[b];
  const int m1 = od.m[0], m2 = od.m[1];
  const int pitch = E::pitch(m1);
  const int npl = m1 * m2;
  const double ks1 = od.kscale[0], ks2 = od.kscale[1];
  const int64_t gp = od.off + (int64_t)z * npl;     // plane start in the batch buffers
  // ---- psi = W_x W_y u
  plane_batched<kPlaneBatch>(m1, npl, pitch, [&](int e) { return T::ldc(a.u, gp + e, a.plane); },
                            [&](int, int pos, V v) { buf[pos] = v; });
  __syncthreads();
  eng_pass<E, OP_CW, 2>(buf, m1, m2, pitch);
  eng_pass<E, OP_CW, 1>(buf, m1, m2, pitch);
  // ---- pointwise stage: rho (group partial, fixed orbital order), e_pot,
  //      y = pot_scale V psi
  double ep = 0.0;
  const double* Vp = a.V + od.voff + (int64_t)z * npl;
  double* rp = SHARED && !RL ? a.rho_part + (int64_t)g * a.M + (int64_t)z * npl : nullptr;
  double* rl = RL ? reinterpret_cast<double*>(buf + m2 * pitch) : nullptr;
  struct VR { double v, r; };
  plane_batched<kPlaneBatch>(
      m1, npl, pitch,
      [&](int e) { return VR{Vp[e], SHARED && rp && bi != 0 ? rp[e] : 0.0}; },
      [&](int e, int pos, VR w) {
        const V psi = buf[pos];
        const double pd = T::d(psi);
        if (RL) rl[pos] = bi == 0 ? od.occ * pd * pd : __builtin_fma(od.occ * pd, pd, rl[pos]);
        else if (SHARED && rp) rp[e] = bi == 0 ? od.occ * pd * pd : __builtin_fma(od.occ * pd, pd, w.r);
        ep = __builtin_fma(w.v * pd, pd, ep);
        buf[pos] = T::scale(psi, w.v * a.pot_scale);
      });
  __syncthreads();
  // ---- t = W_y^T W_x^T y
  eng_pass<E, OP_CWT, 1>(buf, m1, m2, pitch);
  eng_pass<E, OP_CWT, 2>(buf, m1, m2, pitch);
  for (PtIter q(m1); q.e < npl; q.next()) T::st(a.t, gp + q.e, a.plane, buf[q.pos(pitch)]);
  __syncthreads();
  // ---- kxy = (K_x + K_y) c, and <c, (K_x + K_y) c> for the kinetic energy:
  //      K_y c goes straight to kxy, K_x c through LDS once c is no longer
  //      needed, then kxy += the LDS plane
  plane_batched<kPlaneBatch>(m1, npl, pitch, [&](int e) { return T::ldc(a.c, gp + e, a.plane); },
                            [&](int, int pos, V v) { buf[pos] = v; });
  __syncthreads();
  double ek = 0.0;
  if constexpr (E::kFusedK) {
    // K_y c then K_x c accumulated onto it, the axis factors folded into the
    // filters; one dot for the energy, one store of kxy, c never leaves LDS
    typename E::Res r;
    E::template conv<OP_CK, 2, true, false>(buf, m1, m2, pitch, r, ks2);
    E::template conv<OP_CK, 1, true, true>(buf, m1, m2, pitch, r, ks1);
    ek += E::template dot<2>(buf, m1, m2, pitch, r);
    if (a.kin_mul != 1.0) E::scale(r, a.kin_mul);
    E::store_global_y(a.kxy, gp, a.plane, m1, m2, r);
    __syncthreads();
  } else {
    {
      typename E::Res r;
      E::template conv<OP_CK, 2>(buf, m1, m2, pitch, r);
      E::scale(r, ks2);
      ek += E::template dot<2>(buf, m1, m2, pitch, r);
      if (a.kin_mul != 1.0) E::scale(r, a.kin_mul);
      E::store_global_y(a.kxy, gp, a.plane, m1, m2, r);
    }
    {
      typename E::Res r;
      E::template conv<OP_CK, 1>(buf, m1, m2, pitch, r);
      E::scale(r, ks1);
      ek += E::template dot<1>(buf, m1, m2, pitch, r);
      if (a.kin_mul != 1.0) E::scale(r, a.kin_mul);
      __syncthreads();
      E::template store<1>(buf, m1, m2, pitch, r);
    }
    __syncthreads();
    plane_batched<kPlaneBatch>(m1, npl, pitch, [&](int e) { return T::ldc(a.kxy, gp + e, a.plane); },
                              [&](int e, int pos, V ky) {
                                T::st(a.kxy, gp + e, a.plane, T::plus(ky, buf[pos]));
                              });
  }
  // ---- per-(orbital, plane) energies (the block sums end with a barrier)
  const double sp = xy_block_sum(ep);
  const double sk = xy_block_sum(ek);
  if (threadIdx.x == 0) {
    a.epot[a.pq[b] + z] = sp;
    a.ekin[a.pq[b] + z] = sk;
  }
}

// Grid: shared-potential batches (SHARED): blockIdx.x = z * ngroups + g; the
// orbitals are g * G + slot, either one slot per launch (launches in slot
// order; vector engine) or all slots of the group in one workgroup, in order
// (matrix-core engine, slot = -1); either way the group's density partial is
// accumulated in orbital order.  Otherwise one (orbital, plane) per tile via
// the plane prefix pq.
template <int P, typename E, bool SHARED, int WPE, bool RL = false>
__global__ __launch_bounds__(kXyThreads) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_xy(XyArgs a) {
  if (SHARED) {
    const int g = blockIdx.x % a.ngroups;
    const int z = blockIdx.x / a.ngroups;
    if (!E::kGroupLoop) {
      const int b = g * a.G + a.slot;
      if (b >= a.norb) return;
      xy_orbital_plane<P, E, SHARED>(a, b, z, g, a.slot);
    } else {
      // every orbital of the group in turn: the group's density partial of
      // this plane stays in L2 between them (RL: in LDS, written once)
      #pragma nounroll
      for (int slot = 0; slot < a.G; ++slot) {
        const int b = g * a.G + slot;
        if (b >= a.norb) break;
        xy_orbital_plane<P, E, SHARED, RL>(a, b, z, g, slot);
      }
      if (RL) {
        __syncthreads();
        extern __shared__ __align__(16) unsigned char xy_lds[];
        const int m1 = a.orbs[g * a.G].m[0], m2 = a.orbs[g * a.G].m[1];
        const int pitch = E::pitch(m1), npl = m1 * m2;
        const double* rl = reinterpret_cast<const double*>(xy_lds) + m2 * pitch;
        double* rp = a.rho_part + (int64_t)g * a.M + (int64_t)z * npl;
        for (PtIter q(m1); q.e < npl; q.next()) rp[q.e] = rl[q.pos(pitch)];
      }
    }
  } else {
    const PassGeom geo{a.orbs, a.pq, a.norb, a.order, a.perm, a.queue, a.ntiles, 0};
    for_each_tile(geo, [&](int b, int z, int) { xy_orbital_plane<P, E, SHARED>(a, b, z, 0, 0); });
  }
}

// ---------------------------------------------------------------------------
// In-plane part of the preconditioner's operator (the Helmholtz operator of
// Sec. 2, Eq. "precon", with the wavelet transforms and the kinetic filter
// combined, Sec. 6.1): for one (orbital, z-plane) per workgroup,
//     kq += (K_x + K_y) p        (kq holds K_z p from the z pass)
// with the plane of p in LDS, both in-plane passes of the combined kinetic
// filter, and <p, (K_x + K_y) p> per plane for the CG step length.
// ---------------------------------------------------------------------------
template <int P, typename E, int WPE>
__global__ __launch_bounds__(kXyThreads) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_helm_xy(HelmArgs a) {
  using T = Prec<P>;
  using V = typename T::V;
  extern __shared__ __align__(16) unsigned char xy_lds[];
  V* buf = reinterpret_cast<V*>(xy_lds);
  int b, z;
  find_tile(a.pq, a.norb, blockIdx.x, b, z);
  const OrbDev od = a.orbs[b];
  const int m1 = od.m[0], m2 = od.m[1];
  const int pitch = E::pitch(m1);
  const int npl = m1 * m2;
  const int64_t gp = od.off + (int64_t)z * npl;
  plane_batched<kPlaneBatch>(m1, npl, pitch, [&](int e) { return T::ldc(a.p, gp + e, a.plane); },
                            [&](int, int pos, V v) { buf[pos] = v; });
  __syncthreads();
  double ek = 0.0;
  if constexpr (E::kFusedK) {
    typename E::Res r;
    E::template conv<OP_CK, 2, true, false>(buf, m1, m2, pitch, r, od.kscale[1]);
    E::template conv<OP_CK, 1, true, true>(buf, m1, m2, pitch, r, od.kscale[0]);
    ek += E::template dot<2>(buf, m1, m2, pitch, r);
    E::add_global_y(a.kq, gp, a.plane, m1, m2, r);
  } else {
    {
      typename E::Res r;
      E::template conv<OP_CK, 2>(buf, m1, m2, pitch, r);
      E::scale(r, od.kscale[1]);
      ek += E::template dot<2>(buf, m1, m2, pitch, r);
      E::add_global_y(a.kq, gp, a.plane, m1, m2, r);
    }
    {
      typename E::Res r;
      E::template conv<OP_CK, 1>(buf, m1, m2, pitch, r);
      E::scale(r, od.kscale[0]);
      ek += E::template dot<1>(buf, m1, m2, pitch, r);
      __syncthreads();
      E::template store<1>(buf, m1, m2, pitch, r);
    }
    __syncthreads();
    plane_batched<kPlaneBatch>(m1, npl, pitch, [&](int e) { return T::ldc(a.kq, gp + e, a.plane); },
                              [&](int e, int pos, V k) {
                                T::st(a.kq, gp + e, a.plane, T::plus(k, buf[pos]));
                              });
  }
  const double sk = xy_block_sum(ek);
  if (threadIdx.x == 0) a.ekin[blockIdx.x] = sk;
}

template <int P, typename E>
void helm_launch_e(const HelmArgs& a, int nblocks, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_helm_xy<P, E, 4>), dim3(nblocks), dim3(kXyThreads), lds, st, a);
}

template <int P>
void helm_launch_v(const HelmArgs& a, int mi, int nblocks, size_t lds, hipStream_t st) {
  if (mi <= 3) helm_launch_e<P, VecEngine<P, 3>>(a, nblocks, lds, st);
  else if (mi <= 5) helm_launch_e<P, VecEngine<P, 5>>(a, nblocks, lds, st);
  else helm_launch_e<P, VecEngine<P, 8>>(a, nblocks, lds, st);
}

inline void helm_launch_m(const HelmArgs& a, int mt, int nblocks, size_t lds, hipStream_t st) {
  if (mt <= 2) helm_launch_e<F64, MfEngine<2>>(a, nblocks, lds, st);
  else if (mt <= 5) helm_launch_e<F64, MfEngine<5>>(a, nblocks, lds, st);
  else helm_launch_e<F64, MfEngine<8>>(a, nblocks, lds, st);
}

template <int P, typename E, bool SH>
void xy_launch_e(const XyArgs& a, int nblocks, size_t lds, hipStream_t st) {
  // occupancy target: 4 waves per SIMD (two workgroups per CU, <= 128
  // registers) or 2 (one workgroup per CU, <= 256 registers)
  const dim3 g(nblocks), b(kXyThreads);
  if (a.occupancy == 2 && a.rho_lds)
    hipLaunchKernelGGL((k_xy<P, E, SH, 2, E::kGroupLoop && SH>), g, b, lds, st, a);
  else if (a.occupancy == 2) hipLaunchKernelGGL((k_xy<P, E, SH, 2>), g, b, lds, st, a);
  else hipLaunchKernelGGL((k_xy<P, E, SH, 4>), g, b, lds, st, a);
}

template <int P, bool SH>
void xy_launch_v(const XyArgs& a, int mi, int nblocks, size_t lds, hipStream_t st) {
  if (mi <= 3) xy_launch_e<P, VecEngine<P, 3>, SH>(a, nblocks, lds, st);
  else if (mi <= 5) xy_launch_e<P, VecEngine<P, 5>, SH>(a, nblocks, lds, st);
  else xy_launch_e<P, VecEngine<P, 8>, SH>(a, nblocks, lds, st);
}

template <bool SH>
void xy_launch_m(const XyArgs& a, int mt, int nblocks, size_t lds, hipStream_t st) {
  if (mt <= 2) xy_launch_e<F64, MfEngine<2>, SH>(a, nblocks, lds, st);
  else if (mt <= 5) xy_launch_e<F64, MfEngine<5>, SH>(a, nblocks, lds, st);
  else xy_launch_e<F64, MfEngine<8>, SH>(a, nblocks, lds, st);
}

}  // namespace wvl
