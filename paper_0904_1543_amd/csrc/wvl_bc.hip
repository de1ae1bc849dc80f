// 1D passes with isolated (free) or periodic boundary conditions on arrays
// whose length along the pass changes, gfx950.
//
// Sec. 3.1: the boundary conditions decide the values the convolutions see
// outside the box.  Along an isolated axis nothing is outside (zero), and
// each operator writes the whole range its result occupies: the combined
// synthesis + magic filter maps the m interleaved coefficients onto m + 29
// real-space points (global positions -14 .. m + 14), its transpose maps them
// back, and the combined kinetic filter maps m coefficients onto m.  With the
// global position of output k equal to k + d plus that of input 0 (d = -14,
// +14 or 0), a pass computes
//     y[k] = sum_o F_{k mod 2}(o) x[k + d - o]      (x = 0 outside [0, n_in))
// and, along a periodic axis (d = 0, n_in = n_out), x wraps.  The polyphase
// parity is that of the output's global position, which has the parity of k
// because every global offset here is even.
// Strided axes (2, 3): one line per lane, consecutive lanes on consecutive
// lines (coalesced), a register window sliding by two outputs.  Axis 1: a
// tile of rows staged in LDS with the zero or periodic margin already in
// place, then the same window read from LDS.

#include <algorithm>

#include "wvl_internal.h"
#include "wvl_kernels.h"

namespace wvl {

template <int P, int OP>
__device__ __forceinline__ void bc_pair(const typename Prec<P>::V* win, typename Prec<P>::V& y0,
                                        typename Prec<P>::V& y1) {
  using T = Prec<P>;
  constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI;
  typename T::Acc a0 = T::zero(), a1 = T::zero();
  #pragma unroll
  for (int o = OLO; o <= OHI; ++o) {
    if (coef<OP>(0, o, 0) != 0.0) T::template add<OP>(a0, 0, o, win[OHI - o]);
    if (coef<OP>(1, o, 0) != 0.0) T::template add<OP>(a1, 1, o, win[OHI - o + 1]);
  }
  y0 = T::fin(a0);
  y1 = T::fin(a1);
}

template <int P>
__device__ __forceinline__ typename Prec<P>::V bc_load(const void* in, int64_t base, int64_t stride,
                                                       int pos, int n, bool periodic,
                                                       int64_t plane) {
  using T = Prec<P>;
  if (periodic) return T::ldc(in, base + (int64_t)wrapi(pos, n) * stride, plane);
  if (pos < 0 || pos >= n) return T::from_d(0.0);
  return T::ldc(in, base + (int64_t)pos * stride, plane);
}

// Strided pass (AXIS 2 or 3): tile t covers lines [256 t', 256 t' + 256) of
// orbital b (tiles of one orbital are consecutive).
template <int OP, int P, int AXIS, bool K0, bool EN>
__global__ __launch_bounds__(kThreads) void k_bc_strided(BcPass g, const void* __restrict__ in,
                                                         void* out, const void* k0,
                                                         int64_t plane_in, int64_t plane_out,
                                                         double kmul, double* __restrict__ epart) {
  using T = Prec<P>;
  using V = typename T::V;
  constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI, W = OHI - OLO + 1;
  const int b = blockIdx.x / g.tiles;
  const int t = blockIdx.x - b * g.tiles;
  // lines: AXIS 3 -> (y, x) of an (n2, n1) plane; AXIS 2 -> (z, x)
  const int64_t nl = AXIS == 3 ? (int64_t)g.n2 * g.n1 : (int64_t)g.n3 * g.n1;
  const int64_t line = (int64_t)t * kThreads + threadIdx.x;
  double e = 0.0;
  if (line < nl) {
    int64_t bin, bout, sin, sout;
    if (AXIS == 3) {
      sin = sout = (int64_t)g.n2 * g.n1;
      bin = (int64_t)b * g.vol_in + line;
      bout = (int64_t)b * g.vol_out + line;
    } else {
      const int64_t z = line / g.n1, x = line - z * g.n1;
      sin = sout = g.n1;
      bin = (int64_t)b * g.vol_in + z * ((int64_t)g.n_in * g.n1) + x;
      bout = (int64_t)b * g.vol_out + z * ((int64_t)g.n_out * g.n1) + x;
    }
    const double ks = g.orbs[b].kscale[AXIS - 1];
    V win[W + 1];
    #pragma unroll
    for (int i = 0; i < W - 1; ++i)
      win[i] = bc_load<P>(in, bin, sin, g.d - OHI + i, g.n_in, g.periodic, plane_in);
    for (int k = 0; k < g.n_out; k += 2) {
      win[W - 1] = bc_load<P>(in, bin, sin, k + g.d - OLO, g.n_in, g.periodic, plane_in);
      win[W] = bc_load<P>(in, bin, sin, k + 1 + g.d - OLO, g.n_in, g.periodic, plane_in);
      V y0, y1;
      bc_pair<P, OP>(win, y0, y1);
      if (OP == OP_CK || OP == OP_KIN) {
        y0 = T::scale(y0, ks);
        y1 = T::scale(y1, ks);
        if (EN) {   // in_len = out_len, d = 0: win[OHI] is the input at k
          e += T::d(win[OHI]) * T::d(y0);
          if (k + 1 < g.n_out) e += T::d(win[OHI + 1]) * T::d(y1);
        }
        if (kmul != 1.0) { y0 = T::scale(y0, kmul); y1 = T::scale(y1, kmul); }
      }
      const int64_t i0 = bout + (int64_t)k * sout;
      if (K0) y0 = T::plus(y0, T::ldc(k0, i0, g.plane_k0));
      T::st(out, i0, plane_out, y0);
      if (k + 1 < g.n_out) {
        if (K0) y1 = T::plus(y1, T::ldc(k0, i0 + sout, g.plane_k0));
        T::st(out, i0 + sout, plane_out, y1);
      }
      #pragma unroll
      for (int i = 0; i < W - 1; ++i) win[i] = win[i + 2];
    }
  }
  if (EN) block_sum_store(e, epart + blockIdx.x);
}

// Axis-1 pass: tile t covers rows [R t', R t' + R) of orbital b (rows: the
// (z, y) pairs of the array); row r of the tile is staged at lds[r * pitch]
// from input position d - OHI on, so the pair (k, k + 1) reads lds[k ..].
template <int OP, int P, bool K0, bool EN>
__global__ __launch_bounds__(kThreads) void k_bc_contig(BcPass g, const void* in, void* out,
                                                        const void* k0, int64_t plane_in,
                                                        int64_t plane_out, double kmul,
                                                        double* __restrict__ epart) {
  using T = Prec<P>;
  using V = typename T::V;
  constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI, W = OHI - OLO + 1;
  __shared__ V lds[kContigLds];
  const int b = blockIdx.x / g.tiles;
  const int t = blockIdx.x - b * g.tiles;
  const int rows = g.n2 * g.n3;
  const int pitch = g.n_out + W + 1;
  const int R = g.rows_per_tile;
  const int row0 = t * R;
  const int nrows = min(R, rows - row0);
  const int64_t gin = (int64_t)b * g.vol_in + (int64_t)row0 * g.n_in;
  const int64_t gout = (int64_t)b * g.vol_out + (int64_t)row0 * g.n_out;
  const int nload = nrows * pitch;
  for (int q = threadIdx.x; q < nload; q += kThreads) {
    const int r = q / pitch;
    const int pos = q - r * pitch + g.d - OHI;
    lds[q] = bc_load<P>(in, gin + (int64_t)r * g.n_in, 1, pos, g.n_in, g.periodic, plane_in);
  }
  __syncthreads();
  const double ks = g.orbs[b].kscale[0];
  const int half = (g.n_out + 1) >> 1;
  const int npairs = nrows * half;
  double en = 0.0;
  for (int q = threadIdx.x; q < npairs; q += kThreads) {
    const int r = q / half;
    const int k = 2 * (q - r * half);
    const V* src = lds + r * pitch + k;
    V win[W + 1];
    #pragma unroll
    for (int i = 0; i <= W; ++i) win[i] = src[i];
    V y0, y1;
    bc_pair<P, OP>(win, y0, y1);
    if (OP == OP_CK || OP == OP_KIN) {
      y0 = T::scale(y0, ks);
      y1 = T::scale(y1, ks);
      if (EN) {
        en += T::d(win[OHI]) * T::d(y0);
        if (k + 1 < g.n_out) en += T::d(win[OHI + 1]) * T::d(y1);
      }
      if (kmul != 1.0) { y0 = T::scale(y0, kmul); y1 = T::scale(y1, kmul); }
    }
    const int64_t i0 = gout + (int64_t)r * g.n_out + k;
    if (K0) y0 = T::plus(y0, T::ldc(k0, i0, g.plane_k0));
    T::st(out, i0, plane_out, y0);
    if (k + 1 < g.n_out) {
      if (K0) y1 = T::plus(y1, T::ldc(k0, i0 + 1, g.plane_k0));
      T::st(out, i0 + 1, plane_out, y1);
    }
  }
  if (EN) block_sum_store(en, epart + blockIdx.x);
}

template <int OP, int P>
static hipError_t bc_axis(int axis, const BcPass& g, const void* in, void* out, const void* k0,
                          int64_t plane_in, int64_t plane_out, double kmul, double* epart,
                          hipStream_t st) {
  const bool en = epart != nullptr;
  const dim3 grid(g.tiles * g.orbs_n), block(kThreads);
  if (grid.x == 0) return hipSuccess;
#define WVL_L(KERN) hipLaunchKernelGGL((KERN), grid, block, 0, st, g, in, out, k0, plane_in, plane_out, kmul, epart)
  if (axis == 1) {
    if (k0) { if (en) WVL_L((k_bc_contig<OP, P, true, true>)); else WVL_L((k_bc_contig<OP, P, true, false>)); }
    else    { if (en) WVL_L((k_bc_contig<OP, P, false, true>)); else WVL_L((k_bc_contig<OP, P, false, false>)); }
  } else if (axis == 2) {
    if (k0) { if (en) WVL_L((k_bc_strided<OP, P, 2, true, true>)); else WVL_L((k_bc_strided<OP, P, 2, true, false>)); }
    else    { if (en) WVL_L((k_bc_strided<OP, P, 2, false, true>)); else WVL_L((k_bc_strided<OP, P, 2, false, false>)); }
  } else {
    if (k0) { if (en) WVL_L((k_bc_strided<OP, P, 3, true, true>)); else WVL_L((k_bc_strided<OP, P, 3, true, false>)); }
    else    { if (en) WVL_L((k_bc_strided<OP, P, 3, false, true>)); else WVL_L((k_bc_strided<OP, P, 3, false, false>)); }
  }
#undef WVL_L
  return hipGetLastError();
}

template <int P>
static hipError_t bc_op(int op, int axis, const BcPass& g, const void* in, void* out,
                        const void* k0, int64_t plane_in, int64_t plane_out, double kmul,
                        double* epart, hipStream_t st) {
  switch (op) {
    case OP_CW:  return bc_axis<OP_CW, P>(axis, g, in, out, k0, plane_in, plane_out, kmul, epart, st);
    case OP_CWT: return bc_axis<OP_CWT, P>(axis, g, in, out, k0, plane_in, plane_out, kmul, epart, st);
    case OP_CK:  return bc_axis<OP_CK, P>(axis, g, in, out, k0, plane_in, plane_out, kmul, epart, st);
    default:     return hipErrorInvalidValue;
  }
}

int bc_rows_per_tile(int op, int n_out) {
  const int W = op == OP_CW ? OpWin<OP_CW>::OHI - OpWin<OP_CW>::OLO + 1
              : op == OP_CWT ? OpWin<OP_CWT>::OHI - OpWin<OP_CWT>::OLO + 1
                             : OpWin<OP_CK>::OHI - OpWin<OP_CK>::OLO + 1;
  const int r = kContigLds / (n_out + W + 1);
  return r < 1 ? 1 : r;
}

hipError_t launch_bc_pass(int prec, int op, int axis, const BcPass& g, const void* in, void* out,
                          const void* k0, int64_t plane_in, int64_t plane_out, double kmul,
                          double* epart, hipStream_t st) {
  switch (prec) {
    case F64: return bc_op<F64>(op, axis, g, in, out, k0, plane_in, plane_out, kmul, epart, st);
    case F32: return bc_op<F32>(op, axis, g, in, out, k0, plane_in, plane_out, kmul, epart, st);
    default:  return bc_op<F32C>(op, axis, g, in, out, k0, plane_in, plane_out, kmul, epart, st);
  }
}

}  // namespace wvl
