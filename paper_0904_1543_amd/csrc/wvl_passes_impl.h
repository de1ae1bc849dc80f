// 1D periodic convolution passes over a batch of orbitals, gfx950.
//
// The 3D operators of the method are separable: each is three 1D periodic
// convolutions, one along each axis (Sec. 3.1, Eqs. "3dconv", "1dconvtrans";
// the kinetic operator is a sum of three 1D filters, Sec. 3.4, Eq.
// "kinetic1d").  The paper's GPU kernel writes every pass transposed so that
// the next pass again convolves along the slowest axis; here the data stays in
// its natural (m3, m2, m1) layout instead:
//  * passes along axes 2 and 3 (strided axes) give one line to each lane;
//    consecutive lanes own consecutive lines, which are adjacent in memory, so
//    every row of loads and stores is a coalesced 64-lane access, and each lane
//    runs a register sliding window down its line (no LDS needed);
//  * passes along axis 1 (the contiguous axis) stage a block of whole rows in
//    LDS with a periodic halo of 32 values on each side, then every lane
//    computes two neighbouring outputs from a register window read from LDS.
// The periodic boundary (Sec. 3.1) is applied by modular indexing on the
// loads, so lines shorter than the filter are handled as well.

//
// Device code and per-precision launchers (templates); wvl_passes.hip holds
// the dispatch and each wvl_passes_<prec>.hip instantiates one precision.
#pragma once

#include <algorithm>

#include "wvl_internal.h"
#include "wvl_kernels.h"

namespace wvl {

constexpr int kPf = 4;   // output pairs whose loads are in flight (strided passes)

template <int P, int OP>
__device__ __forceinline__ void pair_conv(const typename Prec<P>::V* win, typename Prec<P>::V& y0,
                                          typename Prec<P>::V& y1) {
  using T = Prec<P>;
  constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI;
  typename T::Acc a0 = T::zero(), a1 = T::zero();
  #pragma unroll
  for (int o = OLO; o <= OHI; ++o) {
    // window: win[i] = x[k - OHI + i]; so x[k - o] = win[OHI - o]
    if (coef<OP>(0, o, 0) != 0.0) T::template add<OP>(a0, 0, o, win[OHI - o]);
    if (coef<OP>(1, o, 0) != 0.0) T::template add<OP>(a1, 1, o, win[OHI - o + 1]);
  }
  y0 = T::fin(a0);
  y1 = T::fin(a1);
}

// ---------------------------------------------------------------------------
// Strided-axis pass (AXIS = 2 or 3)
// ---------------------------------------------------------------------------
template <int OP, int P, int AXIS, bool K0, bool EN>
__global__ __launch_bounds__(kThreads) void k_strided(PassGeom g, const void* __restrict__ in,
                                                      void* __restrict__ out, const void* k0,
                                                      int64_t plane, double kmul,
                                                      double* __restrict__ epart) {
  using T = Prec<P>;
  using V = typename T::V;
  constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI, W = OHI - OLO + 1;
  for_each_tile(g, [&](int b, int t, int slot) {
  const OrbDev od = g.orbs[b];
  const int m1 = od.m[0], m2 = od.m[1], m3 = od.m[2];
  const int m = AXIS == 3 ? m3 : m2;
  const int64_t L = AXIS == 3 ? (int64_t)m1 * m2 : (int64_t)m1 * m3;
  const int64_t line = (int64_t)t * kThreads + threadIdx.x;
  double e = 0.0;
  if (line < L) {
    const int64_t stride = AXIS == 3 ? (int64_t)m1 * m2 : (int64_t)m1;
    const int64_t base =
        od.off + (AXIS == 3 ? line : (line / m1) * ((int64_t)m1 * m2) + (line % m1));
    const double ks = AXIS == 3 ? od.kscale[2] : od.kscale[1];
    V win[W + 1];
    #pragma unroll
    for (int i = 0; i < W - 1; ++i) win[i] = T::ldc(in, base + (int64_t)wrapi(i - OHI, m) * stride, plane);
    // The loads of the next kPf output pairs are in flight while a pair is
    // computed (ring of registers, refilled as it is consumed): a wave keeps
    // 2 kPf input loads (and as many accumulator loads) outstanding.
    V q0[kPf], q1[kPf], a0[kPf], a1[kPf];
    #pragma unroll
    for (int d = 0; d < kPf; ++d) {
      const int kk = 2 * d;
      if (kk < m) {
        q0[d] = T::ldc(in, base + (int64_t)wrapi(kk - OLO, m) * stride, plane);
        q1[d] = T::ldc(in, base + (int64_t)wrapi(kk + 1 - OLO, m) * stride, plane);
        if (K0) {
          a0[d] = T::ldc(k0, base + (int64_t)kk * stride, plane);
          a1[d] = T::ldc(k0, base + (int64_t)(kk + 1) * stride, plane);
        }
      }
    }
    for (int k = 0; k < m; k += 2 * kPf) {
      #pragma unroll
      for (int d = 0; d < kPf; ++d) {
        const int kk = k + 2 * d;    // m is even: a pair never straddles the end
        if (kk < m) {
          win[W - 1] = q0[d];
          win[W] = q1[d];
          V c0, c1;
          if (K0) { c0 = a0[d]; c1 = a1[d]; }
          const int kn = kk + 2 * kPf;
          if (kn < m) {
            q0[d] = T::ldc(in, base + (int64_t)wrapi(kn - OLO, m) * stride, plane);
            q1[d] = T::ldc(in, base + (int64_t)wrapi(kn + 1 - OLO, m) * stride, plane);
            if (K0) {
              a0[d] = T::ldc(k0, base + (int64_t)kn * stride, plane);
              a1[d] = T::ldc(k0, base + (int64_t)(kn + 1) * stride, plane);
            }
          }
          V y0, y1;
          pair_conv<P, OP>(win, y0, y1);
          if (OP == OP_KIN || OP == OP_CK) {
            // energies use the unweighted operator; kmul weights the output only
            y0 = T::scale(y0, ks);
            y1 = T::scale(y1, ks);
            if (EN) e += T::d(win[OHI]) * T::d(y0) + T::d(win[OHI + 1]) * T::d(y1);
            if (kmul != 1.0) { y0 = T::scale(y0, kmul); y1 = T::scale(y1, kmul); }
          }
          const int64_t i0 = base + (int64_t)kk * stride, i1 = i0 + stride;
          if (K0) {
            y0 = T::plus(y0, c0);
            y1 = T::plus(y1, c1);
          }
          T::st(out, i0, plane, y0);
          T::st(out, i1, plane, y1);
          #pragma unroll
          for (int i = 0; i < W - 1; ++i) win[i] = win[i + 2];
        }
      }
    }
  }
  if (EN) block_sum_store(e, epart + slot);
  });
}

// ---------------------------------------------------------------------------
// Last step of the plane-resident H*psi, along z, fused:
//     out = W_z^T t + (kmul K_z c + kxy)
// (the two z passes that would otherwise write and re-read kxy), with the
// kinetic energy <c, K_z c> of each tile.  Same association as the two
// separate passes, so the results are the same bit for bit.
// ---------------------------------------------------------------------------
constexpr int kPfZ = 2;   // output pairs in flight (two register windows here)

template <int P, bool EN>
__global__ __launch_bounds__(kThreads) void k_zfinal(PassGeom g, const void* __restrict__ t,
                                                     const void* __restrict__ c, const void* kxy,
                                                     void* __restrict__ out, int64_t plane,
                                                     double kmul, double* __restrict__ epart) {
  using T = Prec<P>;
  using V = typename T::V;
  constexpr int LT = OpWin<OP_CWT>::OLO, HT = OpWin<OP_CWT>::OHI, WT = HT - LT + 1;
  constexpr int LK = OpWin<OP_CK>::OLO, HK = OpWin<OP_CK>::OHI, WK = HK - LK + 1;
  for_each_tile(g, [&](int b, int tl, int slot) {
  const OrbDev od = g.orbs[b];
  const int m1 = od.m[0], m2 = od.m[1], m = od.m[2];
  const int64_t L = (int64_t)m1 * m2;
  const int64_t line = (int64_t)tl * kThreads + threadIdx.x;
  double e = 0.0;
  if (line < L) {
    const int64_t stride = L;
    const int64_t base = od.off + line;
    const double ks = od.kscale[2];
    auto at = [&](int i) { return base + (int64_t)wrapi(i, m) * stride; };
    V wt[WT + 1], wk[WK + 1];
    #pragma unroll
    for (int i = 0; i < WT - 1; ++i) wt[i] = T::ldc(t, at(i - HT), plane);
    #pragma unroll
    for (int i = 0; i < WK - 1; ++i) wk[i] = T::ldc(c, at(i - HK), plane);
    V qt0[kPfZ], qt1[kPfZ], qk0[kPfZ], qk1[kPfZ], a0[kPfZ], a1[kPfZ];
    auto fetch = [&](int d, int kk) {
      qt0[d] = T::ldc(t, at(kk - LT), plane);
      qt1[d] = T::ldc(t, at(kk + 1 - LT), plane);
      qk0[d] = T::ldc(c, at(kk - LK), plane);
      qk1[d] = T::ldc(c, at(kk + 1 - LK), plane);
      a0[d] = T::ldc(kxy, base + (int64_t)kk * stride, plane);
      a1[d] = T::ldc(kxy, base + (int64_t)(kk + 1) * stride, plane);
    };
    #pragma unroll
    for (int d = 0; d < kPfZ; ++d)
      if (2 * d < m) fetch(d, 2 * d);
    for (int k = 0; k < m; k += 2 * kPfZ) {
      #pragma unroll
      for (int d = 0; d < kPfZ; ++d) {
        const int kk = k + 2 * d;    // m is even: a pair never straddles the end
        if (kk < m) {
          wt[WT - 1] = qt0[d];
          wt[WT] = qt1[d];
          wk[WK - 1] = qk0[d];
          wk[WK] = qk1[d];
          const V x0 = a0[d], x1 = a1[d];
          if (kk + 2 * kPfZ < m) fetch(d, kk + 2 * kPfZ);
          V z0, z1, y0, y1;
          pair_conv<P, OP_CK>(wk, z0, z1);
          z0 = T::scale(z0, ks);
          z1 = T::scale(z1, ks);
          if (EN) e += T::d(wk[HK]) * T::d(z0) + T::d(wk[HK + 1]) * T::d(z1);
          if (kmul != 1.0) { z0 = T::scale(z0, kmul); z1 = T::scale(z1, kmul); }
          z0 = T::plus(z0, x0);
          z1 = T::plus(z1, x1);
          pair_conv<P, OP_CWT>(wt, y0, y1);
          const int64_t i0 = base + (int64_t)kk * stride;
          T::st(out, i0, plane, T::plus(y0, z0));
          T::st(out, i0 + stride, plane, T::plus(y1, z1));
          #pragma unroll
          for (int i = 0; i < WT - 1; ++i) wt[i] = wt[i + 2];
          #pragma unroll
          for (int i = 0; i < WK - 1; ++i) wk[i] = wk[i + 2];
        }
      }
    }
  }
  if (EN) block_sum_store(e, epart + slot);
  });
}

// ---------------------------------------------------------------------------
// Contiguous-axis pass (axis 1), LDS row tiles with periodic halo
// ---------------------------------------------------------------------------
template <int OP, int P, bool K0, bool EN>
__global__ __launch_bounds__(kThreads) void k_contig(PassGeom g, const void* in, void* out,
                                                     const void* k0, int64_t plane, double kmul,
                                                     double* __restrict__ epart) {
  using T = Prec<P>;
  using V = typename T::V;
  constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI, W = OHI - OLO + 1;
  static_assert(OHI <= kHalo && -OLO <= kHalo, "halo too small");
  __shared__ V lds[kContigLds];
  for_each_tile(g, [&](int b, int t, int slot) {
  const OrbDev od = g.orbs[b];
  const int m1 = od.m[0];
  const int rows = od.m[1] * od.m[2];
  const int pitch = m1 + 2 * kHalo;
  const int R = contig_rows(m1, g.xdiv);
  const int row0 = t * R;
  const int nrows = min(R, rows - row0);
  const int64_t gbase = od.off + (int64_t)row0 * m1;
  // load rows [row0, row0 + nrows) with halo: lds[r*pitch + p] = x[r][(p - kHalo) mod m1]
  const int nload = nrows * pitch;
  for (int e = threadIdx.x; e < nload; e += kThreads) {
    const int r = e / pitch;
    const int p = e - r * pitch;
    lds[e] = T::ldc(in, gbase + (int64_t)r * m1 + wrapi(p - kHalo, m1), plane);
  }
  __syncthreads();
  const double ks = od.kscale[0];
  const int half = m1 >> 1;
  const int npairs = nrows * half;
  double en = 0.0;
  for (int q = threadIdx.x; q < npairs; q += kThreads) {
    const int r = q / half;
    const int k = 2 * (q - r * half);
    const V* src = lds + r * pitch + kHalo + k - OHI;
    V win[W + 1];
    #pragma unroll
    for (int i = 0; i <= W; ++i) win[i] = src[i];
    V y0, y1;
    pair_conv<P, OP>(win, y0, y1);
    if (OP == OP_KIN || OP == OP_CK) {
      y0 = T::scale(y0, ks);
      y1 = T::scale(y1, ks);
      if (EN) en += T::d(win[OHI]) * T::d(y0) + T::d(win[OHI + 1]) * T::d(y1);
      if (kmul != 1.0) { y0 = T::scale(y0, kmul); y1 = T::scale(y1, kmul); }
    }
    const int64_t i0 = gbase + (int64_t)r * m1 + k;
    if (K0) {
      y0 = T::plus(y0, T::ldc(k0, i0, plane));
      y1 = T::plus(y1, T::ldc(k0, i0 + 1, plane));
    }
    T::st(out, i0, plane, y0);
    T::st(out, i0 + 1, plane, y1);
  }
  if (EN) block_sum_store(en, epart + slot);
  });
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <int OP, int P>
static hipError_t launch_axis(int axis, const PassGeom& g, int ntiles, const void* in, void* out,
                              const void* k0, int64_t plane, double kmul, double* epart,
                              hipStream_t st) {
  const bool en = epart != nullptr;
  dim3 grid(g.queue ? std::min(ntiles, g.grid) : ntiles), block(kThreads);
  if (ntiles == 0) return hipSuccess;
#define WVL_L(KERN) hipLaunchKernelGGL((KERN), grid, block, 0, st, g, in, out, k0, plane, kmul, epart)
  if (axis == 1) {
    if (k0) { if (en) WVL_L((k_contig<OP, P, true, true>)); else WVL_L((k_contig<OP, P, true, false>)); }
    else    { if (en) WVL_L((k_contig<OP, P, false, true>)); else WVL_L((k_contig<OP, P, false, false>)); }
  } else if (axis == 2) {
    if (k0) { if (en) WVL_L((k_strided<OP, P, 2, true, true>)); else WVL_L((k_strided<OP, P, 2, true, false>)); }
    else    { if (en) WVL_L((k_strided<OP, P, 2, false, true>)); else WVL_L((k_strided<OP, P, 2, false, false>)); }
  } else {
    if (k0) { if (en) WVL_L((k_strided<OP, P, 3, true, true>)); else WVL_L((k_strided<OP, P, 3, true, false>)); }
    else    { if (en) WVL_L((k_strided<OP, P, 3, false, true>)); else WVL_L((k_strided<OP, P, 3, false, false>)); }
  }
#undef WVL_L
  return hipGetLastError();
}

template <int P>
hipError_t launch_op(int op, int axis, const PassGeom& g, int ntiles, const void* in,
                            void* out, const void* k0, int64_t plane, double kmul, double* epart,
                            hipStream_t st) {
  switch (op) {
    case OP_MF:  return launch_axis<OP_MF, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    case OP_MFT: return launch_axis<OP_MFT, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    case OP_SYN: return launch_axis<OP_SYN, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    case OP_ANA: return launch_axis<OP_ANA, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    case OP_KIN: return launch_axis<OP_KIN, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    case OP_CW:  return launch_axis<OP_CW, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    case OP_CWT: return launch_axis<OP_CWT, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
    default:     return launch_axis<OP_CK, P>(axis, g, ntiles, in, out, k0, plane, kmul, epart, st);
  }
}

template <int P>
hipError_t zfinal_p(const PassGeom& g, int ntiles, const void* t, const void* c,
                           const void* kxy, void* out, int64_t plane, double kmul, double* epart,
                           hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  dim3 grid(g.queue ? std::min(ntiles, g.grid) : ntiles), block(kThreads);
  if (epart)
    hipLaunchKernelGGL((k_zfinal<P, true>), grid, block, 0, st, g, t, c, kxy, out, plane, kmul, epart);
  else
    hipLaunchKernelGGL((k_zfinal<P, false>), grid, block, 0, st, g, t, c, kxy, out, plane, kmul, epart);
  return hipGetLastError();
}

}  // namespace wvl
