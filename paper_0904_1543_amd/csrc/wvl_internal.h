// Internal definitions shared by the HIP kernels and the host side of libwvl.
//
// Data layout (one orbital, periodic fine grid m_a = 2 n_a): a (m3, m2, m1)
// array in C order, axis 1 fastest.  Coarse coefficients use the same shape
// with scaling/wavelet parts interleaved along every axis (index 2i: scaling,
// 2i+1: wavelet, Sec. 2.1 Eq. "wavef0").  A batch is a packed buffer: orbital b
// starts at element off_b.  The compensated single-precision form stores two
// float planes, hi then lo, each of `plane` elements.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "filters_gen.h"

namespace wvl {

enum PrecId { F64 = 0, F32 = 1, F32C = 2 };

// 1D periodic operators along one axis (Sec. 3.1, Eq. "1dconvtrans", and the
// kinetic recursion of Sec. 3.4).  Every one is written as a polyphase filter
//     y[k] = sum_{o = OLO}^{OHI} F_{k mod 2}(o) x[(k - o) mod m]
enum OpKind { OP_MF = 0, OP_MFT = 1, OP_SYN = 2, OP_ANA = 3, OP_KIN = 4,
              // combined filters (the composition of two or three of the above,
              // Sec. 2.4 last paragraph: synthesis + magic filter, transposed
              // magic filter + analysis, analysis o kinetic o synthesis)
              OP_CW = 5, OP_CWT = 6, OP_CK = 7 };
constexpr int kNumOps = 8;

template <int OP> struct OpWin;
template <> struct OpWin<OP_MF>  { static constexpr int OLO = -7,  OHI = 8;  };
template <> struct OpWin<OP_MFT> { static constexpr int OLO = -8,  OHI = 7;  };
template <> struct OpWin<OP_SYN> { static constexpr int OLO = -8,  OHI = 8;  };
template <> struct OpWin<OP_ANA> { static constexpr int OLO = -8,  OHI = 8;  };
template <> struct OpWin<OP_KIN> { static constexpr int OLO = -14, OHI = 14; };
template <> struct OpWin<OP_CW>  { static constexpr int OLO = WVL_CW_LO,  OHI = WVL_CW_LO + WVL_CW_N - 1; };
template <> struct OpWin<OP_CWT> { static constexpr int OLO = WVL_CWT_LO, OHI = WVL_CWT_LO + WVL_CWT_N - 1; };
template <> struct OpWin<OP_CK>  { static constexpr int OLO = WVL_CK_LO,  OHI = WVL_CK_LO + WVL_CK_N - 1; };

// Base-filter lookups with the out-of-window convention (zero outside j = -7..8).
__host__ __device__ constexpr int tapidx(int j) { return j - WVL_TAP_LO; }
__host__ __device__ constexpr bool intap(int j) { return j >= WVL_TAP_LO && j < WVL_TAP_LO + WVL_NTAP; }

// Polyphase coefficient, part 0 = float64 value, 1 = float32 hi, 2 = float32 lo.
//  MF : y[I] = sum_l w_l x[I - l]          -> F(o) = omega_o
//  MFT: y[i] = sum_l w_l x[i + l]          -> F(o) = omega_{-o}
//  SYN: s[k] = sum_{j = k mod 2} h_j x[k - j] + g_j x[k - j + 1]
//       -> o = p mod 2: h_o ;  o = p + 1 mod 2: g_{o+1}
//  ANA: y[2i] = sum_j h_j s[2i + j], y[2i+1] = sum_j g_j s[2i + j]
//       -> p = 0: h_{-o} ;  p = 1: g_{1-o}
//  KIN: F(o) = r_o (the -1/(2h^2) factor is applied to the sum)
//  CW, CWT, CK: generated tables of the compositions (kinetic: before the
//  -1/(2h^2) factor)
template <int OP>
__host__ __device__ constexpr double coef(int p, int o, int part) {
  if (OP == OP_CW || OP == OP_CWT || OP == OP_CK) {
    const int lo = OP == OP_CW ? WVL_CW_LO : OP == OP_CWT ? WVL_CWT_LO : WVL_CK_LO;
    const int n = OP == OP_CW ? WVL_CW_N : OP == OP_CWT ? WVL_CWT_N : WVL_CK_N;
    const int i = o - lo;
    if (i < 0 || i >= n) return 0.0;
    if (OP == OP_CW)
      return p == 0 ? (part == 0 ? WVL_CW0[i] : part == 1 ? (double)WVL_CW0_32_HI[i] : (double)WVL_CW0_32_LO[i])
                    : (part == 0 ? WVL_CW1[i] : part == 1 ? (double)WVL_CW1_32_HI[i] : (double)WVL_CW1_32_LO[i]);
    if (OP == OP_CWT)
      return p == 0 ? (part == 0 ? WVL_CWT0[i] : part == 1 ? (double)WVL_CWT0_32_HI[i] : (double)WVL_CWT0_32_LO[i])
                    : (part == 0 ? WVL_CWT1[i] : part == 1 ? (double)WVL_CWT1_32_HI[i] : (double)WVL_CWT1_32_LO[i]);
    return p == 0 ? (part == 0 ? WVL_CK0[i] : part == 1 ? (double)WVL_CK0_32_HI[i] : (double)WVL_CK0_32_LO[i])
                  : (part == 0 ? WVL_CK1[i] : part == 1 ? (double)WVL_CK1_32_HI[i] : (double)WVL_CK1_32_LO[i]);
  }
  int j = 0;
  int which = 0;  // 0 h, 1 g, 2 omega, 3 kinetic
  bool zero = false;
  if (OP == OP_MF) { which = 2; j = o; zero = !intap(j); }
  else if (OP == OP_MFT) { which = 2; j = -o; zero = !intap(j); }
  else if (OP == OP_SYN) {
    if (((o - p) & 1) == 0) { which = 0; j = o; } else { which = 1; j = o + 1; }
    zero = !intap(j);
  } else if (OP == OP_ANA) {
    if (p == 0) { which = 0; j = -o; } else { which = 1; j = 1 - o; }
    zero = !intap(j);
  } else { which = 3; j = o; zero = (o < -WVL_KIN_HALF || o > WVL_KIN_HALF); }
  if (zero) return 0.0;
  if (which == 3) {
    int i = j + WVL_KIN_HALF;
    return part == 0 ? WVL_KIN[i] : part == 1 ? (double)WVL_KIN32_HI[i] : (double)WVL_KIN32_LO[i];
  }
  int i = tapidx(j);
  if (which == 0) return part == 0 ? WVL_H[i] : part == 1 ? (double)WVL_H32_HI[i] : (double)WVL_H32_LO[i];
  if (which == 1) return part == 0 ? WVL_G[i] : part == 1 ? (double)WVL_G32_HI[i] : (double)WVL_G32_LO[i];
  return part == 0 ? WVL_OMEGA[i] : part == 1 ? (double)WVL_OMEGA32_HI[i] : (double)WVL_OMEGA32_LO[i];
}

// ---------------------------------------------------------------------------
// Device descriptors
// ---------------------------------------------------------------------------
constexpr int kThreads = 256;          // threads per workgroup for the pass kernels
constexpr int kContigLds = 4096;       // LDS values per x-pass tile
constexpr int kHalo = 32;              // periodic halo kept on each side in LDS

struct OrbDev {
  int32_t m[3];        // fine dims m1, m2, m3
  int32_t pad;
  int64_t off;         // element offset of the orbital in packed batch buffers
  int64_t voff;        // element offset of its potential (0 for a shared V)
  double kscale[3];    // -1 / (2 h_a^2), per axis
  double occ;          // occupation f_i
  double kdiag[3][2];  // diagonal of the kinetic operator in the wavelet basis,
                       // per axis: [0] scaling, [1] wavelet coefficients
};

// Tiling of one kind of pass: tile t of the launch belongs to the orbital b
// with prefix[b] <= t < prefix[b+1].  Persistent launches (queue != nullptr)
// run `grid` workgroups that take tiles from a work queue (an int counter,
// zero before the launch) until all ntiles are done, in the order of
// `order`: the prefix over the orbitals perm[0], perm[1], ... listed by
// decreasing cost per tile, so the largest tiles start first and the small
// ones fill the end (longest-processing-time-first list scheduling).
struct PassGeom {
  const OrbDev* orbs;
  const int32_t* prefix;
  int32_t norb;
  const int32_t* order;
  const int32_t* perm;
  int32_t* queue;
  int32_t ntiles;
  int32_t grid;
  int32_t xdiv;    // axis-1 passes: rows per tile = (rows that fit in LDS) / xdiv
};

// rows of length m1 per axis-1 tile (kContigLds values of LDS with halo)
__host__ __device__ inline int contig_rows(int m1, int xdiv) {
  int r = kContigLds / (m1 + 2 * kHalo);
  r = xdiv > 1 ? r / xdiv : r;
  return r < 1 ? 1 : r;
}


__device__ __forceinline__ void find_tile(const int32_t* prefix, int norb, int tile, int& b, int& t) {
  int lo = 0, hi = norb;  // prefix[lo] <= tile < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (__ldg(prefix + mid) <= tile) lo = mid; else hi = mid;
  }
  b = lo;
  t = tile - __ldg(prefix + lo);
}

// Runs body(b, t, slot) for every tile of the workgroup: the tile of its own
// index, or (persistent launch) tiles from the queue until it runs dry.  slot
// is the tile's index in `prefix` order (where per-tile partial sums go).
// Every thread of the workgroup takes the same path, so body may use
// barriers; every workgroup leaves once the counter has passed ntiles.
template <typename F>
__device__ __forceinline__ void for_each_tile(const PassGeom& g, F&& body) {
  if (g.queue == nullptr) {
    int b, t;
    find_tile(g.prefix, g.norb, blockIdx.x, b, t);
    body(b, t, (int)blockIdx.x);
    return;
  }
  __shared__ int s_tile;
  for (;;) {
    __syncthreads();   // the previous tile is finished and s_tile has been read
    if (threadIdx.x == 0) s_tile = atomicAdd(g.queue, 1);
    __syncthreads();
    const int vt = s_tile;
    if (vt >= g.ntiles) break;
    int r, t;
    find_tile(g.order, g.norb, vt, r, t);
    const int b = __ldg(g.perm + r);
    body(b, t, __ldg(g.prefix + b) + t);
  }
}

__device__ __forceinline__ int wrapi(int i, int m) {
  if ((unsigned)i < (unsigned)m) return i;
  i %= m;
  return i < 0 ? i + m : i;
}

// ---------------------------------------------------------------------------
// Precision traits.  V is the register value; storage is planar.
// ---------------------------------------------------------------------------
struct f2 { float hi, lo; };

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float z = s - a;
  e = (a - (s - z)) + (b - z);
}
__device__ __forceinline__ void fast_two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  e = b - (s - a);
}

template <int P> struct Prec;

template <> struct Prec<F64> {
  using V = double;
  struct Acc { double s; };
  static constexpr int bytes = 8;
  __device__ static V ldc(const void* p, int64_t i, int64_t) { return ((const double*)p)[i]; }
  __device__ static void st(void* p, int64_t i, int64_t, V v) { ((double*)p)[i] = v; }
  __device__ static Acc zero() { return Acc{0.0}; }
  template <int OP> __device__ static void add(Acc& a, int par, int o, const V& x) {
    a.s = __builtin_fma(coef<OP>(par, o, 0), x, a.s);
  }
  __device__ static V fin(const Acc& a) { return a.s; }
  __device__ static V scale(V v, double s) { return v * s; }
  __device__ static V plus(V a, V b) { return a + b; }
  __device__ static double d(V v) { return v; }
  __device__ static V from_d(double x) { return x; }
};

template <> struct Prec<F32> {
  using V = float;
  struct Acc { float s; };
  static constexpr int bytes = 4;
  __device__ static V ldc(const void* p, int64_t i, int64_t) { return ((const float*)p)[i]; }
  __device__ static void st(void* p, int64_t i, int64_t, V v) { ((float*)p)[i] = v; }
  __device__ static Acc zero() { return Acc{0.0f}; }
  template <int OP> __device__ static void add(Acc& a, int par, int o, const V& x) {
    a.s = __builtin_fmaf((float)coef<OP>(par, o, 1), x, a.s);
  }
  __device__ static V fin(const Acc& a) { return a.s; }
  __device__ static V scale(V v, double s) { return v * (float)s; }
  __device__ static V plus(V a, V b) { return a + b; }
  __device__ static double d(V v) { return (double)v; }
  __device__ static V from_d(double x) { return (float)x; }
};

// Compensated single precision: every value is an unevaluated pair hi + lo of
// floats.  A filter sum y = sum_o w_o x_o is accumulated with error-free
// transforms on the hi parts (TwoProduct by FMA, TwoSum) and the first-order
// cross terms w_hi x_lo + w_lo x_hi in plain float, all in float arithmetic.
template <> struct Prec<F32C> {
  using V = f2;
  struct Acc { float s, c; };
  static constexpr int bytes = 8;
  __device__ static V ldc(const void* p, int64_t i, int64_t plane) {
    const float* f = (const float*)p;
    return f2{f[i], f[plane + i]};
  }
  __device__ static void st(void* p, int64_t i, int64_t plane, V v) {
    float* f = (float*)p;
    f[i] = v.hi;
    f[plane + i] = v.lo;
  }
  __device__ static Acc zero() { return Acc{0.0f, 0.0f}; }
  template <int OP> __device__ static void add(Acc& a, int par, int o, const V& x) {
    const float wh = (float)coef<OP>(par, o, 1);
    const float wl = (float)coef<OP>(par, o, 2);
    float p = wh * x.hi;
    float e = __builtin_fmaf(wh, x.hi, -p);
    float s, q;
    two_sum(a.s, p, s, q);
    a.s = s;
    float c = a.c + (q + e);
    c = __builtin_fmaf(wh, x.lo, c);
    a.c = __builtin_fmaf(wl, x.hi, c);
  }
  __device__ static V fin(const Acc& a) {
    V r;
    two_sum(a.s, a.c, r.hi, r.lo);
    return r;
  }
  // (hi + lo) * s with s split into float hi/lo parts
  __device__ static V scale(V v, double sd) {
    float sh = (float)sd;
    float sl = (float)(sd - (double)sh);
    float p = v.hi * sh;
    float e = __builtin_fmaf(v.hi, sh, -p);
    e = __builtin_fmaf(v.hi, sl, e);
    e = __builtin_fmaf(v.lo, sh, e);
    V r;
    fast_two_sum(p, e, r.hi, r.lo);
    return r;
  }
  __device__ static V plus(V a, V b) {
    float s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    V r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
  }
  __device__ static double d(V v) { return (double)v.hi + (double)v.lo; }
  __device__ static V from_d(double x) {
    float h = (float)x;
    return f2{h, (float)(x - (double)h)};
  }
};

}  // namespace wvl
