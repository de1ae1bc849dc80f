// Exact-product engine of the compensated single-precision form, gfx950.
//
// Every 1D pass of the local Hamiltonian is a banded circulant product
// (Sec. 3.1).  In the compensated form the values are float pairs hi + lo;
// here a pass does not evaluate the pair arithmetic tap by tap but splits the
// data and the filter into base-256 digits and multiplies the digits on the
// int8 matrix cores, where products and sums are exact (int32 accumulation):
//
//   x = 2^(e - 47) X,  X = sum_{i<6} d_i 256^(5-i),  d_i in [-128, 127]
//   f = 2^(EF - 47) F, F = sum_{j<6} g_j 256^(5-j)
//   f x = 2^(e + EF - 94) sum_s acc_s 256^(10-s),   acc_s = sum_{i+j=s} g_j d_i
//
// with e the exponent of the plane (every |x| < 0.99 2^e) and EF that of
// the filter.  The groups s <= 5 are kept (21 digit products per output
// tile): the rest weigh less than 2^-40 of the largest term.  The six int32
// group sums are recombined exactly into an int64 T = sum_s acc_s 256^(5-s),
// value 2^(e + EF - 54) T, which either becomes the next pass's digits
// (rounded to 47 bits below the pass's growth bound 2^(e + GF), GF =
// ceil(log2 ||f||_1)) or a float pair again.  Float arithmetic is left for
// the conversions and the pointwise stage (pair products), float64 for the
// density and energy sums only.
//
// Layout in LDS: six digit planes (digit 0 most significant), each a set of
// lines of `pitch` bytes, the contracted axis contiguous.  A 16 x 16 output
// tile of a pass reads its lines' window of 64 inputs per step in chunks of
// 16 bytes (one 16-byte LDS read per lane and digit); tile origins and line
// lengths are multiples of 16, so a chunk never straddles the periodic wrap.
#pragma once

#include "wvl_plane.h"

namespace wvl {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kOzDig = 6;            // base-256 digits per value
constexpr int kOzMaxTiles = 36;      // 16 x 16 tiles of a plane (up to 96 x 96 or 48 x 192)
constexpr int kOzMaxQuads = 2304;    // 4-value quads of a plane (m1 m2 <= 9216)
constexpr uint64_t kOzC = 0x808080808080ull;   // 128 in every digit: balanced digits by XOR
// per workgroup of NW waves: tiles per wave and pass, quads per thread
constexpr int oz_mt(int nw) { return (kOzMaxTiles + nw - 1) / nw; }
constexpr int oz_q(int nw) { return (kOzMaxQuads + 64 * nw - 1) / (64 * nw); }

constexpr double oz_pow2(int e) {
  double r = 1.0;
  if (e >= 0) for (int i = 0; i < e; ++i) r *= 2.0;
  else for (int i = 0; i < -e; ++i) r *= 0.5;
  return r;
}
constexpr double oz_abs(double x) { return x < 0 ? -x : x; }

template <int OP> constexpr double oz_maxabs() {
  double m = 0.0;
  for (int p = 0; p < 2; ++p)
    for (int o = OpWin<OP>::OLO; o <= OpWin<OP>::OHI; ++o)
      m = oz_abs(coef<OP>(p, o, 0)) > m ? oz_abs(coef<OP>(p, o, 0)) : m;
  return m;
}
template <int OP> constexpr double oz_l1() {
  double m = 0.0;
  for (int p = 0; p < 2; ++p) {
    double s = 0.0;
    for (int o = OpWin<OP>::OLO; o <= OpWin<OP>::OHI; ++o) s += oz_abs(coef<OP>(p, o, 0));
    m = s > m ? s : m;
  }
  return m;
}
// smallest e with maxabs < 0.99 2^e (filter digits: |F| < 0.99 2^47)
template <int OP> constexpr int oz_ef() {
  int e = -60;
  while (!(oz_maxabs<OP>() < 0.99 * oz_pow2(e))) ++e;
  return e;
}
// smallest g >= 0 with ||f||_1 (plus the digit rounding) below 2^g
template <int OP> constexpr int oz_gf() {
  int g = 0;
  while (!(oz_l1<OP>() * (1.0 + 1e-6) <= oz_pow2(g))) ++g;
  return g;
}
// round(v 2^k) to an int64 (v 2^k is exact; ties away from zero)
constexpr int64_t oz_round(double v, int k) {
  const double s = v * oz_pow2(k);
  int64_t i = (int64_t)s;
  const double f = s - (double)i;
  if (f >= 0.5) ++i;
  if (f <= -0.5) --i;
  return i;
}

// Filter fragments of operator OP: for window step s and digit q, lane
// l = n + 16 g holds, in bytes j = 0..15, digit q of the filter at tap
// o = n + WOFF - 64 s - 16 g - j for output parity n mod 2: the operand of
// output column n (or row n) against the window chunk g.  The same bytes
// serve as the A operand (filter rows) and the B operand (filter columns).
template <int OP>
struct OzFilt {
  static constexpr int OLO = OpWin<OP>::OLO, OHI = OpWin<OP>::OHI;
  static constexpr int WOFF = 16 * ((OHI + 15) / 16);          // window starts WOFF before k0
  static constexpr int NSTEP = (WOFF + 16 - OLO + 63) / 64;     // 64-input steps per tile
  static constexpr int NT = OHI - OLO + 1;
  uint32_t v[NSTEP][kOzDig][64][4];
  constexpr OzFilt() : v() {
    constexpr int EF = oz_ef<OP>();
    uint64_t Z[2][NT] = {};
    for (int p = 0; p < 2; ++p)
      for (int o = OLO; o <= OHI; ++o)
        Z[p][o - OLO] = ((uint64_t)oz_round(coef<OP>(p, o, 0), 47 - EF) + kOzC) ^ kOzC;
    for (int s = 0; s < NSTEP; ++s)
      for (int q = 0; q < kOzDig; ++q)
        for (int l = 0; l < 64; ++l)
          for (int w = 0; w < 4; ++w) {
            uint32_t word = 0;
            for (int b = 0; b < 4; ++b) {
              const int n = l & 15, g = l >> 4, j = 4 * w + b;
              const int o = n + WOFF - 64 * s - 16 * g - j;
              // taps outside the filter: every digit of zero is 0
              const uint32_t byte = (o >= OLO && o <= OHI)
                                        ? (uint32_t)((Z[n & 1][o - OLO] >> (8 * (5 - q))) & 0xff) : 0u;
              word |= byte << (8 * b);
            }
            v[s][q][l][w] = word;
          }
  }
};

static __device__ const OzFilt<OP_CW> kOzCW = OzFilt<OP_CW>();
static __device__ const OzFilt<OP_CWT> kOzCWT = OzFilt<OP_CWT>();
static __device__ const OzFilt<OP_CK> kOzCK = OzFilt<OP_CK>();

template <int OP> __device__ __forceinline__ const uint32_t* oz_frag_tab() {
  return OP == OP_CW ? &kOzCW.v[0][0][0][0] : OP == OP_CWT ? &kOzCWT.v[0][0][0][0] : &kOzCK.v[0][0][0][0];
}

// Pass constants: EF (filter exponent), GF (growth), R (shift of the sums
// onto the next pass's 47-bit digits).
template <int OP> struct OzK {
  static constexpr int EF = oz_ef<OP>();
  static constexpr int GF = oz_gf<OP>();
  static constexpr int R = GF + 7 - EF;
  static_assert(R >= 1 && R <= 16, "digit shift out of range (T + K must fit 63 bits)");
};

// ---------------------------------------------------------------------------
// conversions

// exponent e of a plane from max |hi|: every |hi + lo| < 0.99 2^e
__device__ __forceinline__ int oz_exp_of(float maxhi) {
  return ((__float_as_int(maxhi * 1.02f) >> 23) & 255) - 126;
}

// X = round((hi + lo) 2^s) as an int64 (|X| < 0.99 2^47 for s = 47 - e)
// (the integer part of hi 2^(s - 24) is exact; its fraction times 2^24 plus
// lo 2^s is below 2^24 + 2^22 and rounds once in the fused multiply-add:
// |error| <= 1.5)
__device__ __forceinline__ int64_t oz_fix(float hi, float lo, int s) {
  const float v = ldexpf(hi, s - 24);                 // |v| < 2^23
  const float vh = truncf(v);
  const float w = rintf(__builtin_fmaf(v - vh, 0x1p24f, ldexpf(lo, s)));
  return (int64_t)(int32_t)vh * 16777216LL + (int64_t)(int32_t)w;
}

// 2^E T as a float pair (hi, lo), |lo| <= ulp(hi) / 2.  a 2^32 is the high
// word rounded to a float and fr the rest (below 2^32 when the high word is
// exact, below the high part's ulp otherwise), so |a 2^32| >= |fr| or a = 0:
// the fast two-sum is exact.
__device__ __forceinline__ f2 oz_tof(int64_t T, int E) {
  const int32_t th = (int32_t)(T >> 32);
  const uint32_t tl = (uint32_t)T;
  const float a = (float)th;
  const int32_t rh = th - (int32_t)a;
  const float fr = __builtin_fmaf((float)rh, 0x1p32f, (float)tl);
  f2 r;
  fast_two_sum(ldexpf(a, E + 32), ldexpf(fr, E), r.hi, r.lo);
  return r;
}

// 2^E T as a double (density and energy sums)
__device__ __forceinline__ double oz_tod(int64_t T, int E) {
  return ldexp(__builtin_fma((double)(int32_t)(T >> 32), 4294967296.0, (double)(uint32_t)T), E);
}

// Compact float pairs of the intermediate arrays (6 bytes a value): the hi
// float plane, then the lo part as an int16 plane in units of 2^-16 ulp(hi)
// (|lo| <= ulp(hi) / 2, so |q| <= 2^15; relative error <= 2^-40).
__device__ __forceinline__ int oz_ulp_exp(float hi) {    // log2 ulp(hi) - 16
  const int eb = (__float_as_int(hi) >> 23) & 255;
  return (eb > 1 ? eb : 1) - 166;
}
__device__ __forceinline__ int16_t oz_lo16(float hi, float lo) {
  const float q = rintf(ldexpf(lo, -oz_ulp_exp(hi)));
  return (int16_t)(int)fminf(fmaxf(q, -32767.0f), 32767.0f);
}
__device__ __forceinline__ float oz_lo_of(float hi, int16_t q) {
  return ldexpf((float)q, oz_ulp_exp(hi));
}
__device__ __forceinline__ const int16_t* oz_lo_plane(const float* base, int64_t plane) {
  return reinterpret_cast<const int16_t*>(base + plane);
}
__device__ __forceinline__ int16_t* oz_lo_plane(float* base, int64_t plane) {
  return reinterpret_cast<int16_t*>(base + plane);
}
// four consecutive values at `at` (a multiple of 4)
__device__ __forceinline__ void oz_store4_cp(float* base, int64_t plane, int64_t at, const f2 (&r)[4]) {
  *reinterpret_cast<float4*>(base + at) = make_float4(r[0].hi, r[1].hi, r[2].hi, r[3].hi);
  uint2 w;
  w.x = (uint32_t)(uint16_t)oz_lo16(r[0].hi, r[0].lo) | ((uint32_t)(uint16_t)oz_lo16(r[1].hi, r[1].lo) << 16);
  w.y = (uint32_t)(uint16_t)oz_lo16(r[2].hi, r[2].lo) | ((uint32_t)(uint16_t)oz_lo16(r[3].hi, r[3].lo) << 16);
  *reinterpret_cast<uint2*>(oz_lo_plane(base, plane) + at) = w;
}
__device__ __forceinline__ void oz_load4_cp(const float* base, int64_t plane, int64_t at, f2 (&r)[4]) {
  const float4 h = *reinterpret_cast<const float4*>(base + at);
  const uint2 w = *reinterpret_cast<const uint2*>(oz_lo_plane(base, plane) + at);
  r[0] = f2{h.x, oz_lo_of(h.x, (int16_t)(w.x & 0xffff))};
  r[1] = f2{h.y, oz_lo_of(h.y, (int16_t)(w.x >> 16))};
  r[2] = f2{h.z, oz_lo_of(h.z, (int16_t)(w.y & 0xffff))};
  r[3] = f2{h.w, oz_lo_of(h.w, (int16_t)(w.y >> 16))};
}

// balanced digits of X (|X| < 0.99 2^47): bytes of Z, digit 5 in byte 0
struct OzZ { uint32_t lo, hi; };
__device__ __forceinline__ OzZ oz_digits(int64_t X) {
  const uint64_t z = ((uint64_t)X + kOzC) ^ kOzC;
  return OzZ{(uint32_t)z, (uint32_t)(z >> 32)};
}
// X of value v (byte v of each digit plane's word dw[q], digit 0 most
// significant): the inverse of oz_digits
__device__ __forceinline__ int64_t oz_undigits(const uint32_t (&dw)[kOzDig], int v) {
  const uint32_t sel = 0x0c0c0c00u | (uint32_t)v;       // byte v, then zeros
  const uint32_t b5 = __builtin_amdgcn_perm(0u, dw[5], sel), b4 = __builtin_amdgcn_perm(0u, dw[4], sel);
  const uint32_t b3 = __builtin_amdgcn_perm(0u, dw[3], sel), b2 = __builtin_amdgcn_perm(0u, dw[2], sel);
  const uint32_t b1 = __builtin_amdgcn_perm(0u, dw[1], sel), b0 = __builtin_amdgcn_perm(0u, dw[0], sel);
  const uint64_t z = ((uint64_t)(b1 | (b0 << 8)) << 32) | (b5 | (b4 << 8) | (b3 << 16) | (b2 << 24));
  return (int64_t)((z ^ kOzC) - kOzC);
}

// digits of round(T 2^-R) (the next pass's fixed point), same form
template <int R>
__device__ __forceinline__ OzZ oz_digits_shift(int64_t T) {
  const uint64_t K = (1ull << (R - 1)) + (kOzC << R);
  const uint64_t z = (((uint64_t)T + K) >> R) ^ kOzC;
  return OzZ{(uint32_t)z, (uint32_t)(z >> 32)};
}

// The digits of four consecutive values, one dword per digit plane
// (d[q] byte v = digit q of value v).
__device__ __forceinline__ void oz_pack(const OzZ (&z)[4], uint32_t (&d)[kOzDig]) {
  const uint32_t a01l = __builtin_amdgcn_perm(z[1].lo, z[0].lo, 0x05010400u);
  const uint32_t a01h = __builtin_amdgcn_perm(z[1].lo, z[0].lo, 0x07030602u);
  const uint32_t a23l = __builtin_amdgcn_perm(z[3].lo, z[2].lo, 0x05010400u);
  const uint32_t a23h = __builtin_amdgcn_perm(z[3].lo, z[2].lo, 0x07030602u);
  d[5] = __builtin_amdgcn_perm(a23l, a01l, 0x05040100u);
  d[4] = __builtin_amdgcn_perm(a23l, a01l, 0x07060302u);
  d[3] = __builtin_amdgcn_perm(a23h, a01h, 0x05040100u);
  d[2] = __builtin_amdgcn_perm(a23h, a01h, 0x07060302u);
  const uint32_t h01 = __builtin_amdgcn_perm(z[1].hi, z[0].hi, 0x05010400u);
  const uint32_t h23 = __builtin_amdgcn_perm(z[3].hi, z[2].hi, 0x05010400u);
  d[1] = __builtin_amdgcn_perm(h23, h01, 0x05040100u);
  d[0] = __builtin_amdgcn_perm(h23, h01, 0x07060302u);
}

// LDS geometry of one layout: contracted length mc, lines mo, pitch bytes per
// line, dstride bytes per digit plane
struct OzGeo { int mc, mo, pitch, dstride; };

// The geometry as values the optimiser cannot see through: per-tile
// addresses are then computed inside each pass instead of being hoisted out
// of the loop over a group's orbitals (and kept live across it).
__device__ __forceinline__ OzGeo oz_opaque(OzGeo g) {
  asm volatile("" : "+s"(g.mc), "+s"(g.mo), "+s"(g.pitch), "+s"(g.dstride));
  return g;
}

// pitch of a line of mc bytes: a multiple of 16 with an odd number of 16-byte
// chunks, so that 16 lanes reading a chunk each from consecutive lines, and
// the 64 dword stores of a tile, fall on distinct banks
__host__ __device__ inline int oz_pitch(int mc) {
  int c = (mc >> 4) + 1;
  if ((c & 1) == 0) ++c;
  return c << 4;
}

// row pitch (doubles) of the density plane kept in LDS: 4 (mod 32), so that
// 16 lanes reading 4 doubles each from 16 consecutive rows spread over the banks
__host__ __device__ inline int oz_rho_pitch(int m1) { return m1 + ((36 - (m1 & 31)) & 31); }

// block-wide max of v (all threads get it), NW waves
template <int NW>
__device__ __forceinline__ float oz_block_max(float v) {
  __shared__ float red[NW];
  #pragma unroll
  for (int s = 32; s > 0; s >>= 1) v = fmaxf(v, __shfl_xor(v, s, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = red[0];
  #pragma unroll
  for (int w = 1; w < NW; ++w) t = fmaxf(t, red[w]);
  __syncthreads();
  return t;
}

// block-wide float64 sum (all threads get it), NW waves
template <int NW>
__device__ __forceinline__ double oz_block_sum(double v) {
  __shared__ double red[NW];
  #pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  #pragma unroll
  for (int w = 0; w < NW; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Load a plane of float pairs into the digit planes of `dst` (layout g):
// value (line L, index k) at src[gp + k * ks + L * ls] (hi; lo at + plane).
// ROWS: ks == 1 (4 consecutive k per 16-byte load); otherwise ls == 1 and
// each thread loads 4 values of one column.  e < -1000: take the plane's
// exponent from its values (block max); returns the exponent used.
// CP: the source is a compact pair array (hi floats, int16 lo plane).
template <bool ROWS, int NW, bool CP = false>
__device__ __forceinline__ int oz_load(const float* src, int64_t plane, int64_t gp, int64_t stride,
                                       const OzGeo& g_, uint8_t* dst, int e) {
  const OzGeo g = oz_opaque(g_);
  constexpr int Q = oz_q(NW);
  const int nq = (g.mc >> 2) * g.mo;
  // quad i of this thread: qd = tid + i 64 NW, at (line L, index k); ROWS
  // steps along lines of mc / 4 quads, otherwise along columns of mo quads.
  // (L, k) are stepped incrementally (one division per call).
  const int per = ROWS ? (g.mc >> 2) : g.mo;        // quads per row of the quad grid
  const int dq = (64 * NW) / per, dr = 64 * NW - dq * per;
  int qa = (int)threadIdx.x / per, qb = (int)threadIdx.x - qa * per;
  int La[Q], ka[Q];
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    La[i] = ROWS ? qa : qb;
    ka[i] = ROWS ? qb << 2 : qa << 2;
    qa += dq;
    qb += dr;
    if (qb >= per) { qb -= per; ++qa; }
  }
  float h[Q][4], l[Q][4];
  float m = 0.0f;
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int qd = threadIdx.x + i * 64 * NW;
    if (qd < nq) {
      const int L = La[i], k = ka[i];
      if (ROWS) {
        const int64_t a = gp + (int64_t)L * stride + k;
        if (CP) {
          f2 r[4];
          oz_load4_cp(src, plane, a, r);
          #pragma unroll
          for (int v = 0; v < 4; ++v) { h[i][v] = r[v].hi; l[i][v] = r[v].lo; }
        } else {
          const float4 hv = *reinterpret_cast<const float4*>(src + a);
          const float4 lv = *reinterpret_cast<const float4*>(src + plane + a);
          h[i][0] = hv.x; h[i][1] = hv.y; h[i][2] = hv.z; h[i][3] = hv.w;
          l[i][0] = lv.x; l[i][1] = lv.y; l[i][2] = lv.z; l[i][3] = lv.w;
        }
      } else {
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t a = gp + (int64_t)(k + v) * stride + L;
          h[i][v] = src[a];
          l[i][v] = CP ? oz_lo_of(h[i][v], oz_lo_plane(src, plane)[a]) : src[plane + a];
        }
      }
      #pragma unroll
      for (int v = 0; v < 4; ++v) m = fmaxf(m, fabsf(h[i][v]));
    }
  }
  if (e < -1000) e = oz_exp_of(oz_block_max<NW>(m));
  const int s = 47 - e;
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int qd = threadIdx.x + i * 64 * NW;
    if (qd < nq) {
      OzZ z[4];
      #pragma unroll
      for (int v = 0; v < 4; ++v) z[v] = oz_digits(oz_fix(h[i][v], l[i][v], s));
      uint32_t d[kOzDig];
      oz_pack(z, d);
      uint8_t* p = dst + La[i] * g.pitch + ka[i];
      #pragma unroll
      for (int q = 0; q < kOzDig; ++q) *reinterpret_cast<uint32_t*>(p + q * g.dstride) = d[q];
    }
  }
  return e;
}

// Digits of a plane in layout g ([y][x]: lines y of mc = m1 bytes) rewritten
// in layout gt ([x][y]), in place: each thread moves 4 x 4 blocks (4 rows of
// one 4-byte word per digit plane, transposed with byte permutes); a wave
// covers 8 x 8 blocks (rows and columns in steps of 4 lines: at most two
// lanes per bank).  All blocks are read before the barrier, written after it.
template <int NW>
__device__ __forceinline__ void oz_transpose(uint8_t* lds, const OzGeo& g_, const OzGeo& gt_) {
  const OzGeo g = oz_opaque(g_), gt = oz_opaque(gt_);
  const int nbx = g.mc >> 2, nby = g.mo >> 2;             // 4 x 4 blocks along x and y
  const int wtx = (nbx + 7) >> 3, wty = (nby + 7) >> 3;   // 8 x 8 block tiles
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  constexpr int KB = (kOzMaxQuads / 4 + 64 * NW - 1) / (64 * NW);   // block tiles per wave
  uint32_t d[KB][kOzDig][4];
  int bx[KB], by[KB];
  bool ok[KB];
  #pragma unroll
  for (int r = 0; r < KB; ++r) {
    const int wt = wave + r * NW;
    const int ty = wt / (wtx > 0 ? wtx : 1), tx = wt - ty * wtx;
    bx[r] = tx * 8 + (lane & 7);
    by[r] = ty * 8 + (lane >> 3);
    ok[r] = wt < wtx * wty && bx[r] < nbx && by[r] < nby;
    if (ok[r]) {
      const uint8_t* src = lds + (4 * by[r]) * g.pitch + 4 * bx[r];
      #pragma unroll
      for (int q = 0; q < kOzDig; ++q)
        #pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          d[r][q][rr] = *reinterpret_cast<const uint32_t*>(src + q * g.dstride + rr * g.pitch);
    }
  }
  __syncthreads();
  #pragma unroll
  for (int r = 0; r < KB; ++r) {
    if (!ok[r]) continue;
    uint8_t* dst = lds + (4 * bx[r]) * gt.pitch + 4 * by[r];
    #pragma unroll
    for (int q = 0; q < kOzDig; ++q) {
      const uint32_t* D = d[r][q];
      const uint32_t t01l = __builtin_amdgcn_perm(D[1], D[0], 0x05010400u);
      const uint32_t t23l = __builtin_amdgcn_perm(D[3], D[2], 0x05010400u);
      const uint32_t t01h = __builtin_amdgcn_perm(D[1], D[0], 0x07030602u);
      const uint32_t t23h = __builtin_amdgcn_perm(D[3], D[2], 0x07030602u);
      uint8_t* o = dst + q * gt.dstride;
      *reinterpret_cast<uint32_t*>(o) = __builtin_amdgcn_perm(t23l, t01l, 0x05040100u);
      *reinterpret_cast<uint32_t*>(o + gt.pitch) = __builtin_amdgcn_perm(t23l, t01l, 0x07060302u);
      *reinterpret_cast<uint32_t*>(o + 2 * gt.pitch) = __builtin_amdgcn_perm(t23h, t01h, 0x05040100u);
      *reinterpret_cast<uint32_t*>(o + 3 * gt.pitch) = __builtin_amdgcn_perm(t23h, t01h, 0x07060302u);
    }
  }
  __syncthreads();
}

// The tiles of this wave (tile = wave + t NW) in one pass, enumerated with
// scalar arithmetic (the wave index is uniform) and without a division per
// tile: tile = a nb + b.  Order 0 (an x pass in (y block, x block) order, or
// any pass): output block k0 = 16 b along the contracted axis (nb = mc / 16),
// line block o0 = 16 a.  Order 2 (a y pass in (y block, x block) order,
// lines x): k0 = 16 a, o0 = 16 b (nb = mo / 16), so that an x pass and a y
// pass of one plane give a lane the same plane elements.
template <int NW>
struct OzTiles {
  int a, b, nb, da, db;
  __device__ __forceinline__ OzTiles(const OzGeo& g, int order) {
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    nb = order == 2 ? g.mo >> 4 : g.mc >> 4;
    a = wave / nb;
    b = wave - a * nb;
    da = NW / nb;
    db = NW - da * nb;
  }
  __device__ __forceinline__ int k0(int order) const { return (order == 2 ? a : b) << 4; }
  __device__ __forceinline__ int o0(int order) const { return (order == 2 ? b : a) << 4; }
  __device__ __forceinline__ void next() {
    a += da;
    b += db;
    if (b >= nb) { b -= nb; ++a; }
  }
};

// One pass of operator OP over the digit planes in `src`.  DA: data as the A
// operand (rows = lines), else as the B operand (columns = lines).  For every
// tile t of this wave (output block k0, line block o0) epi(t, k0, o0, T) gets
// the exact sums T[v] of the lane's four elements: (line o0 + 4 g + v, output
// k0 + n) with DA, (output k0 + 4 g + v, line o0 + n) without, lane = n + 16 g;
// value 2^(e + EF - 54) T[v] for input exponent e.
// RF: every step's filter digits held in registers for the whole pass (else
// a two-step filter reloads them per tile and step, 24 registers fewer)
template <int OP, bool DA, int NW, bool RF = true, typename Epi>
__device__ __forceinline__ void oz_pass(const uint8_t* src, const OzGeo& g_, int yx, Epi&& epi) {
  using Fl = OzFilt<OP>;
  const OzGeo g = oz_opaque(g_);
  const int lane = threadIdx.x & 63, n = lane & 15, gq = lane >> 4;
  const int nt = (g.mc >> 4) * (g.mo >> 4);
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int order = yx == 2 ? 2 : 0;
  OzTiles<NW> it(g, order);
  // chunk offset of this lane's window in step st relative to k0, reduced
  // into [0, mc) once per pass: the chunk starts at (k0 + off[st]) mod mc
  int off[Fl::NSTEP];
  #pragma unroll
  for (int st = 0; st < Fl::NSTEP; ++st) {
    int o = (-Fl::WOFF + 64 * st + 16 * gq) % g.mc;
    off[st] = o < 0 ? o + g.mc : o;
  }
  const uint8_t* lane_src = src + n * g.pitch;
  const uint32_t* ft = oz_frag_tab<OP>();
  asm volatile("" : "+s"(ft));     // keep the table loads inside the pass
  constexpr int NR = (RF || Fl::NSTEP == 1) ? Fl::NSTEP : 0;   // steps held in registers
  v4i f0[NR > 0 ? NR : 1][kOzDig];
  #pragma unroll
  for (int st = 0; st < NR; ++st)
    #pragma unroll
    for (int q = 0; q < kOzDig; ++q)
      f0[st][q] = *reinterpret_cast<const v4i*>(ft + ((st * kOzDig + q) * 64 + lane) * 4);
  #pragma unroll
  for (int t = 0; t < oz_mt(NW); ++t, it.next()) {
    if (wave + t * NW >= nt) break;
    const int k0 = it.k0(order), o0 = it.o0(order);
    const uint8_t* lp = lane_src + o0 * g.pitch;
    v4i acc[kOzDig];
    #pragma unroll
    for (int s = 0; s < kOzDig; ++s) acc[s] = v4i{0, 0, 0, 0};
    #pragma unroll
    for (int st = 0; st < Fl::NSTEP; ++st) {
      v4i f[kOzDig];
      #pragma unroll
      for (int q = 0; q < kOzDig; ++q)
        f[q] = st < NR ? f0[st < NR ? st : 0][q]
                       : *reinterpret_cast<const v4i*>(ft + ((st * kOzDig + q) * 64 + lane) * 4);
      int c0 = k0 + off[st];
      c0 = c0 >= g.mc ? c0 - g.mc : c0;
      // data digit i against filter digits j <= 5 - i; the next digit's LDS
      // read is issued before this digit's products (two digits in flight)
      const uint8_t* dp = lp + c0;
      v4i a = *reinterpret_cast<const v4i*>(dp);
      #pragma unroll
      for (int i = 0; i < kOzDig; ++i) {
        v4i an = a;
        if (i + 1 < kOzDig) an = *reinterpret_cast<const v4i*>(dp + (i + 1) * g.dstride);
        #pragma unroll
        for (int j = 0; j + i < kOzDig; ++j)
          acc[i + j] = DA ? __builtin_amdgcn_mfma_i32_16x16x64_i8(a, f[j], acc[i + j], 0, 0, 0)
                          : __builtin_amdgcn_mfma_i32_16x16x64_i8(f[j], a, acc[i + j], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        a = an;
      }
    }
    // exact recombination: T = sum_s acc_s 256^(5 - s) (pairs in 32 bits:
    // |acc_s| < 2^23 for <= 64 nonzero taps)
    int64_t T[4];
    #pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int32_t p01 = (int32_t)((uint32_t)acc[0][v] << 8) + acc[1][v];
      const int32_t p23 = (int32_t)((uint32_t)acc[2][v] << 8) + acc[3][v];
      const int32_t p45 = (int32_t)((uint32_t)acc[4][v] << 8) + acc[5][v];
      T[v] = (int64_t)p01 * 4294967296LL + (int64_t)p23 * 65536LL + (int64_t)p45;
    }
    epi(t, k0, o0, T);
    // one tile in flight at a time (hoisting the next tile's loads would
    // exceed the register budget)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Digits kept in registers between a pass (all its reads) and the barrier
// after which they overwrite the plane: tile t's four elements (consecutive
// along the next pass's contracted axis) go to line k0 + n, index o0 + 4 g of
// layout gn.
template <int NW>
struct OzPacked {
  uint32_t d[oz_mt(NW)][kOzDig];
  int n;
};

// g, yx: the geometry and tile order of the pass that produced pk
template <int NW>
__device__ __forceinline__ void oz_store_packed(const OzPacked<NW>& pk, const OzGeo& g_, int yx,
                                                uint8_t* dst, const OzGeo& gn_) {
  const OzGeo g = oz_opaque(g_), gn = oz_opaque(gn_);
  const int lane = threadIdx.x & 63, n = lane & 15, gq = lane >> 4;
  const int order = yx == 2 ? 2 : 0;
  OzTiles<NW> it(g, order);
  uint8_t* lane_dst = dst + n * gn.pitch + 4 * gq;
  #pragma unroll
  for (int t = 0; t < oz_mt(NW); ++t, it.next()) {
    if (t >= pk.n) break;
    uint8_t* p = lane_dst + it.k0(order) * gn.pitch + it.o0(order);
    #pragma unroll
    for (int q = 0; q < kOzDig; ++q) *reinterpret_cast<uint32_t*>(p + q * gn.dstride) = pk.d[t][q];
  }
}

// A pass whose results become the next pass's digits (shift R), in place:
// read everything, barrier, write the digits in layout gn, barrier.
template <int OP, int NW>
__device__ __forceinline__ void oz_pass_to_digits(uint8_t* lds, const OzGeo& g, const OzGeo& gn) {
  OzPacked<NW> pk;
  pk.n = 0;
  oz_pass<OP, true, NW>(lds, g, 0, [&](int t, int, int, const int64_t (&T)[4]) {
    OzZ z[4];
    #pragma unroll
    for (int v = 0; v < 4; ++v) z[v] = oz_digits_shift<OzK<OP>::R>(T[v]);
    oz_pack(z, pk.d[t]);
    pk.n = t + 1;
  });
  __syncthreads();
  oz_store_packed(pk, g, 0, lds, gn);
  __syncthreads();
}

// float-pair arithmetic of the pointwise and final stages
__device__ __forceinline__ f2 oz_add(f2 a, f2 b) {
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  f2 r;
  fast_two_sum(s, e, r.hi, r.lo);
  return r;
}
__device__ __forceinline__ f2 oz_mul(f2 a, f2 b) {
  const float p = a.hi * b.hi;
  float e = __builtin_fmaf(a.hi, b.hi, -p);
  e = __builtin_fmaf(a.hi, b.lo, e);
  e = __builtin_fmaf(a.lo, b.hi, e);
  f2 r;
  fast_two_sum(p, e, r.hi, r.lo);
  return r;
}

}  // namespace wvl
