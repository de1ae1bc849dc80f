// Orbital overlap matrix and Cholesky orthonormalisation in float64, gfx950.
//
// Sec. 2.6 and Sec. 5 (step VIII): scalar products between orbitals are taken
// directly on the coefficients because the basis is orthonormal; the overlap
// matrix S = X X^T (X: one row of coefficients per orbital) is factorised as
// S = L L^T and the orbitals are replaced by the rows of L^{-1} X.  The paper
// runs the SYRK on the GPU and the factorisation on the host; here everything
// stays on the GPU, in float64:
//  * SYRK on the float64 matrix cores (v_mfma_f64_16x16x4f64).  A step sums
//    over 4 coefficients; since the sum does not depend on their order, lane
//    group q of step s takes coefficient 4q + s of a 16-coefficient chunk for
//    both operands.  Up to 256 orbitals, one workgroup per coefficient slice
//    stages the chunks of all rows in LDS and its waves compute 32x32 blocks
//    of the lower triangle; for more orbitals one wave owns a 64x64 block over
//    a slice, reading its rows as whole 128-byte lines, with the blocks of one
//    slice placed on one XCD.  Slice partials are summed in a fixed order;
//  * blocked Cholesky and L^{-1} in one single-workgroup launch: 32 x 32
//    diagonal blocks factorised in registers, panels, trailing updates and
//    the blocks of L^{-1} on the float64 matrix cores;
//  * X <- L^{-1} X on the matrix cores, skipping the zero blocks of L^{-1}.

#include "wvl_kernels.h"

namespace wvl {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kBlk = 64;        // rows of an S block (one wave)
constexpr int kSlice = 2048;    // coefficients per wave
constexpr int kXcd = 8;         // XCDs of the MI355X

__host__ __device__ inline int nblk64(int norb) { return (norb + kBlk - 1) / kBlk; }
__host__ __device__ inline int ntri(int nb) { return nb * (nb + 1) / 2; }

static int64_t syrk32_partials(int norb, int64_t len);
static bool syrk32_used(int norb);

// doubles of slice partials the overlap of this shape uses
int64_t syrk_partials(int norb, int64_t len) {
  if (syrk32_used(norb)) return syrk32_partials(norb, len);
  const int64_t nslice = (len + kSlice - 1) / kSlice;
  return nslice * ntri(nblk64(norb)) * kBlk * kBlk;
}

// 4 consecutive coefficients of one row as float64 (zero outside the matrix)
template <int P>
__device__ __forceinline__ void load4(const void* X, int64_t plane, int64_t row, int norb,
                                      int64_t len, int64_t k, double v[4]) {
  using T = Prec<P>;
  #pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = 0.0;
  if (row >= norb) return;
  const int64_t base = row * len + k;
  if (k + 3 < len) {
    #pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = T::d(T::ldc(X, base + s, plane));
  } else {
    #pragma unroll
    for (int s = 0; s < 4; ++s)
      if (k + s < len) v[s] = T::d(T::ldc(X, base + s, plane));
  }
}

// N (2, 4 or 8) consecutive values at element i (i a multiple of N; batch
// lengths are multiples of 8) as float64, with vector loads
template <int P, int N>
__device__ __forceinline__ void ld_run(const void* X, int64_t plane, int64_t i, double (&v)[N]) {
  if (P == F64) {
    const double2* p = reinterpret_cast<const double2*>((const double*)X + i);
    #pragma unroll
    for (int u = 0; u < N / 2; ++u) {
      const double2 d = p[u];
      v[2 * u] = d.x;
      v[2 * u + 1] = d.y;
    }
  } else if (N == 2) {
    const float2 a = *reinterpret_cast<const float2*>((const float*)X + i);
    float2 b = make_float2(0.f, 0.f);
    if (P == F32C) b = *reinterpret_cast<const float2*>((const float*)X + plane + i);
    v[0] = (double)a.x + (double)b.x;
    v[1] = (double)a.y + (double)b.y;
  } else {
    const float4* h = reinterpret_cast<const float4*>((const float*)X + i);
    const float4* l = reinterpret_cast<const float4*>((const float*)X + plane + i);
    #pragma unroll
    for (int u = 0; u < N / 4; ++u) {
      const float4 a = h[u];
      float4 b = make_float4(0.f, 0.f, 0.f, 0.f);
      if (P == F32C) b = l[u];
      v[4 * u] = (double)a.x + (double)b.x;
      v[4 * u + 1] = (double)a.y + (double)b.y;
      v[4 * u + 2] = (double)a.z + (double)b.z;
      v[4 * u + 3] = (double)a.w + (double)b.w;
    }
  }
}

// grid: one wave per (slice, lower-triangle block); the blocks of one slice
// share blockIdx.x mod 8, i.e. run on one XCD.
template <int P>
__global__ __launch_bounds__(64) void k_syrk(const void* __restrict__ X, int64_t plane, int norb,
                                             int64_t len, int nslice, double* __restrict__ part) {
  const int nb = nblk64(norb), nt = ntri(nb);
  const int b = blockIdx.x;
  const int xcd = b % kXcd, r = b / kXcd;         // r-th block placed on this XCD
  const int sgrp = r / nt, tri = r % nt;
  const int slice = sgrp * kXcd + xcd;
  if (slice >= nslice) return;
  int I = 0;                                      // tri -> (I, J), I >= J
  while ((I + 1) * (I + 2) / 2 <= tri) ++I;
  const int J = tri - I * (I + 1) / 2;
  const int lane = threadIdx.x;
  const int li = lane & 15, q = lane >> 4;
  const int64_t k0 = (int64_t)slice * kSlice;
  const int64_t k1 = min(len, k0 + (int64_t)kSlice);
  d4 acc[4][4];
  #pragma unroll
  for (int a = 0; a < 4; ++a)
    #pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k = k0; k < k1; k += 16) {
    double av[4][4], bv[4][4];
    #pragma unroll
    for (int t = 0; t < 4; ++t) {
      load4<P>(X, plane, (int64_t)I * kBlk + t * 16 + li, norb, len, k + 4 * q, av[t]);
      if (I != J) load4<P>(X, plane, (int64_t)J * kBlk + t * 16 + li, norb, len, k + 4 * q, bv[t]);
    }
    if (I == J) {
      #pragma unroll
      for (int t = 0; t < 4; ++t)
        #pragma unroll
        for (int s = 0; s < 4; ++s) bv[t][s] = av[t][s];
    }
    #pragma unroll
    for (int s = 0; s < 4; ++s)
      #pragma unroll
      for (int a = 0; a < 4; ++a)
        #pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][s], bv[c][s], acc[a][c], 0, 0, 0);
  }
  // tile element (i, j) is in lane j + 16 (i mod 4), register i / 4 (checked on the device)
  double* dst = part + ((int64_t)slice * nt + tri) * kBlk * kBlk;
  #pragma unroll
  for (int a = 0; a < 4; ++a)
    #pragma unroll
    for (int c = 0; c < 4; ++c)
      #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = a * 16 + q + 4 * v;
        const int col = c * 16 + li;
        dst[row * kBlk + col] = acc[a][c][v];
      }
}

// S[i][j] (and S[j][i]) = sum over slices in slice order.
__global__ void k_syrk_reduce(const double* __restrict__ part, int norb, int nslice,
                              double* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)norb * norb) return;
  const int i = (int)(idx / norb), j = (int)(idx % norb);
  if (j > i) return;
  const int nt = ntri(nblk64(norb));
  const int I = i / kBlk, J = j / kBlk;
  const int tri = I * (I + 1) / 2 + J;
  const int r = i % kBlk, c = j % kBlk;
  double s = 0.0;
  for (int q = 0; q < nslice; ++q) s += part[((int64_t)q * nt + tri) * kBlk * kBlk + r * kBlk + c];
  S[(int64_t)i * norb + j] = s;
  S[(int64_t)j * norb + i] = s;
}

// ---------------------------------------------------------------------------
// SYRK for up to 256 orbitals, one workgroup (8 waves) per coefficient slice.
// Chunks of 16 coefficients of every orbital are staged in LDS (double
// buffered: the next chunk's loads are in flight while the current one is
// multiplied), so HBM is read once; the lower triangle of S is cut into
// 32 x 32 blocks, dealt to the waves round-robin, each a 2 x 2 set of 16 x 16
// matrix-core tiles (a diagonal block skips its tile above the diagonal,
// which the reduction never reads).  Lane group q of step s takes
// coefficient 4 q + s of the chunk for both operands (the sum does not
// depend on the order).  Slice partials are summed in slice order by
// k_syrk32_reduce.
// ---------------------------------------------------------------------------
constexpr int kS32Waves = 8;
constexpr int kS32MaxBlocks = 5;     // ceil(36 / 8) blocks per wave at 256 orbitals
constexpr int kS32Pitch = 17;        // doubles per staged row (16 + 1: distinct banks)
constexpr int kS32Rows = 256;

__host__ __device__ inline int nblk32(int norb) { return (norb + 31) / 32; }

template <int P>
__global__ __launch_bounds__(512) void k_syrk32(const void* __restrict__ X, int64_t plane, int norb,
                                                int64_t len, int64_t slen, double* __restrict__ part) {
  using T = Prec<P>;
  __shared__ double lds[2][kS32Rows * kS32Pitch];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, q = lane >> 4;
  const int nb = nblk32(norb), nt = ntri(nb);
  const int rows = nb * 32;
  const int64_t k0 = (int64_t)blockIdx.x * slen;
  const int64_t k1 = min(len, k0 + slen);
  // staging: thread -> (row, half of the 16 coefficients)
  const int srow = tid >> 1, shalf = (tid & 1) * 8;
  double stage[8];
  auto fetch = [&](int64_t k) {
    if (srow < norb && k + shalf + 8 <= k1) {
      ld_run<P, 8>(X, plane, (int64_t)srow * len + k + shalf, stage);
      return;
    }
    #pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t kk = k + shalf + u;
      stage[u] = (srow < norb && kk < k1) ? T::d(T::ldc(X, (int64_t)srow * len + kk, plane)) : 0.0;
    }
  };
  auto put = [&](int buf) {
    if (srow < rows) {
      #pragma unroll
      for (int u = 0; u < 8; ++u) lds[buf][srow * kS32Pitch + shalf + u] = stage[u];
    }
  };
  // blocks of this wave: tri = w + 8 m -> (I, J), I >= J
  int bi[kS32MaxBlocks], bj[kS32MaxBlocks];
  #pragma unroll
  for (int m = 0; m < kS32MaxBlocks; ++m) {
    const int tri = w + kS32Waves * m;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= tri) ++I;
    bi[m] = I;
    bj[m] = tri - I * (I + 1) / 2;
  }
  d4 acc[kS32MaxBlocks][2][2];
  #pragma unroll
  for (int m = 0; m < kS32MaxBlocks; ++m)
    #pragma unroll
    for (int a = 0; a < 2; ++a)
      #pragma unroll
      for (int c = 0; c < 2; ++c) acc[m][a][c] = d4{0.0, 0.0, 0.0, 0.0};
  int buf = 0;
  if (k0 < k1) {
    fetch(k0);
    put(0);
  }
  __syncthreads();
  for (int64_t k = k0; k < k1; k += 16) {
    const bool more = k + 16 < k1;
    if (more) fetch(k + 16);                     // in flight during the products
    const double* L = lds[buf];
    #pragma unroll
    for (int m = 0; m < kS32MaxBlocks; ++m) {
      if (w + kS32Waves * m >= nt) break;
      const int I = bi[m], J = bj[m];
      #pragma unroll
      for (int s = 0; s < 4; ++s) {
        double av[2], bv[2];
        #pragma unroll
        for (int a = 0; a < 2; ++a) {
          av[a] = L[(I * 32 + a * 16 + li) * kS32Pitch + 4 * q + s];
          bv[a] = L[(J * 32 + a * 16 + li) * kS32Pitch + 4 * q + s];
        }
        #pragma unroll
        for (int a = 0; a < 2; ++a)
          #pragma unroll
          for (int c = 0; c < 2; ++c) {
            if (I == J && a == 0 && c == 1) continue;   // above the diagonal: never read
            acc[m][a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[m][a][c], 0, 0, 0);
          }
      }
    }
    if (more) put(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // tile element (i, j) is in lane j + 16 (i mod 4), register i / 4
  #pragma unroll
  for (int m = 0; m < kS32MaxBlocks; ++m) {
    const int tri = w + kS32Waves * m;
    if (tri >= nt) break;
    double* dst = part + ((int64_t)blockIdx.x * nt + tri) * 1024;
    #pragma unroll
    for (int a = 0; a < 2; ++a)
      #pragma unroll
      for (int c = 0; c < 2; ++c)
        #pragma unroll
        for (int v = 0; v < 4; ++v) dst[(a * 16 + q + 4 * v) * 32 + c * 16 + li] = acc[m][a][c][v];
  }
}

// S[i][j] (and S[j][i]) = sum over slices, in slice order.
__global__ void k_syrk32_reduce(const double* __restrict__ part, int norb, int nslice,
                                double* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)norb * norb) return;
  const int i = (int)(idx / norb), j = (int)(idx % norb);
  if (j > i) return;
  const int nt = ntri(nblk32(norb));
  const int I = i / 32, J = j / 32;
  const int tri = I * (I + 1) / 2 + J;
  const int r = i % 32, c = j % 32;
  double s = 0.0;
  for (int q = 0; q < nslice; ++q) s += part[((int64_t)q * nt + tri) * 1024 + r * 32 + c];
  S[(int64_t)i * norb + j] = s;
  S[(int64_t)j * norb + i] = s;
}

constexpr int kS32Slices = 256;      // one workgroup per CU

static int64_t syrk32_slice(int64_t len) {
  int64_t sl = (len + kS32Slices - 1) / kS32Slices;
  sl = (sl + 15) / 16 * 16;
  return sl < 16 ? 16 : sl;
}

static bool syrk32_used(int norb) { return norb <= kS32Rows; }

static int64_t syrk32_partials(int norb, int64_t len) {
  if (!syrk32_used(norb)) return 0;
  const int64_t sl = syrk32_slice(len);
  return ((len + sl - 1) / sl) * ntri(nblk32(norb)) * 1024;
}

template <int P>
static hipError_t overlap_p(const void* X, int64_t plane, int norb, int64_t len, double* S,
                            double* work, hipStream_t st) {
  if (syrk32_used(norb)) {
    const int64_t sl = syrk32_slice(len);
    const int nslice = (int)((len + sl - 1) / sl);
    hipLaunchKernelGGL((k_syrk32<P>), dim3((unsigned)nslice), dim3(512), 0, st, X, plane, norb, len,
                       sl, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n2 = (int64_t)norb * norb;
    hipLaunchKernelGGL(k_syrk32_reduce, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, work,
                       norb, nslice, S);
    return hipGetLastError();
  }
  const int nt = ntri(nblk64(norb));
  const int nslice = (int)((len + kSlice - 1) / kSlice);
  const int ngrp = (nslice + kXcd - 1) / kXcd;
  const int64_t nwg = (int64_t)ngrp * nt * kXcd;
  hipLaunchKernelGGL((k_syrk<P>), dim3((unsigned)nwg), dim3(64), 0, st, X, plane, norb, len, nslice,
                     work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n2 = (int64_t)norb * norb;
  hipLaunchKernelGGL(k_syrk_reduce, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, work, norb,
                     nslice, S);
  return hipGetLastError();
}

hipError_t launch_overlap_p(int prec, const void* X, int64_t plane, int norb, int64_t len,
                            double* S, double* work, hipStream_t st) {
  switch (prec) {
    case F64: return overlap_p<F64>(X, plane, norb, len, S, work, st);
    case F32: return overlap_p<F32>(X, plane, norb, len, S, work, st);
    default:  return overlap_p<F32C>(X, plane, norb, len, S, work, st);
  }
}

// ---------------------------------------------------------------------------
// Cholesky S = L L^T and Linv = L^{-1} (n <= 256) in one launch of one
// workgroup (8 waves); S, L and Linv stay in the L2 cache between the steps.
// Right-looking, by block columns J of 32, with the inverse built alongside
// as the solution Y of L Y = I by the same elimination (Linv holds the
// updated right-hand side R of the block rows not yet reached):
//  * the panel (rows r0.. of the block column) is staged in LDS;
//  * wave 0 factorises the diagonal block with its rows in registers (lane r
//    holds row r; each column of L is broadcast through LDS) and inverts it
//    by forward elimination alongside (lane c holds column c of inv(L_JJ));
//  * the panel below becomes L_IJ = S_IJ inv(L_JJ)^T;
//  * block row J of Linv: Y_J,K = inv(L_JJ) R_J,K (K < J), Y_J,J = inv(L_JJ);
//  * the rows below are updated: S_IK -= L_IJ L_KJ^T (trailing lower
//    triangle) and R_I,0:J+1 -= L_IJ Y_J,0:J+1.
// All products run on the float64 matrix cores from LDS operands; the
// read-modify-writes of S and R are batched four tiles at a time.  A
// non-positive pivot sets info[0] to its row + 1 (the first one only) and is
// replaced by 1.
// ---------------------------------------------------------------------------
constexpr int kCb = 32;                  // diagonal block
constexpr int kChPitch = 36;             // doubles per staged panel row
constexpr int kChRows = 256;             // panel rows staged (n <= 256)
constexpr int kChYPitch = kChRows + 4;   // doubles per staged row of Y_J
constexpr int kChThreads = 512;

__device__ __forceinline__ double rd_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// row and column tile of pair p of the lower triangle of nt x nt tiles
__device__ __forceinline__ void tri_pair(int p, int& it, int& kt) {
  it = 0;
  while ((it + 1) * (it + 2) / 2 <= p) ++it;
  kt = p - it * (it + 1) / 2;
}

__global__ __launch_bounds__(kChThreads) void k_chol_inv(double* __restrict__ A,
                                                         double* __restrict__ Li, int n,
                                                         int* __restrict__ info) {
  extern __shared__ double lds_chol[];
  double* pan = lds_chol;                          // kChRows x kChPitch
  double* dinv = pan + kChRows * kChPitch;         // kCb x kChPitch: inv(L_JJ)
  double* col = dinv + kCb * kChPitch;             // kCb: one column of L_JJ
  double* yb = col + kCb;                          // kCb x kChYPitch: Y_J,0:J+1
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NW = kChThreads / 64;
  const int li = lane & 15, q = lane >> 4;
  const int nb = (n + kCb - 1) / kCb;
  // R = 0 off the diagonal blocks (the diagonal blocks are written as found)
  for (int idx = tid; idx < n * n; idx += kChThreads) Li[idx] = 0.0;
  __syncthreads();
  for (int J = 0; J < nb; ++J) {
    const int r0 = J * kCb, b = min(kCb, n - r0), nr = n - r0;
    // panel rows 0..kChRows-1 (relative to r0): S values, the diagonal block
    // padded with the identity, zero below the matrix
    #pragma unroll 4
    for (int idx = tid; idx < kChRows * kCb; idx += kChThreads) {
      const int i = idx / kCb, c = idx - i * kCb;
      double v = (i == c) ? 1.0 : 0.0;
      if (i < nr && c < b) v = A[(int64_t)(r0 + i) * n + r0 + c];
      pan[i * kChPitch + c] = v;
    }
    __syncthreads();
    if (wave == 0) {
      // lane r: row r of the block (a) and column r of its inverse (x, by
      // forward elimination on the identity, one column of L at a time);
      // r is opaque so that nothing depending on it leaves the J loop
      int r = lane & (kCb - 1);
      asm volatile("" : "+v"(r));
      double a[kCb], x[kCb];
      #pragma unroll
      for (int c = 0; c < kCb; ++c) {
        a[c] = pan[r * kChPitch + c];
        x[c] = (c == r) ? 1.0 : 0.0;
      }
      #pragma unroll
      for (int j = 0; j < kCb; ++j) {
        double d = rd_lane(a[j], j);
        if (!(d > 0.0)) {
          if (lane == 0 && j < b && info[0] == 0) info[0] = r0 + j + 1;
          d = 1.0;
        }
        const double l = sqrt(d), il = 1.0 / l;
        // rows above j (r < j) hold the unused upper part: updated too, never read
        a[j] = (r == j) ? l : a[j] * il;
        // column j of L to every lane (LDS broadcast reads)
        if (lane < kCb) col[r] = a[j];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        x[j] *= il;
        double lk[kCb];
        #pragma unroll
        for (int k = j + 1; k < kCb; ++k) lk[k] = col[k];
        #pragma unroll
        for (int k = j + 1; k < kCb; ++k) {
          a[k] = __builtin_fma(-a[j], lk[k], a[k]);
          x[k] = __builtin_fma(-lk[k], x[j], x[k]);
        }
        // applied now: the updates are not deferred to their use (which
        // would hold every column in registers)
        #pragma unroll
        for (int k = j + 1; k < kCb; ++k) asm volatile("" : "+v"(a[k]), "+v"(x[k]));
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      if (lane < kCb) {
        #pragma unroll
        for (int c = 0; c < kCb; ++c) {
          pan[r * kChPitch + c] = c <= r ? a[c] : 0.0;
          dinv[c * kChPitch + r] = x[c];
        }
      }
    }
    __syncthreads();
    // the diagonal blocks of L and Linv to memory (L's upper part zero);
    // Y_J,J = inv(L_JJ) staged as columns r0.. of yb
    for (int idx = tid; idx < kCb * kCb; idx += kChThreads) {
      const int i = idx / kCb, c = idx - i * kCb;
      yb[i * kChYPitch + r0 + c] = dinv[i * kChPitch + c];
      if (i < b && c < b) {
        A[(int64_t)(r0 + i) * n + r0 + c] = pan[i * kChPitch + c];
        Li[(int64_t)(r0 + i) * n + r0 + c] = dinv[i * kChPitch + c];
      }
    }
    // block row J of Linv: Y_J,K = inv(L_JJ) R_J,K for the column tiles left
    // of the diagonal block (both row tiles of a column tile in one wave: the
    // tile is read whole before it is overwritten)
    for (int kt = wave; kt < (r0 >> 4); kt += NW) {
      double bv[kCb / 4];
      #pragma unroll
      for (int s = 0; s < kCb / 4; ++s) {
        const int m = 4 * s + q;
        bv[s] = m < b ? Li[(int64_t)(r0 + m) * n + 16 * kt + li] : 0.0;
      }
      #pragma unroll
      for (int it = 0; it < 2; ++it) {
        d4 y = d4{0.0, 0.0, 0.0, 0.0};
        #pragma unroll
        for (int s = 0; s < kCb / 4; ++s)
          y = __builtin_amdgcn_mfma_f64_16x16x4f64(dinv[(16 * it + li) * kChPitch + 4 * s + q], bv[s],
                                                   y, 0, 0, 0);
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * it + q + 4 * v;
          yb[row * kChYPitch + 16 * kt + li] = y[v];
          if (row < b) Li[(int64_t)(r0 + row) * n + 16 * kt + li] = y[v];
        }
      }
    }
    const int rem = nr - b;
    if (rem <= 0) break;
    const int nt = (rem + 15) >> 4;               // 16-row tiles below the diagonal block
    // panel: L_IJ = S_IJ inv(L_JJ)^T, tile (it, ct) -> rows b + 16 it, columns 16 ct
    d4 acc[4];
    #pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc[u] = d4{0.0, 0.0, 0.0, 0.0};
      const int tt = wave + u * NW;
      if (tt >= 2 * nt) continue;
      const int it = tt >> 1, ct = tt & 1;
      #pragma unroll
      for (int s = 0; s < kCb / 4; ++s) {
        const double av = pan[(b + 16 * it + li) * kChPitch + 4 * s + q];
        const double bw = dinv[(16 * ct + li) * kChPitch + 4 * s + q];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bw, acc[u], 0, 0, 0);
      }
    }
    __syncthreads();
    // element (i, j) of a tile: lane j + 16 (i mod 4), register i / 4
    #pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tt = wave + u * NW;
      if (tt >= 2 * nt) continue;
      const int it = tt >> 1, ct = tt & 1;
      #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = b + 16 * it + q + 4 * v, c = 16 * ct + li;
        pan[row * kChPitch + c] = acc[u][v];
        if (row < nr) A[(int64_t)(r0 + row) * n + r0 + c] = acc[u][v];
      }
    }
    __syncthreads();
    // rows below: tiles of the trailing lower triangle of S (pairs it >= kt)
    // and of R_I,0:J+1 (nt x ncy), four per wave at a time, each tile's
    // target read before the products
    const int npair = nt * (nt + 1) / 2, ncy = (r0 + kCb) >> 4;
    const int ntot = npair + nt * ncy;
    for (int t0 = wave; t0 < ntot; t0 += 4 * NW) {
      double cv[4][4];
      double* dst[4];
      int ti[4], tk[4];
      bool ys[4], ok[4];
      #pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int tt = t0 + u * NW;
        ok[u] = tt < ntot;
        ys[u] = tt >= npair;
        if (ys[u]) {
          ti[u] = (tt - npair) / ncy;
          tk[u] = (tt - npair) - ti[u] * ncy;
          dst[u] = Li + (int64_t)(r0 + b + 16 * ti[u]) * n + 16 * tk[u];
        } else {
          tri_pair(tt, ti[u], tk[u]);
          dst[u] = A + (int64_t)(r0 + b + 16 * ti[u]) * n + r0 + b + 16 * tk[u];
        }
        const int cmax = ys[u] ? n : nr - b - 16 * tk[u];
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = b + 16 * ti[u] + q + 4 * v;
          cv[u][v] = (ok[u] && row < nr && li < cmax) ? dst[u][(int64_t)(q + 4 * v) * n + li] : 0.0;
        }
      }
      #pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!ok[u]) continue;
        d4 t = d4{0.0, 0.0, 0.0, 0.0};
        #pragma unroll
        for (int s = 0; s < kCb / 4; ++s) {
          const double av = pan[(b + 16 * ti[u] + li) * kChPitch + 4 * s + q];
          const double bw = ys[u] ? yb[(4 * s + q) * kChYPitch + 16 * tk[u] + li]
                                  : pan[(b + 16 * tk[u] + li) * kChPitch + 4 * s + q];
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bw, t, 0, 0, 0);
        }
        const int cmax = ys[u] ? n : nr - b - 16 * tk[u];
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = b + 16 * ti[u] + q + 4 * v;
          if (row < nr && li < cmax) dst[u][(int64_t)(q + 4 * v) * n + li] = cv[u][v] - t[v];
        }
      }
    }
    __syncthreads();
  }
}

size_t chol_lds_bytes() {
  return sizeof(double) * ((size_t)kChRows * kChPitch + (size_t)kCb * kChPitch + kCb +
                           (size_t)kCb * kChYPitch);
}

// S (n x n, overwritten with L: lower triangle, zero upper part of the
// diagonal blocks), Linv (n x n, complete with zeros above the diagonal);
// info[0] = 0 on entry.
hipError_t launch_cholesky_inv(double* S, double* Linv, int n, int* info, hipStream_t st) {
  if (n > kChRows) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kChThreads), chol_lds_bytes(), st, S, Linv, n, info);
  return hipGetLastError();
}

__global__ void k_zero_upper_copy(const double* __restrict__ src, double* __restrict__ dst, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), k = (int)(idx % n);
  dst[idx] = (k <= i) ? src[idx] : 0.0;
}

hipError_t launch_chol_factor(const double* S, const double* Linv, int norb, double* L,
                              hipStream_t st) {
  const int64_t n2 = (int64_t)norb * norb;
  hipLaunchKernelGGL(k_zero_upper_copy, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, S, L,
                     norb);
  (void)Linv;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// X <- L^{-1} X for up to 256 orbitals, one 8-wave workgroup per slice of 64
// coefficients (columns).  Chunks of 16 rows of the slice are staged in LDS
// (double buffered, the next chunk and the next L^{-1} operands in flight
// during the products).  Wave w owns the row tiles w and 15 - w, so every
// wave does the same number of nonzero tile products of the triangle.  The
// results are written after the last chunk has been read (in place is safe:
// a workgroup only touches its own columns).
constexpr int kTr2Cols = 64;
constexpr int kTr2Pitch = 68;        // doubles per staged row: 2-way banks at most

template <int P>
__global__ __launch_bounds__(512) void k_trmm2(const double* __restrict__ Li, const void* X, void* Y,
                                               int64_t plane, int n, int64_t len) {
  using T = Prec<P>;
  __shared__ double lds[2][16 * kTr2Pitch];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, q = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * kTr2Cols;
  const int ntile = (n + 15) / 16;
  const int tiles[2] = {w, 15 - w};
  // staging: thread -> (row r of the chunk, two neighbouring columns)
  const int sr = tid >> 5, sc = (tid & 31) * 2;
  double xs[2];
  auto fetch = [&](int kc) {
    const int row = 16 * kc + sr;
    if (row < n && c0 + sc + 2 <= len) {
      ld_run<P, 2>(X, plane, (int64_t)row * len + c0 + sc, xs);
      return;
    }
    #pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t col = c0 + sc + u;
      xs[u] = (row < n && col < len) ? T::d(T::ldc(X, (int64_t)row * len + col, plane)) : 0.0;
    }
  };
  auto put = [&](int buf) {
    lds[buf][sr * kTr2Pitch + sc] = xs[0];
    lds[buf][sr * kTr2Pitch + sc + 1] = xs[1];
  };
  // L^{-1} operands of chunk kc: lane (li, q) step s takes column 16 kc + 4 q + s
  double an[2][4];
  // (the four values of a lane are consecutive in its row: two 16-byte loads
  // when they are inside the matrix and n is even, so that they are aligned)
  auto fetch_a = [&](int kc) {
    #pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int row = 16 * tiles[a] + li;
      const int k = 16 * kc + 4 * q;
      const bool act = tiles[a] >= kc && tiles[a] < ntile;
      if (act && row < n && k + 4 <= n && (n & 1) == 0) {
        const double2* p = reinterpret_cast<const double2*>(Li + (int64_t)row * n + k);
        const double2 x0 = p[0], x1 = p[1];
        an[a][0] = x0.x;
        an[a][1] = x0.y;
        an[a][2] = x1.x;
        an[a][3] = x1.y;
      } else {
        #pragma unroll
        for (int s = 0; s < 4; ++s)
          an[a][s] = (act && row < n && k + s < n) ? Li[(int64_t)row * n + k + s] : 0.0;
      }
    }
  };
  d4 acc[2][4];
  #pragma unroll
  for (int a = 0; a < 2; ++a)
    #pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  fetch_a(0);
  put(0);
  __syncthreads();
  int buf = 0;
  for (int kc = 0; kc < ntile; ++kc) {
    double av[2][4];
    #pragma unroll
    for (int a = 0; a < 2; ++a)
      #pragma unroll
      for (int s = 0; s < 4; ++s) av[a][s] = an[a][s];
    const bool more = kc + 1 < ntile;
    if (more) {
      fetch(kc + 1);
      fetch_a(kc + 1);
    }
    const double* L = lds[buf];
    #pragma unroll
    for (int s = 0; s < 4; ++s) {
      double bv[4];
      #pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = L[(4 * q + s) * kTr2Pitch + 16 * c + li];
      #pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (tiles[a] < kc || tiles[a] >= ntile) continue;
        #pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][s], bv[c], acc[a][c], 0, 0, 0);
      }
    }
    if (more) put(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // tile element (i, j) is in lane j + 16 (i mod 4), register i / 4
  #pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int ti = tiles[a];
    if (ti >= ntile) continue;
    #pragma unroll
    for (int c = 0; c < 4; ++c)
      #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * ti + q + 4 * v;
        const int64_t col = c0 + 16 * c + li;
        if (r < n && col < len) T::st(Y, (int64_t)r * len + col, plane, T::from_d(acc[a][c][v]));
      }
  }
}

hipError_t launch_trmm_rows_p(int prec, const double* Li, const void* X, void* Y, int64_t plane,
                              int norb, int64_t len, hipStream_t st) {
  if (norb > 256) return hipErrorInvalidValue;
  const int64_t nblk = (len + kTr2Cols - 1) / kTr2Cols;
  switch (prec) {
    case F64: hipLaunchKernelGGL((k_trmm2<F64>), dim3((unsigned)nblk), dim3(512), 0, st, Li, X, Y, plane, norb, len); break;
    case F32: hipLaunchKernelGGL((k_trmm2<F32>), dim3((unsigned)nblk), dim3(512), 0, st, Li, X, Y, plane, norb, len); break;
    default:  hipLaunchKernelGGL((k_trmm2<F32C>), dim3((unsigned)nblk), dim3(512), 0, st, Li, X, Y, plane, norb, len); break;
  }
  return hipGetLastError();
}

}  // namespace wvl
