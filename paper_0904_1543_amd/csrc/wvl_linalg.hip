// Orbital overlap matrix and Cholesky orthonormalisation in float64, gfx950.
//
// Sec. 2.6 and Sec. 5 (step VIII): scalar products between orbitals are taken
// directly on the coefficients because the basis is orthonormal; the overlap
// matrix S = X X^T (X: one row of coefficients per orbital) is factorised as
// S = L L^T and the orbitals are replaced by the rows of L^{-1} X.  The paper
// runs the SYRK on the GPU and the factorisation on the host; here everything
// stays on the GPU:
//  * SYRK on the float64 matrix cores (v_mfma_f64_16x16x4f64): each workgroup
//    takes a slice of the coefficient axis, stages 256 orbitals x 8
//    coefficients at a time in LDS and accumulates one 64x64 block of S per wave; the
//    slices' partial matrices are summed in a fixed order (deterministic);
//  * Cholesky and the triangular inverse: one workgroup, right-looking, the
//    matrix held in global memory (it fits in L2);
//  * X <- L^{-1} X on the matrix cores, skipping the zero blocks of L^{-1}.

#include "wvl_kernels.h"

namespace wvl {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kSyrkRows = 256;   // orbitals per row block
constexpr int kSyrkK = 8;        // coefficients staged per step
constexpr int kSyrkPitch = kSyrkK + 1;
constexpr int kSyrkSlice = 4096; // coefficients per workgroup

int64_t syrk_partials(int norb, int64_t len) {
  const int64_t nslice = (len + kSyrkSlice - 1) / kSyrkSlice;
  const int64_t nb = (norb + kSyrkRows - 1) / kSyrkRows;
  return nslice * nb * nb * kSyrkRows * kSyrkRows;
}

// One workgroup: rows [I*256, +256) x cols [J*256, +256) of S over coefficient
// slice `blockIdx.x`; 16 waves, wave w owns the 64x64 sub-block (w/4, w%4).
template <int P>
__global__ __launch_bounds__(1024) void k_syrk(const void* __restrict__ X, int64_t plane, int norb,
                                               int64_t len, double* __restrict__ part) {
  using T = Prec<P>;
  __shared__ double A[kSyrkRows * kSyrkPitch];
  __shared__ double B[kSyrkRows * kSyrkPitch];
  const int nb = (norb + kSyrkRows - 1) / kSyrkRows;
  const int I = blockIdx.y / nb, J = blockIdx.y % nb;
  const int64_t k0 = (int64_t)blockIdx.x * kSyrkSlice;
  const int64_t k1 = min(len, k0 + (int64_t)kSyrkSlice);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wid >> 2, wc = wid & 3;
  d4 acc[4][4];
  #pragma unroll
  for (int a = 0; a < 4; ++a)
    #pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t kb = k0; kb < k1; kb += kSyrkK) {
    // stage 256 rows x 32 coefficients of the I and J row blocks
    for (int e = threadIdx.x; e < kSyrkRows * kSyrkK; e += 1024) {
      const int r = e / kSyrkK, c = e % kSyrkK;
      const int64_t kk = kb + c;
      const int ra = I * kSyrkRows + r, rb = J * kSyrkRows + r;
      A[r * kSyrkPitch + c] = (ra < norb && kk < k1) ? T::d(T::ldc(X, (int64_t)ra * len + kk, plane)) : 0.0;
      B[r * kSyrkPitch + c] = (rb < norb && kk < k1) ? T::d(T::ldc(X, (int64_t)rb * len + kk, plane)) : 0.0;
    }
    __syncthreads();
    #pragma unroll
    for (int ks = 0; ks < kSyrkK; ks += 4) {
      double av[4], bv[4];
      // operand layouts: A tile 16x4 -> lane = i + 16 k; B tile 4x16 -> lane = j + 16 k
      #pragma unroll
      for (int t = 0; t < 4; ++t) {
        av[t] = A[(wr * 64 + t * 16 + (lane & 15)) * kSyrkPitch + ks + (lane >> 4)];
        bv[t] = B[(wc * 64 + t * 16 + (lane & 15)) * kSyrkPitch + ks + (lane >> 4)];
      }
      #pragma unroll
      for (int a = 0; a < 4; ++a)
        #pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
    }
    __syncthreads();
  }
  // result layout of a 16x16 tile (checked on the device): element (i, j) is in
  // lane j + 16 (i mod 4), register i / 4

  double* dst = part + ((int64_t)blockIdx.x * nb * nb + blockIdx.y) * kSyrkRows * kSyrkRows;
  #pragma unroll
  for (int a = 0; a < 4; ++a)
    #pragma unroll
    for (int c = 0; c < 4; ++c)
      #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + a * 16 + (lane >> 4) + 4 * v;
        const int col = wc * 64 + c * 16 + (lane & 15);
        dst[row * kSyrkRows + col] = acc[a][c][v];
      }
}

// S[i][j] = sum over slices, fixed order; writes the full symmetric matrix.
__global__ void k_syrk_reduce(const double* __restrict__ part, int norb, int nslice,
                              double* __restrict__ S) {
  const int nb = (norb + kSyrkRows - 1) / kSyrkRows;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)norb * norb) return;
  const int i = (int)(idx / norb), j = (int)(idx % norb);
  const int I = i / kSyrkRows, J = j / kSyrkRows;
  const int64_t blk = (int64_t)I * nb + J;
  const int r = i % kSyrkRows, c = j % kSyrkRows;
  double s = 0.0;
  for (int q = 0; q < nslice; ++q)
    s += part[((int64_t)q * nb * nb + blk) * kSyrkRows * kSyrkRows + r * kSyrkRows + c];
  S[idx] = s;
}

template <int P>
static hipError_t overlap_p(const void* X, int64_t plane, int norb, int64_t len, double* S,
                            double* work, hipStream_t st) {
  const int nb = (norb + kSyrkRows - 1) / kSyrkRows;
  const int nslice = (int)((len + kSyrkSlice - 1) / kSyrkSlice);
  hipLaunchKernelGGL((k_syrk<P>), dim3(nslice, nb * nb), dim3(1024), 0, st, X, plane, norb, len, work);
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
// Cholesky S = L L^T (lower, in place) and Linv = L^{-1}; one workgroup.
// info[0] = 0 on success, j+1 if the j-th pivot is not positive.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_cholesky_inv(double* S, double* Li, int n, int* info) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int tid = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = S[(int64_t)j * n + j];
      if (!(d > 0.0)) { if (!bad) bad = j + 1; S[(int64_t)j * n + j] = 1.0; }
      else S[(int64_t)j * n + j] = sqrt(d);
    }
    __syncthreads();
    const double djj = S[(int64_t)j * n + j];
    for (int i = j + 1 + tid; i < n; i += 1024) S[(int64_t)i * n + j] /= djj;
    __syncthreads();
    const int ti = tid >> 5, tk = tid & 31;
    for (int i = j + 1 + ti; i < n; i += 32) {
      const double sij = S[(int64_t)i * n + j];
      for (int k = j + 1 + tk; k <= i; k += 32) S[(int64_t)i * n + k] -= sij * S[(int64_t)k * n + j];
    }
    __syncthreads();
  }
  // zero the strict upper triangle so that S holds exactly L
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    const int i = (int)(e / n), k = (int)(e % n);
    if (k > i) S[e] = 0.0;
  }
  __syncthreads();
  // Linv: row by row, Li[i][c] = (delta_ic - sum_{k=c}^{i-1} L[i][k] Li[k][c]) / L[i][i]
  for (int i = 0; i < n; ++i) {
    const double lii = S[(int64_t)i * n + i];
    for (int c = tid; c < n; c += 1024) {
      double v = 0.0;
      if (c <= i) {
        double s = (c == i) ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) s -= S[(int64_t)i * n + k] * Li[(int64_t)k * n + c];
        v = s / lii;
      }
      Li[(int64_t)i * n + c] = v;
    }
    __syncthreads();
  }
  if (tid == 0) info[0] = bad;
}

hipError_t launch_cholesky_inv(double* S_to_L, double* Linv, int norb, int* info, hipStream_t st) {
  hipLaunchKernelGGL(k_cholesky_inv, dim3(1), dim3(1024), 0, st, S_to_L, Linv, norb, info);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Y = Linv X (rows = orbitals); Linv lower triangular.  Workgroup: all rows x
// 16 coefficients; 16 waves, wave w owns output row tiles {w, w+16, ...} of 16
// rows.  Y may alias X (each workgroup reads its
// columns into LDS before writing).
// ---------------------------------------------------------------------------
constexpr int kTrCols = 16;

template <int P>
__global__ __launch_bounds__(1024) void k_trmm(const double* __restrict__ Li, const void* X,
                                               void* Y, int64_t plane, int norb, int64_t len) {
  using T = Prec<P>;
  extern __shared__ double sx[];  // [nrow_pad][kTrCols + 1]
  const int npad = (norb + 15) & ~15;
  const int pitch = kTrCols + 1;
  const int64_t c0 = (int64_t)blockIdx.x * kTrCols;
  for (int e = threadIdx.x; e < npad * kTrCols; e += 1024) {
    const int r = e / kTrCols, c = e % kTrCols;
    const int64_t cc = c0 + c;
    sx[r * pitch + c] = (r < norb && cc < len) ? T::d(T::ldc(X, (int64_t)r * len + cc, plane)) : 0.0;
  }
  __syncthreads();
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ntile = npad / 16;
  for (int ti = wid; ti < ntile; ti += 16) {
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    const int row = ti * 16 + (lane & 15);
    // only k < (ti+1)*16 contribute (Linv is lower triangular)
    for (int k = 0; k < (ti + 1) * 16; k += 4) {
      const int kk = k + (lane >> 4);
      const double a = (row < norb && kk < norb) ? Li[(int64_t)row * norb + kk] : 0.0;
      const double bv = sx[kk * pitch + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
    }
    #pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = ti * 16 + (lane >> 4) + 4 * v;
      const int64_t ca = c0 + (lane & 15);
      if (r < norb && ca < len) T::st(Y, (int64_t)r * len + ca, plane, T::from_d(acc[v]));
    }
  }
}

template <int P>
static hipError_t trmm_p(const double* Li, const void* X, void* Y, int64_t plane, int norb,
                         int64_t len, hipStream_t st) {
  const int npad = (norb + 15) & ~15;
  const size_t lds = (size_t)npad * (kTrCols + 1) * sizeof(double);
  const int64_t nblk = (len + kTrCols - 1) / kTrCols;
  hipLaunchKernelGGL((k_trmm<P>), dim3((unsigned)nblk), dim3(1024), lds, st, Li, X, Y, plane, norb, len);
  return hipGetLastError();
}

hipError_t launch_trmm_rows_p(int prec, const double* Li, const void* X, void* Y, int64_t plane,
                              int norb, int64_t len, hipStream_t st) {
  switch (prec) {
    case F64: return trmm_p<F64>(Li, X, Y, plane, norb, len, st);
    case F32: return trmm_p<F32>(Li, X, Y, plane, norb, len, st);
    default:  return trmm_p<F32C>(Li, X, Y, plane, norb, len, st);
  }
}

}  // namespace wvl
