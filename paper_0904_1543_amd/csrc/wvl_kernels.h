// Host-side launchers of the gfx950 kernels (internal to libwvl).
#pragma once

#include "wvl_internal.h"

namespace wvl {

// Deterministic block reduction of one double per thread (fixed order: wave
// butterfly, then the waves in index order); thread 0 stores.  Ends with a
// barrier so it can be called repeatedly.
__device__ __forceinline__ void block_sum_store(double v, double* dst) {
  __shared__ double red[kThreads / 64];
  #pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    #pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += red[w];
    *dst = t;
  }
  __syncthreads();
}

// One 1D pass of operator `op` along `axis` (1 = contiguous, 2, 3) for every
// orbital of the geometry.  k0 (nullable) is added to the result; epart
// (nullable, kinetic only) receives per-tile partial sums of x * (T x).
// out = CWT_z t + (kmul CK_z c + kxy), with the per-tile kinetic energies
// <c, CK_z c> in epart (nullable); z lines, tiling of the z passes
hipError_t launch_zfinal(int prec, const PassGeom& g, int ntiles, const void* t, const void* c,
                         const void* kxy, void* out, int64_t plane, double kmul, double* epart,
                         hipStream_t st);
hipError_t launch_pass(int prec, int op, int axis, const PassGeom& g, int ntiles, const void* in,
                       void* out, const void* k0, int64_t plane, double kmul, double* epart,
                       hipStream_t st);

// Pointwise stage on a shared potential (all orbitals on one grid of M points):
// rho (nullable) = [rho +] sum_b f_b psi_b^2 in float64; y_b = pot_scale V psi_b
// (nullable y); rvpart[block] = sum over the block of V * (sum_b f_b psi_b^2);
// ppart (nullable) [b][block] = sum over the block of V psi_b^2.
hipError_t launch_pot_shared(int prec, const OrbDev* orbs, int norb, int64_t M, const void* psi,
                             void* y, const double* V, double pot_scale, int64_t plane,
                             double* rho, int rho_acc, double* rvpart, double* ppart,
                             hipStream_t st);

// Pointwise stage with one potential per orbital (uneven batches):
// y_b = pot_scale V_b psi_b, ppart[tile] = sum over the tile of V_b psi_b^2.
hipError_t launch_pot_orb(int prec, const PassGeom& g, int ntiles, const void* psi, void* y,
                          const double* V, double pot_scale, int64_t plane, double* ppart,
                          hipStream_t st);

// x_b <- mul * f_b * x_b over every orbital (tiles of kThreads points, prefix g)
hipError_t launch_scale_occ(int prec, const PassGeom& g, int ntiles, void* x, double mul,
                            int64_t plane, hipStream_t st);

// Preconditioner: vector stages of the conjugate-gradient iteration (see
// wvl_precond.hip).  g: tiles of cg_tile_elems() points (prefix pc); sc:
// per-orbital scalars (cg_scalar_bytes() each); partial arrays: one double
// per tile.
size_t cg_scalar_bytes();
int cg_tile_elems();
hipError_t launch_cg_init(int prec, const PassGeom& g, int ntiles, const void* gin, void* x,
                          void* r, void* p, const double* eps, int64_t plane, double* prz,
                          double* ppp, double* prr, hipStream_t st);
hipError_t launch_cg_alpha(int norb, const int32_t* pz, const int32_t* py, const int32_t* px,
                           const int32_t* pp, const double* ez, const double* ey, const double* ex,
                           const double* prz, const double* ppp, const double* eps, void* sc,
                           hipStream_t st);
hipError_t launch_cg_update1(int prec, const PassGeom& g, int ntiles, void* x, void* r,
                             const void* p, const void* q, const double* eps, int shift,
                             const void* sc, int64_t plane, double* prz, double* prr,
                             hipStream_t st);
hipError_t launch_cg_beta(int norb, const int32_t* pp, const double* prz, void* sc, hipStream_t st);
hipError_t launch_cg_update2(int prec, const PassGeom& g, int ntiles, const void* r, void* p,
                             const double* eps, const void* sc, int64_t plane, double* ppp,
                             hipStream_t st);
hipError_t launch_cg_shift(int prec, const PassGeom& g, int ntiles, const void* s, void* k0,
                           const double* eps, int64_t plane, hipStream_t st);
hipError_t launch_cg_res(int norb, const int32_t* pp, const double* prr, double* res,
                         hipStream_t st);

// 1D pass with isolated or periodic boundary conditions (wvl_bc.hip) on a
// uniform batch: input arrays (n3, n2, n1) with the pass axis of length n_in,
// output the same with n_out; y[k] = sum_o F(o) x[k + d - o], zero outside the
// input (isolated) or wrapped (periodic, d = 0, n_in = n_out).  Batch stride
// vol_in / vol_out; `tiles` tiles per orbital (256 lines, or rows_per_tile
// rows along axis 1); k0 (nullable) is in the output shape, with its own
// plane stride.
struct BcPass {
  const OrbDev* orbs;
  int32_t orbs_n;
  int32_t n1, n2, n3;      // dims of the arrays along the axes other than the pass
  int32_t n_in, n_out, d;
  int32_t periodic;
  int64_t vol_in, vol_out;
  int32_t tiles, rows_per_tile;
  int64_t plane_k0;        // compensated float32: plane stride of k0
};
int bc_rows_per_tile(int op, int n_out);
hipError_t launch_bc_pass(int prec, int op, int axis, const BcPass& g, const void* in, void* out,
                          const void* k0, int64_t plane_in, int64_t plane_out, double kmul,
                          double* epart, hipStream_t st);

// Compressed storage (wvl_compress.hip): uniform batch of norb orbitals of M
// points; compressed vectors of L = nvc + 7 nvf values at b * L.
hipError_t launch_decompress(int prec, const OrbDev* orbs, int norb, int64_t M,
                             const int32_t* map_c, const int32_t* map_f, int64_t nvc, int64_t L,
                             const void* in, int64_t plane_in, void* out, int64_t plane_out,
                             hipStream_t st);
hipError_t launch_compress(int prec, const OrbDev* orbs, int norb, const int32_t* list_c,
                           const int32_t* list_f, int64_t nvc, int64_t L, const void* in,
                           int64_t plane_in, void* out, int64_t plane_out, hipStream_t st);

// Per-orbital energies eorb[b] (potential) and eorb[norb + b] (kinetic) from
// the tile partials; pot_mode 0: none, 1: per-orbital tiles (prefix pp),
// 2: shared-grid blocks laid out [norb][nblk].
hipError_t launch_orb_sums(const OrbDev* orbs, int norb, const int32_t* pz, const int32_t* py,
                           const int32_t* px, const double* ez, const double* ey, const double* ex,
                           const double* ppart, int pot_mode, const int32_t* pp, int nblk,
                           double* eorb, hipStream_t st);

// Totals: e_kin = sum_b f_b eorb[norb+b]; e_loc = sum of rvpart (nrv > 0) or
// sum_b f_b eorb[b].
hipError_t launch_totals(const OrbDev* orbs, int norb, const double* eorb, const double* rvpart,
                         int nrv, double* e_loc, double* e_kin, hipStream_t st);

// Element-wise format conversion between F64, F32 and F32C (hi/lo planes).
hipError_t launch_convert(const void* src, int sp, void* dst, int dp, int64_t n, hipStream_t st);

// Fill with a float64 value (used instead of memset nodes so that sequences
// can be captured in graphs).
hipError_t launch_fill(double* dst, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_int(int32_t* dst, int n, hipStream_t st);

// In-plane part of the local Hamiltonian (one z-plane per workgroup):
// psi = W_x W_y u, rho/e_pot, t = W_y^T W_x^T (pot_scale V psi),
// kxy = kin_mul (K_x + K_y) c.  See wvl_xy.hip.
struct XyArgs {
  const OrbDev* orbs;
  const int32_t* pq;     // plane prefix: slot of (b, z) is pq[b] + z
  int32_t norb;
  int32_t shared;        // shared potential: orbital groups of G, rho partials
  int32_t ngroups, G;
  int64_t M;             // points of the shared grid
  const void* u;
  const void* c;
  void* t;
  void* kxy;
  const double* V;
  double pot_scale, kin_mul;
  int64_t plane;
  double* rho_part;      // [ngroups][M] (shared) or nullptr
  double* epot;          // per (orbital, plane)
  double* ekin;          // per (orbital, plane): <c, (K_x + K_y) c> over the plane
  int32_t occupancy;     // waves per SIMD the kernel is compiled for (2 or 4)
  int32_t slot;          // shared: orbital g * G + slot of every group g; -1: all slots in turn
  int32_t engine;        // 0: vector FMA passes, 1: float64 matrix-core passes
  int32_t rho_lds;       // shared, matrix engine, 2 waves per SIMD: the group's
                         // density plane kept in LDS (set by launch_xy)
  // persistent launch of the unshared path (queue != nullptr): planes taken
  // from the queue in the order of `order` (prefix of planes over perm)
  const int32_t* order;
  const int32_t* perm;
  int32_t* queue;
  int32_t ntiles;
};
// In-plane part of the preconditioner's operator: kq += (K_x + K_y) p for
// every (orbital, z-plane) (one workgroup each, slots pq[b] + z), with
// ekin[slot] = <p, (K_x + K_y) p> over the plane.
struct HelmArgs {
  const OrbDev* orbs;
  const int32_t* pq;
  int32_t norb;
  const void* p;
  void* kq;
  int64_t plane;
  double* ekin;
};
hipError_t launch_helm_xy(int prec, const HelmArgs& a, int m1, int m2, int nblocks, bool engine,
                          hipStream_t st);

// engine: the float64 matrix-core form of the in-plane passes
bool xy_matrix_engine(int prec, int m1, int m2);
// Exact-product engine of the compensated form (wvl_oz.hip): uniform batches
// with a shared potential, fine lengths multiples of 16.  Float pairs: hi
// plane then lo plane, `plane` floats apart.
struct OzArgs {
  const OrbDev* orbs;
  int32_t norb, m1, m2, m3;
  const float* c;
  float* out;
  float* t;
  float* u;
  float* kxy;
  int64_t plane;
  const float* vhl;      // the potential as float pairs (hi, then lo M floats later)
  const int* vexp;       // per z-plane exponent of max |V|
  int64_t M;
  int32_t pexp;          // |pot_scale| <= 2^pexp
  float ps_hi, ps_lo;    // pot_scale as a float pair
  int32_t ps_scaled;     // pot_scale != 1
  double kin_mul;        // kin_scale
  double* rho_part;      // [ngroups][M] group partials
  int32_t ngroups, G;
  double* epot;          // per (orbital, z-plane) at pq[b] + z
  const int32_t* pq;
  double* ekin;          // per (orbital, y) at b * m2 + y: <c, k (K_x + K_y + K_z) c>
  int32_t dxy, dz;       // digit-plane strides (bytes) of the xy and xz kernels
};
// The preconditioner's operator with the exact products (same batches
// without the potential): q = k K p, e per xz-plane (K_z) and per z-plane.
struct OzHelmArgs {
  const OrbDev* orbs;
  int32_t norb, m1, m2, m3;
  const float* p;
  float* q;
  int64_t plane;
  double* ez;            // <p, k K_z p> per (orbital, y) at b * m2 + y
  double* exy;           // <p, k (K_x + K_y) p> per (orbital, z) at b * m3 + z
  int32_t dxy, dz;
};
hipError_t launch_oz_helm(const OzHelmArgs& a, hipStream_t st);
struct OzLds { int dxy, dz; size_t xy_bytes, z_bytes; };
OzLds oz_lds(int m1, int m2, int m3);
bool oz_supported(int m1, int m2, int m3);
hipError_t launch_oz_vprep(const double* V, int npl, int m3, float* vhl, int64_t M, int* vexp,
                           hipStream_t st);
hipError_t launch_oz_z(const OzArgs& a, hipStream_t st);
hipError_t launch_oz_xy(const OzArgs& a, hipStream_t st);
hipError_t launch_oz_zfinal(const OzArgs& a, int occ, hipStream_t st);

size_t xy_lds_bytes(int prec, int m1, int m2, bool engine);
bool xy_supported(int prec, int m1, int m2, bool engine);
// m1, m2: the plane of every orbital of the launch (the largest one for uneven
// batches; LDS is sized for it)
hipError_t launch_xy(int prec, const XyArgs& a, int m1, int m2, int nblocks, hipStream_t st);
hipError_t launch_rho_reduce(const double* part, int ngroups, int64_t M, const double* V,
                             double* rho, double* rvpart, hipStream_t st);

// Overlap S = X X^T (X: norb rows of `len` coefficients stored in precision
// `prec`, plane stride `plane`), Cholesky S = L L^T with L^{-1}, and
// Y = L^{-1} X.  syrk_partials: workspace of the overlap in doubles.
int64_t syrk_partials(int norb, int64_t len);
hipError_t launch_overlap_p(int prec, const void* X, int64_t plane, int norb, int64_t len,
                            double* S, double* work, hipStream_t st);
// Blocked Cholesky (n <= 256, one launch): S (n x n) overwritten with L
// (upper part not touched except the diagonal blocks), Linv = L^{-1} (n x n,
// zero above the diagonal); info[0] = first non-positive pivot row + 1.
hipError_t launch_cholesky_inv(double* S, double* Linv, int n, int* info, hipStream_t st);
// L output: the lower triangle of the factorised S.
hipError_t launch_chol_factor(const double* S, const double* Linv, int norb, double* L,
                              hipStream_t st);
hipError_t launch_trmm_rows_p(int prec, const double* Li, const void* X, void* Y, int64_t plane,
                              int norb, int64_t len, hipStream_t st);

}  // namespace wvl
