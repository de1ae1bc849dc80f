/* wvl.h -- C ABI of libwvl: the local Hamiltonian of the Daubechies-wavelet
 * Kohn-Sham method (Genovese et al., "Density Functional Theory calculation on
 * many-cores hybrid CPU-GPU architectures") on one AMD MI355X (gfx950) GPU.
 *
 * Conventions common to every call
 * --------------------------------
 * Grids.  One orbital lives on a periodic coarse grid of n1 x n2 x n3 points
 * (axis 1 fastest).  Its fine grid (spacing h/2, Sec. 2.1, Eq. "wavefhigh")
 * has m_a = 2 n_a points per axis and is stored as a C-order (m3, m2, m1)
 * array.  Coarse coefficients (one scaling + seven wavelet components per
 * coarse point, Sec. 2.1, Eq. "wavef0") use the same (m3, m2, m1) array with
 * the two levels interleaved along every axis: along axis a, index 2i holds
 * the scaling part and 2i+1 the wavelet part of coarse point i; component
 * mu = b1 + 2 b2 + 4 b3 of coarse point (i1, i2, i3) sits at
 * (2 i3 + b3, 2 i2 + b2, 2 i1 + b1).  Boundary conditions are periodic
 * (Sec. 3.1).
 *
 * Batches.  A plan describes a batch of orbitals (Sec. 5.1: every orbital is
 * processed independently).  Batch arrays are packed buffers: orbital b
 * occupies elements [off_b, off_b + m1 m2 m3).  The element type depends on
 * the plan precision: WVL_F64 -> double; WVL_F32 -> float; WVL_F32C -> two
 * float planes, hi then lo, each of wvl_plan_elements() elements (value =
 * hi + lo).  Potentials, densities, energies and overlap matrices are always
 * double.
 *
 * Memory.  Every data pointer is a DEVICE pointer owned by the caller; the
 * library neither frees nor keeps it after the call returns (except the graph
 * cache of WVL_USE_GRAPH, which records pointers and re-records when they
 * change).  Batch arrays start on a 16-byte boundary (WVL_EINVAL otherwise;
 * hipMalloc and torch allocations are).  `ws` is caller-owned device
 * workspace of wvl_plan_workspace() bytes (256-byte aligned).  `stream` is a
 * hipStream_t (NULL = default stream).
 *
 * Errors.  Every call returns a wvl_status.  Arguments are checked before any
 * HIP call is made; HIP failures map to WVL_EHIP.  Calls are asynchronous on
 * `stream`; device-side failures (a non-positive pivot in the Cholesky step)
 * are reported by wvl_plan_sync().  wvl_last_error() returns a thread-local
 * message about the last failure.  No call aborts the process.
 */
#ifndef WVL_PUBLIC_API_H_
#define WVL_PUBLIC_API_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WVL_OK = 0,
  WVL_EINVAL = -1,       /* bad argument (null pointer, bad size, aliasing ...) */
  WVL_EUNSUPPORTED = -2, /* valid but not supported by this plan              */
  WVL_ENOMEM = -3,       /* device allocation failed (forced for every device
                            allocation of the library when the environment
                            variable WVL_DEBUG_FAIL_ALLOC is 1)               */
  WVL_EHIP = -4,         /* HIP runtime error                                  */
  WVL_ETIMEOUT = -5,     /* reserved: no call waits on the device (work-queue
                            kernels take tiles with atomics and never wait for
                            one another), so none returns it                  */
  WVL_ENODEV = -6        /* no usable GPU (also: dry plans on a host)          */
} wvl_status;

typedef enum { WVL_F64 = 0, WVL_F32 = 1, WVL_F32C = 2 } wvl_prec;

/* plan flags */
#define WVL_SHARED_V   1u  /* all orbitals share one potential (and one grid)   */
#define WVL_USE_GRAPH  2u  /* record wvl_local_hpsi in a hipGraph and replay it  */
/* WVL_PERSISTENT: every pass launch of wvl_local_hpsi (z, y and x passes,
 * the per-orbital potential stage and, without WVL_SHARED_V, the in-plane
 * kernel) runs as a persistent launch: a fixed number of workgroups take
 * tiles from a work queue, largest orbitals first (longest-processing-time-
 * first order), which balances batches of uneven orbitals.  The queue
 * counters live in the workspace, so calls that share a workspace must not
 * overlap.
 * WVL_AUTOTUNE: at plan creation, time the launch-sequence candidates of
 * wvl_local_hpsi on the plan's own batch (temporary device buffers of about
 * three batch arrays plus the workspace) and keep the fastest; see
 * wvl_plan_tuning. */
#define WVL_PERSISTENT 4u  /* persistent, work-queue launches (see above)        */
#define WVL_AUTOTUNE   8u  /* time the launch candidates at plan creation       */
/* Boundary conditions (Sec. 3.1; periodic when neither flag is set).
 * WVL_FREE_BC: isolated along every axis; WVL_SURFACE_BC: isolated along
 * axis 2, periodic along axes 1 and 3 (a slab).  Along an isolated axis the
 * orbital has its m = 2n coefficients and nothing outside the box; the
 * synthesis spreads them over m + 14 fine scaling coefficients and the magic
 * filter over m + 29 real-space points, global positions -14 .. m + 14 of the
 * fine grid (position 0: the first coefficient).  V and rho live on that
 * real-space grid (wvl_plan_grid_points() points, C order (M3, M2, M1) with
 * M_a = m_a + 29 along isolated axes).  Such plans need WVL_SHARED_V and a
 * dense uniform batch; they run wvl_local_hpsi, wvl_local_density,
 * wvl_energy_gradient, wvl_precondition (combined-filter form), the overlap
 * and orthonormalisation and the compressed-storage calls, with one 1D pass
 * per axis and operator (no plane kernel, no persistent launches, no tuner);
 * wvl_synthesis, wvl_analysis, wvl_magic_filter and wvl_kinetic are
 * periodic only (WVL_EUNSUPPORTED). */
#define WVL_FREE_BC    16u
#define WVL_SURFACE_BC 32u

typedef struct {
  int32_t n[3];     /* coarse dims n1, n2, n3 (>= 2 each); fine dims are 2n     */
  int32_t reserved; /* must be 0                                               */
  int64_t off;      /* element offset of the orbital in packed batch buffers   */
  int64_t v_off;    /* element offset of its potential (ignored with SHARED_V) */
  double hgrid[3];  /* fine grid spacing per axis (> 0)                         */
  double occ;       /* occupation number f_i                                    */
} wvl_orbital;

typedef struct wvl_ctx wvl_ctx;
typedef struct wvl_plan wvl_plan;

/* Library context on GPU `device`.  device = -1 creates a "dry" context with
 * no GPU: plans can be created and every argument check runs, but every call
 * that would touch the GPU returns WVL_ENODEV.  Returns WVL_ENODEV if the GPU
 * does not exist. */
int wvl_create(wvl_ctx **ctx, int device);
int wvl_destroy(wvl_ctx *ctx);

/* Plan for a batch of `norb` orbitals in precision `prec`.  Copies the
 * descriptor table to the device and fixes the tiling.  Requirements: n_a >= 2,
 * orbitals do not overlap in the packed buffers; with WVL_SHARED_V all
 * orbitals have the same dims.  wvl_overlap/wvl_orthonormalize need
 * off_b = b * m1 m2 m3 (a dense [norb][M] matrix). */
int wvl_plan_create(wvl_ctx *ctx, const wvl_orbital *orbs, int32_t norb, int32_t prec,
                    uint32_t flags, wvl_plan **plan);
int wvl_plan_destroy(wvl_plan *plan);
/* bytes of workspace every call of this plan needs */
int wvl_plan_workspace(const wvl_plan *plan, size_t *bytes);
/* elements of one packed batch array (per plane for WVL_F32C) */
int wvl_plan_elements(const wvl_plan *plan, int64_t *elems);
/* points of the shared grid (WVL_SHARED_V plans), the length of V and rho */
int wvl_plan_grid_points(const wvl_plan *plan, int64_t *points);

/* Fast wavelet transform, coarse -> fine scaling coefficients (Sec. 2.1 and
 * Sec. 2.4 step 2): per axis s[(2i + j) mod m] += h_j c_i + g_j d_i.
 * `s` must not overlap `c` (WVL_EINVAL). */
int wvl_synthesis(wvl_plan *plan, const void *c, void *s, void *ws, void *stream);

/* Inverse transform (Sec. 2.4 step 6): c_i = sum_j h_j s[(2i+j) mod m],
 * d_i = sum_j g_j s[(2i+j) mod m].  `c` must not overlap `s` (WVL_EINVAL). */
int wvl_analysis(wvl_plan *plan, const void *s, void *c, void *ws, void *stream);

/* Magic filter (Sec. 2.3, Eq. "magicfilter"): out[I] = sum_l w_l in[I-l] per
 * axis; with transpose != 0 the transposed filter out[i] = sum_l w_l in[i+l]
 * (Sec. 2.4 step 3c).  `out` must not overlap `in` (WVL_EINVAL). */
int wvl_magic_filter(wvl_plan *plan, const void *in, void *out, int transpose, void *ws,
                     void *stream);

/* Kinetic operator -1/2 nabla^2 on fine scaling coefficients (Sec. 2.2,
 * Eqs. "kiner", "fprod"), with the accumulation of Sec. 3.4 (Eq. "kinetic1d"):
 * out = Kin(s) + k0.  k0 may be NULL (taken as 0), equal to out, or disjoint
 * from it; neither out nor k0 may overlap `s` (WVL_EINVAL). */
int wvl_kinetic(wvl_plan *plan, const void *s, const void *k0, void *out, void *ws,
                void *stream);

/* Local density (Sec. 2.5): steps 2 and 3a of Sec. 2.4 followed by
 * rho = [rho +] sum_b f_b psi_b^2 (Sec. 2, Eq. "density"), float64.
 * WVL_SHARED_V plans only; accumulate != 0 adds to the existing rho. */
int wvl_local_density(wvl_plan *plan, const void *c, double *rho, int accumulate, void *ws,
                      void *stream);

/* Local Hamiltonian (Sec. 2.4 steps 2-6): per orbital s = S c, psi = Omega s,
 * y = pot_scale V psi, Hc = A (Omega^T y + kin_scale Kin s), written to hpsi.
 * hpsi may be c itself (the result then replaces the coefficients); any other
 * overlap of hpsi with c is rejected with WVL_EINVAL.  The optional outputs
 * must not overlap c or hpsi.  Optional outputs (NULL to skip), all float64:
 *   rho    sum_b f_b psi_b^2 (WVL_SHARED_V plans; overwritten)
 *   e_loc  sum_r V rho (shared V) or sum_b f_b e_pot_b (per-orbital V)
 *   e_kin  sum_b f_b <s_b, Kin s_b>
 *   e_orb  [2 * norb]: e_pot_b = sum_r V psi_b^2, then e_kin_b = <s_b, Kin s_b>
 * V: the shared potential (m3 m2 m1 doubles) or, without WVL_SHARED_V, a
 * buffer holding orbital b's potential at v_off_b.  With pot_scale = kin_scale
 * = 1 this is the plain local Hamiltonian; other scales give the weighted
 * operator the energy gradients need. */
int wvl_local_hpsi(wvl_plan *plan, const void *c, const double *V, double pot_scale,
                   double kin_scale, void *hpsi, double *rho, double *e_loc, double *e_kin,
                   double *e_orb, void *ws, void *stream);

/* Compressed storage (Sec. 2.1): an orbital keeps its scaling coefficient
 * only at the coarse grid points of the low-resolution region and its seven
 * wavelet coefficients only at the points of the high-resolution region.
 * wvl_plan_set_regions() fixes the two regions of a plan whose orbitals all
 * share one grid.  A region is `nseg` segments [start, end) (int32 pairs,
 * HOST memory) of consecutive coarse points in the linear coarse index
 * i1 + n1 (i2 + n2 i3), increasing and disjoint, inside [0, n1 n2 n3); the
 * fine region need not lie inside the coarse one.  The call allocates and
 * uploads per-point maps (2 n1 n2 n3 int32) and the region point lists;
 * calling it again replaces them.
 * Compressed vector of one orbital: the nvctr_c coarse-region scaling
 * coefficients in segment order, then for every one of the nvctr_f
 * fine-region points in segment order its components mu = 1..7 (mu = b1 +
 * 2 b2 + 4 b3: wavelet along the axes whose bit is set), L = nvctr_c +
 * 7 nvctr_f values.  A compressed batch array holds orbital b at b * L, in
 * the plan precision (WVL_F32C: hi plane then lo plane of norb * L floats). */
int wvl_plan_set_regions(wvl_plan *plan, const int32_t *seg_c, int32_t nseg_c,
                         const int32_t *seg_f, int32_t nseg_f);
int wvl_plan_compressed_size(const wvl_plan *plan, int64_t *nvctr_c, int64_t *nvctr_f);
/* Step 1 of Sec. 2.4: the full coefficient array c (a batch array of the plan,
 * zero outside the regions) from the compressed batch psi_c. */
int wvl_decompress(wvl_plan *plan, const void *psi_c, void *c, void *stream);
/* Step 7 of Sec. 2.4: the region coefficients of c, packed into psi_c. */
int wvl_compress(wvl_plan *plan, const void *c, void *psi_c, void *stream);
/* Local Hamiltonian on compressed orbitals, steps 1-7 of Sec. 2.4:
 * decompress into the workspace, wvl_local_hpsi on the whole grid (in place
 * there), compress into hpsi_c, which may be psi_c itself.  The other
 * arguments and outputs are those of wvl_local_hpsi (rho and the energies of
 * the decompressed orbitals).  WVL_EUNSUPPORTED without regions. */
int wvl_local_hpsi_compressed(wvl_plan *plan, const void *psi_c, const double *V,
                              double pot_scale, double kin_scale, void *hpsi_c, double *rho,
                              double *e_loc, double *e_kin, double *e_orb, void *ws, void *stream);

/* Gradient of the energy functional E = g_loc E_loc + g_kin E_kin with respect
 * to the coefficients (Sec. 2 and Sec. 5: the minimisation needs the gradient
 * of the total energy with respect to every orbital).  Both energies are
 * quadratic forms of c_b with the symmetric operators of wvl_local_hpsi, so
 *     grad_b = 2 f_b (g_loc Hloc + g_kin Kin) c_b
 * with f_b the orbital's occupation; the weights are applied on the device.
 * grad may be c itself (not a partial overlap).  Not recorded in the plan's
 * graph (WVL_USE_GRAPH plans run it eagerly). */
int wvl_energy_gradient(wvl_plan *plan, const void *c, const double *V, double g_loc,
                        double g_kin, void *grad, void *ws, void *stream);

/* Preconditioner (Sec. 2, Eq. "precon"): for every orbital b, the
 * preconditioned gradient gt_b approximately solves the Helmholtz equation
 *     (-1/2 nabla^2 - eps_b) gt_b = g_b
 * in the wavelet basis, where the operator is A Kin S - eps_b I: the kinetic
 * recursion with K_0 = -eps_b s (Sec. 3.4, last sentence) followed by the
 * analysis.  It runs `iters` steps (0..10000) of preconditioned conjugate
 * gradients from gt_b = 0, with the diagonal of the operator in the wavelet
 * basis as preconditioner (one kinetic value per axis for scaling and one
 * for wavelet coefficients, minus eps_b); a step with no positive curvature
 * leaves gt_b unchanged.  Every eps_b must be negative (a bound orbital: the
 * operator is then positive definite), else WVL_EINVAL.
 *   g     batch array of the plan (read only)
 *   eps   HOST array of norb doubles, copied before the call returns
 *   mode  0: the operator as one combined filter per axis (synthesis,
 *         kinetic filter and analysis composed, Sec. 2.4 last paragraph and
 *         Sec. 6.1: the fused wavelet + kinetic kernel), with both in-plane
 *         axes applied by one plane-resident kernel when the plane fits it
 *         (periodic plans), else one pass per axis; WVL_F32C plans that the
 *         exact digit-product engine covers (uniform, fine lengths multiples
 *         of 16, equal spacing on all axes; no shared potential needed) run
 *         that form with exact int8 products (WVL_Q_PRECOND_FORM tells which
 *         form a plan takes); WVL_PRECOND_PASSES: the
 *         combined filter, one pass per axis; WVL_PRECOND_SEPARATE: the
 *         separate 3D synthesis, kinetic (with K_0) and analysis passes of
 *         the paper's GPU design (Sec. 2.4, Sec. 3.4)
 *   gt    output batch array, must not overlap g (WVL_EINVAL)
 *   res   nullable device array of norb doubles: the residual norm
 *         ||g_b - H gt_b|| of the recurrence after the last step
 * The convolution passes run in the plan's precision; the CG vector updates
 * and scalars in float64.  Ordinary (not persistent) launches; not recorded
 * in the plan's graph. */
#define WVL_PRECOND_SEPARATE 1u
#define WVL_PRECOND_PASSES   2u
int wvl_precondition(wvl_plan *plan, const void *g, const double *eps, int32_t iters,
                     uint32_t mode, void *gt, double *res, void *ws, void *stream);

/* Overlap matrix S_ij = <c_i, c_j> over all coefficients (Sec. 2.6; Sec. 5
 * step VIII), norb x norb float64, row-major.  Dense batches only. */
int wvl_overlap(wvl_plan *plan, const void *c, double *S, void *ws, void *stream);

/* Cholesky orthonormalisation (Sec. 5 step VIII): S = L L^T, c <- L^{-1} c
 * (rows = orbitals), in place.  S and L (nullable, norb x norb row-major)
 * receive the overlap matrix and the lower Cholesky factor.  A non-positive
 * pivot is reported by wvl_plan_sync() as WVL_EINVAL.  Up to 256 orbitals. */
int wvl_orthonormalize(wvl_plan *plan, void *c, double *S, double *L, void *ws, void *stream);

/* wvl_orthonormalize for callers that cannot allocate device memory (code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation and the same kernels, but the scratch memory
 * (overlap slice partials, L, L^{-1}) is a static device
 * array of the library instead of a caller workspace, so no `ws` argument.
 * The array holds 80 MiB on every GPU the library runs on, from the first
 * wvl_create() on that device until the process ends; every batch of up to
 * 256 orbitals fits (larger needs are rejected with WVL_EUNSUPPORTED before
 * any GPU work).  The call itself allocates nothing.  All calls on one GPU
 * share that one array: calls that overlap in time on the same GPU (other
 * streams, other threads, other plans) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero. */
int wvl_orthonormalize_noalloc(wvl_plan *plan, void *c, double *S, double *L, void *stream);

/* Format conversion of `count` values between WVL_F64, WVL_F32 and WVL_F32C
 * (hi/lo planes of `count` floats each); src and dst must not overlap. */
int wvl_convert(wvl_ctx *ctx, const void *src, int32_t src_prec, void *dst, int32_t dst_prec,
                int64_t count, void *stream);

/* Wait for `stream` and report device-side errors of this plan. */
int wvl_plan_sync(wvl_plan *plan, void *stream);

/* Choice made at plan creation for the hpsi kernels: variant id (0: one 1D
 * pass per axis and operator; 1: z passes around the plane-resident kernel
 * with vector-FMA in-plane passes, chosen whenever every orbital's (x, y)
 * plane fits in LDS; 2: the same with the in-plane passes of WVL_F64 on the
 * float64 matrix cores, chosen for WVL_F64 when the plane fits their 16 x 16
 * tiling (up to 128 x 128); 3: WVL_F32C with exact int8 digit products on
 * the matrix cores (every pass of float pairs split into six base-256 digits
 * per plane, the digit products summed exactly in int32, recombined in
 * int64), chosen for WVL_F32C plans with WVL_SHARED_V, periodic boundaries,
 * fine lengths that are multiples of 16, planes of at most 36 tiles of
 * 16 x 16 and the same grid spacing along every axis of an orbital.  Without
 * WVL_AUTOTUNE the environment variable WVL_NO_PLANE_KERNEL forces 0,
 * WVL_F32C_VECTOR keeps WVL_F32C off variant 3 and WVL_XY_VECTOR forces 1
 * over 2; the variable WVL_PLANE_OCCUPANCY=2 compiles
 * the plane kernel's choice for 2 instead of 4 waves per SIMD (where the
 * float64 matrix-core form then keeps its density group's plane in LDS;
 * WVL_NO_RHO_LDS keeps it in memory),
 * WVL_EXACT_OCCUPANCY_Z=2 the last z kernel of variant 3 for 2, and
 * WVL_NO_ZFUSE runs the last z step as two passes instead of one fused
 * launch (same results bit for bit; the fused launch is used for WVL_F64 and
 * WVL_F32).)  With WVL_AUTOTUNE, times_ms[k] (k < ntimes, at most 15
 * candidates) receives the mean time of candidate k = 3 seq + shape, or -1
 * where it was not available:
 *   seq 0 one pass per axis; 1 plane kernel at 4 waves per SIMD (default
 *   engine); 2 the same at 2 waves per SIMD; 3 plane kernel with the vector
 *   engine (WVL_F64 only); 4 the exact digit products (variant 3);
 *   shape 0 default tiles; 1 axis-1 tiles of half as many rows (seq 0 only);
 *   2 persistent launches of 4 instead of 8 workgroups per CU (WVL_PERSISTENT
 *   plans only).
 * The kept candidate is reported by wvl_plan_query.  Without WVL_AUTOTUNE
 * times_ms is filled with -1. */
int wvl_plan_tuning(const wvl_plan *plan, int32_t *variant, double *times_ms, int32_t ntimes);

/* Plan queries (*value receives the answer):
 *   WVL_Q_VARIANT     launch sequence of wvl_local_hpsi (see wvl_plan_tuning)
 *   WVL_Q_GROUP       orbitals per density group of the plane kernel (shared
 *                     potential, plane sequence), 0 otherwise
 *   WVL_Q_PERSISTENT  1 if the sequence's launches take tiles from work queues
 *   WVL_Q_XDIV        axis-1 tiles hold 1/XDIV of the rows that fit in LDS
 *   WVL_Q_PGRID       workgroups per CU of the persistent pass launches
 *   WVL_Q_TUNE_BEST   tuner candidate kept (index into times_ms), -1 untuned
 *   WVL_Q_FUSED_Z     1 if the last z step runs as one fused launch (it does
 *                     not when hpsi is c; see wvl_local_hpsi)
 *   WVL_Q_PRECOND_FORM operator of wvl_precondition's default mode: 0 one
 *                     combined-filter pass per axis, 1 z pass + plane-resident
 *                     in-plane kernel, 2 the same with the exact digit
 *                     products (WVL_F32C uniform periodic plans, fine lengths
 *                     multiples of 16, equal spacing on all axes) */
#define WVL_Q_VARIANT 0
#define WVL_Q_GROUP 1
#define WVL_Q_PERSISTENT 2
#define WVL_Q_XDIV 3
#define WVL_Q_PGRID 4
#define WVL_Q_TUNE_BEST 5
#define WVL_Q_FUSED_Z 6
#define WVL_Q_PRECOND_FORM 7
int wvl_plan_query(const wvl_plan *plan, int32_t what, int64_t *value);

/* Launch profiling: with capacity > 0, every kernel launch of the following
 * calls on this plan (eager mode; graph replays are not split) is bracketed
 * by a pair of hipEvents recorded on the call's stream, up to `capacity`
 * launches; capacity = 0 disables.  wvl_plan_profile_read() waits for the
 * recorded events, returns up to `max` (stage id, milliseconds) pairs in
 * launch order, their number in *count, and clears the records.
 * wvl_stage_name() names a stage id ("kin_z", "potential", "overlap",
 * "xy_plane", "z_final", ...). */
int wvl_plan_profile(wvl_plan *plan, int32_t capacity);
int wvl_plan_profile_read(wvl_plan *plan, int32_t *stage, double *ms, int32_t max,
                          int32_t *count);
const char *wvl_stage_name(int32_t stage);

const char *wvl_last_error(void);
const char *wvl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WVL_PUBLIC_API_H_ */
