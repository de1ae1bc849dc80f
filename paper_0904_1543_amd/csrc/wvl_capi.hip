// Host side of libwvl: argument checking, plans, workspace layout and the
// launch sequences of the C ABI declared in include/wvl.h.
//
// Every entry point validates its arguments before the first HIP call, so the
// whole contract can be exercised on a machine without a GPU (dry contexts).

#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "wvl.h"
#include "wvl_kernels.h"

using namespace wvl;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hipfail(hipError_t e, const char* where) {
  return fail(e == hipErrorOutOfMemory ? WVL_ENOMEM : WVL_EHIP, "%s: %s", where,
              hipGetErrorString(e));
}

#define WVL_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return hipfail(_e, #call);    \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Every device allocation of the library goes through here.  With the
// environment variable WVL_DEBUG_FAIL_ALLOC=1 it fails as an exhausted device
// would, so that the out-of-memory paths can be exercised.
hipError_t dev_malloc(void** p, size_t bytes) {
  const char* f = getenv("WVL_DEBUG_FAIL_ALLOC");
  if (f && f[0] == '1') {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

}  // namespace

struct wvl_ctx {
  int device;
  bool dry;
  size_t lds_per_block;
  int cus;
};

struct GraphKey {
  const void* p[8];
  double s[2];
  bool operator==(const GraphKey& o) const {
    for (int i = 0; i < 8; ++i) if (p[i] != o.p[i]) return false;
    return s[0] == o.s[0] && s[1] == o.s[1];
  }
};

struct wvl_plan {
  wvl_ctx* ctx = nullptr;
  int prec = 0;
  uint32_t flags = 0;
  int norb = 0;
  bool shared = false;   // shared potential + uniform grid
  bool dense = false;    // off_b = b * M, all dims equal
  bool occ_uniform = true;  // every orbital has the same occupation
  int64_t M = 0;         // points per orbital when uniform
  // boundary conditions (Sec. 3.1): isolated axes; real-space grid of V and
  // rho (m_a + 29 points along isolated axes) and its points per orbital
  bool bc_free[3] = {false, false, false};
  bool bc_any = false;
  int Mr[3] = {0, 0, 0};
  int64_t Mrs = 0;
  int bc_tiles[3] = {0, 0, 0};   // tiles per orbital of the kinetic passes, axes 1..3
  OrbDev* d_orbs_rs = nullptr;   // real-space offsets (b * Mrs) for the pointwise stage
  int32_t* d_pb = nullptr;       // prefixes b * bc_tiles[a] of the kinetic passes (3 arrays)
  int64_t elems = 0;     // elements per packed plane
  int64_t elems_rs = 0;  // elements of a real-space batch array (per plane)
  int64_t vlen = 0;      // minimal length of a per-orbital V buffer
  std::vector<OrbDev> orbs;
  std::vector<int32_t> pz, py, px, pp, pq, pc;
  int nblk = 0;          // 256-point blocks of the shared grid
  // plane-resident path of wvl_local_hpsi
  bool use_xy = false;
  bool xy_ok = false;    // some form of the plane path fits (workspace reserved)
  int xy_m1 = 0, xy_m2 = 0, xy_G = 1, xy_ngroups = 0, xy_blocks = 0, xy_occ = 4;
  int xy_engine = 0;   // in-plane passes: 0 vector FMA, 1 float64 matrix cores
  bool zfuse = true;   // last two z passes of the plane path fused (not for F32C)
  // exact-product engine of the compensated form (uniform batches with a
  // shared potential, lengths multiples of 16, isotropic grid spacing)
  bool oz_ok = false, use_oz = false;
  bool oz_pc = false;   // the preconditioner's operator with the exact products (no potential needed)
  int oz_occ_z = 4;   // waves per SIMD of the exact engine's final z kernel
  std::vector<int32_t> pxz;          // prefix of xz-planes (m2 per orbital)
  int32_t* d_pxz = nullptr;
  // persistent launches (WVL_PERSISTENT) of the plane path: work order by
  // decreasing cost per tile, and the number of resident workgroups
  bool persistent = false;
  std::vector<int32_t> perm_z, order_z, perm_q, order_q, px2, perm_y, order_y, perm_x, order_x,
      order_x2, perm_p, order_p;
  int pgrid_pass = 0;
  // launch shape (picked by the tuner): axis-1 rows-per-tile divisor and
  // workgroups per CU of the persistent pass launches
  int xdiv = 1, pgrid_mul = 8;
  // device copies
  OrbDev* d_orbs = nullptr;
  int32_t* d_pz = nullptr;
  int32_t* d_py = nullptr;
  int32_t* d_px = nullptr;
  int32_t* d_pp = nullptr;
  int32_t* d_pq = nullptr;
  int32_t *d_perm_z = nullptr, *d_order_z = nullptr, *d_perm_q = nullptr, *d_order_q = nullptr;
  int32_t *d_pc = nullptr;   // preconditioner element tiles
  int32_t *d_px2 = nullptr, *d_perm_y = nullptr, *d_order_y = nullptr, *d_perm_x = nullptr,
          *d_order_x = nullptr, *d_order_x2 = nullptr, *d_perm_p = nullptr, *d_order_p = nullptr;
  int* d_info = nullptr;
  // compressed storage (Sec. 2.1): regions of a uniform batch
  int64_t nvc = -1, nvf = 0;   // coarse-region and fine-region points (-1: no regions)
  int32_t *d_map_c = nullptr, *d_map_f = nullptr, *d_list_c = nullptr, *d_list_f = nullptr;
  // workspace layout (byte offsets)
  size_t ws = 0, o_A = 0, o_B = 0, o_S = 0, o_D = 0, o_cg = 0, o_ez = 0, o_ey = 0, o_ex = 0, o_pp = 0, o_rv = 0,
         o_rho = 0, o_eorb = 0, o_syrk = 0, o_L = 0, o_Li = 0, o_rhop = 0, o_epl = 0,
         o_kpl = 0, o_queue = 0, o_ozv = 0, o_oze = 0, o_kpl2 = 0;
  // graph cache
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec = nullptr;
  GraphKey gkey{};
  int variant = 0;
  int tune_best = -1;            // tuner: index of the candidate kept
  std::vector<double> tune_ms;
  // launch profiling (hipEvent pairs around every launch of a call)
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> prof;
  int prof_cap = 0, prof_used = 0;
  bool capturing = false;
};

// Stage ids for profiling: 1D passes are op * 3 + (axis - 1); then:
enum { ST_POT = 15, ST_ENERGY = 16, ST_OVERLAP = 17, ST_CHOL = 18, ST_TRMM = 19, ST_XY = 29,
       ST_RHO = 30, ST_ZFIN = 31, ST_CG = 32, ST_HELM = 33, ST_NSTAGE = 34 };
static int stage_of(int op, int axis) {
  return op < 5 ? op * 3 + axis - 1 : 20 + (op - 5) * 3 + axis - 1;
}
static const char* kStageNames[ST_NSTAGE] = {
    "mf_x", "mf_y", "mf_z", "mft_x", "mft_y", "mft_z", "syn_x", "syn_y", "syn_z",
    "ana_x", "ana_y", "ana_z", "kin_x", "kin_y", "kin_z", "potential", "energies",
    "overlap", "cholesky", "trmm", "cw_x", "cw_y", "cw_z", "cwt_x", "cwt_y", "cwt_z",
    "ck_x", "ck_y", "ck_z", "xy_plane", "rho_reduce", "z_final", "cg_update", "helm_plane"};

namespace {
struct Mark {
  wvl_plan* p;
  hipStream_t st;
  int slot = -1;
  Mark(wvl_plan* pl, hipStream_t s, int stage) : p(pl), st(s) {
    if (p->prof_cap <= 0 || p->capturing || p->prof_used >= p->prof_cap) return;
    if ((int)p->prof.size() <= p->prof_used) {
      wvl_plan::Rec r{stage, nullptr, nullptr};
      if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
      p->prof.push_back(r);
    }
    slot = p->prof_used++;
    p->prof[slot].stage = stage;
    (void)hipEventRecord(p->prof[slot].a, st);
  }
  ~Mark() {
    if (slot >= 0) (void)hipEventRecord(p->prof[slot].b, st);
  }
};
}  // namespace

static int esize(int prec) { return prec == WVL_F32 ? 4 : 8; }

constexpr int kBcExtra = 29;   // real-space points added along an isolated axis

constexpr int kQueueCounters = 16;   // work-queue counters per launch sequence
constexpr int kTuneCands = 15;       // launch candidates of the tuner (5 sequences x 3 shapes)

static int check_plan(const wvl_plan* p) {
  if (!p) return fail(WVL_EINVAL, "plan is NULL");
  return WVL_OK;
}

// the single 3D transforms keep the array shape: periodic plans only
static int check_periodic(const wvl_plan* p, const char* what) {
  if (p->bc_any)
    return fail(WVL_EUNSUPPORTED, "%s: periodic plans only (isolated axes change the array length)",
                what);
  return WVL_OK;
}

static int check_gpu(const wvl_plan* p) {
  if (p->ctx->dry) return fail(WVL_ENODEV, "dry context: no GPU");
  hipError_t e = hipSetDevice(p->ctx->device);
  if (e != hipSuccess) return hipfail(e, "hipSetDevice");
  return WVL_OK;
}

static inline char* wsp(void* ws, size_t off) { return (char*)ws + off; }

// Preconditioner part of the workspace: three arrays of one double per
// 256-point tile (r.z, p.p and r.r partials), eps per orbital, CG scalars.
struct CgLayout { size_t rz, pp, rr, eps, sc, bytes; };
static CgLayout cg_layout(const wvl_plan* p) {
  const size_t np = align256(sizeof(double) * (size_t)p->pc[p->norb]);
  CgLayout l;
  l.rz = 0;
  l.pp = np;
  l.rr = 2 * np;
  l.eps = 3 * np;
  l.sc = l.eps + align256(sizeof(double) * (size_t)p->norb);
  l.bytes = l.sc + align256(cg_scalar_bytes() * (size_t)p->norb);
  return l;
}
static size_t cg_bytes(const wvl_plan* p) { return cg_layout(p).bytes; }

// bytes of one packed batch array of the plan (both planes for WVL_F32C)
static size_t batch_bytes(const wvl_plan* p) {
  return (size_t)p->elems * (p->prec == WVL_F32 ? 4 : 8);
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// batch arrays start on a 16-byte boundary (the kernels move four elements
// of a plane per access); nullptrs are checked elsewhere
static int check_aligned(const char* what, std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs)
    if (((uintptr_t)q & 15) != 0)
      return fail(WVL_EINVAL, "%s: batch array %p is not 16-byte aligned", what, q);
  return WVL_OK;
}

// input and output batch arrays of an operation must not share memory
static int check_disjoint(const wvl_plan* p, const void* in, const void* out, const char* what) {
  if (overlap(in, batch_bytes(p), out, batch_bytes(p)))
    return fail(WVL_EINVAL, "%s: output overlaps input", what);
  return WVL_OK;
}

namespace {
int autotune(wvl_plan* p);
int scratch_setup(int device);
}  // namespace

extern "C" {

const char* wvl_last_error(void) { return g_err.c_str(); }
const char* wvl_version(void) { return "wvl 1.0 (gfx950)"; }

int wvl_create(wvl_ctx** ctx, int device) {
  if (!ctx) return fail(WVL_EINVAL, "ctx is NULL");
  *ctx = nullptr;
  if (device < -1) return fail(WVL_EINVAL, "device %d < -1", device);
  wvl_ctx* c = new wvl_ctx();
  c->device = device;
  c->dry = device < 0;
  c->lds_per_block = 65536;
  c->cus = 256;
  if (!c->dry) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= device) {
      delete c;
      return fail(WVL_ENODEV, "no GPU %d (hipGetDeviceCount: %s, count %d)", device,
                  e == hipSuccess ? "ok" : hipGetErrorString(e), n);
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) { delete c; return hipfail(e, "hipGetDeviceProperties"); }
    c->lds_per_block = prop.sharedMemPerBlock;
    c->cus = prop.multiProcessorCount;
    // the no-allocation entry point's scratch array on this device
    e = hipSetDevice(device);
    if (e != hipSuccess) { delete c; return hipfail(e, "hipSetDevice"); }
    if (int r = scratch_setup(device)) { delete c; return r; }
  }
  *ctx = c;
  return WVL_OK;
}

int wvl_destroy(wvl_ctx* ctx) {
  if (!ctx) return fail(WVL_EINVAL, "ctx is NULL");
  delete ctx;
  return WVL_OK;
}

int wvl_plan_create(wvl_ctx* ctx, const wvl_orbital* orbs, int32_t norb, int32_t prec,
                    uint32_t flags, wvl_plan** plan) {
  if (!plan) return fail(WVL_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (!ctx) return fail(WVL_EINVAL, "ctx is NULL");
  if (norb <= 0) return fail(WVL_EINVAL, "norb = %d must be positive", norb);
  if (!orbs) return fail(WVL_EINVAL, "orbs is NULL");
  if (prec < WVL_F64 || prec > WVL_F32C) return fail(WVL_EINVAL, "unknown precision %d", prec);
  if (flags & ~(uint32_t)(WVL_SHARED_V | WVL_USE_GRAPH | WVL_PERSISTENT | WVL_AUTOTUNE |
                          WVL_FREE_BC | WVL_SURFACE_BC))
    return fail(WVL_EINVAL, "unknown flag bits 0x%x", flags);
  if ((flags & WVL_FREE_BC) && (flags & WVL_SURFACE_BC))
    return fail(WVL_EINVAL, "WVL_FREE_BC and WVL_SURFACE_BC exclude each other");
  wvl_plan* p = new wvl_plan();
  p->ctx = ctx;
  p->prec = prec;
  p->flags = flags;
  p->norb = norb;
  p->orbs.resize(norb);
  bool uniform = true, dense = true;
  int64_t end = 0;
  std::vector<std::pair<int64_t, int64_t>> spans;
  for (int b = 0; b < norb; ++b) {
    const wvl_orbital& o = orbs[b];
    for (int a = 0; a < 3; ++a) {
      if (o.n[a] < 2 || o.n[a] > (1 << 14)) {
        delete p;
        return fail(WVL_EINVAL, "orbital %d: n[%d] = %d out of range [2, 16384]", b, a, o.n[a]);
      }
      if (!(o.hgrid[a] > 0.0) || !isfinite(o.hgrid[a])) {
        delete p;
        return fail(WVL_EINVAL, "orbital %d: hgrid[%d] must be positive", b, a);
      }
    }
    if (o.reserved != 0) { delete p; return fail(WVL_EINVAL, "orbital %d: reserved must be 0", b); }
    if (2 * o.n[0] + 2 * kHalo > kContigLds) {
      delete p;
      return fail(WVL_EUNSUPPORTED, "orbital %d: n1 = %d exceeds %d (axis-1 lines are staged in LDS)",
                  b, o.n[0], (kContigLds - 2 * kHalo) / 2);
    }
    if (!isfinite(o.occ)) { delete p; return fail(WVL_EINVAL, "orbital %d: occupation not finite", b); }
    if (o.off < 0 || o.v_off < 0) { delete p; return fail(WVL_EINVAL, "orbital %d: negative offset", b); }
    OrbDev& d = p->orbs[b];
    for (int a = 0; a < 3; ++a) {
      d.m[a] = 2 * o.n[a];
      d.kscale[a] = -1.0 / (2.0 * o.hgrid[a] * o.hgrid[a]);
      // diagonal of A Kin S along this axis: the combined kinetic filter's
      // taps that map a coefficient onto itself on the periodic line
      // (offsets o = 0 mod m), for scaling (even) and wavelet (odd) outputs
      const bool iso = (flags & WVL_FREE_BC) || ((flags & WVL_SURFACE_BC) && a == 1);
      for (int par = 0; par < 2; ++par) {
        double sum = 0.0;
        for (int off = WVL_CK_LO; off < WVL_CK_LO + WVL_CK_N; ++off)
          if (iso ? off == 0 : off % d.m[a] == 0) sum += coef<OP_CK>(par, off, 0);
        d.kdiag[a][par] = d.kscale[a] * sum;
      }
    }
    d.pad = 0;
    d.off = o.off;
    d.voff = (flags & WVL_SHARED_V) ? 0 : o.v_off;
    d.occ = o.occ;
    const int64_t M = (int64_t)d.m[0] * d.m[1] * d.m[2];
    if (M > (int64_t)1 << 31) { delete p; return fail(WVL_EINVAL, "orbital %d: grid too large", b); }
    spans.push_back({o.off, o.off + M});
    end = std::max(end, o.off + M);
    p->vlen = std::max(p->vlen, d.voff + M);
    if (b > 0 && (d.m[0] != p->orbs[0].m[0] || d.m[1] != p->orbs[0].m[1] || d.m[2] != p->orbs[0].m[2]))
      uniform = false;
    if (o.off != (int64_t)b * M) dense = false;
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); ++i)
    if (spans[i].first < spans[i - 1].second) {
      delete p;
      return fail(WVL_EINVAL, "orbitals overlap in the packed buffer");
    }
  if ((flags & WVL_SHARED_V) && !uniform) {
    delete p;
    return fail(WVL_EINVAL, "WVL_SHARED_V needs every orbital on the same grid");
  }
  p->shared = (flags & WVL_SHARED_V) != 0;
  p->dense = dense && uniform;
  for (int b = 1; b < norb; ++b)
    if (p->orbs[b].occ != p->orbs[0].occ) p->occ_uniform = false;
  // boundary conditions: isolated along every axis, or along axis 2 (slab)
  for (int a = 0; a < 3; ++a)
    p->bc_free[a] = (flags & WVL_FREE_BC) || ((flags & WVL_SURFACE_BC) && a == 1);
  p->bc_any = p->bc_free[0] || p->bc_free[1] || p->bc_free[2];
  if (p->bc_any && !(p->shared && p->dense)) {
    delete p;
    return fail(WVL_EUNSUPPORTED,
                "isolated/surface boundary conditions need WVL_SHARED_V and a dense uniform batch");
  }
  for (int a = 0; a < 3; ++a) p->Mr[a] = p->orbs[0].m[a] + (p->bc_free[a] ? kBcExtra : 0);
  p->Mrs = uniform ? (int64_t)p->Mr[0] * p->Mr[1] * p->Mr[2] : 0;
  if (p->bc_any) {
    const int m1 = p->orbs[0].m[0], m2 = p->orbs[0].m[1], m3 = p->orbs[0].m[2];
    p->bc_tiles[0] = (m2 * m3 + bc_rows_per_tile(OP_CK, m1) - 1) / bc_rows_per_tile(OP_CK, m1);
    p->bc_tiles[1] = (m1 * m3 + kThreads - 1) / kThreads;
    p->bc_tiles[2] = (m1 * m2 + kThreads - 1) / kThreads;
  }
  p->M = uniform ? (int64_t)p->orbs[0].m[0] * p->orbs[0].m[1] * p->orbs[0].m[2] : 0;
  p->elems = end;
  if (end > ((int64_t)1 << 40)) { delete p; return fail(WVL_EINVAL, "batch too large"); }
  // tiling
  p->pz.assign(norb + 1, 0);
  p->py.assign(norb + 1, 0);
  p->px.assign(norb + 1, 0);
  p->pp.assign(norb + 1, 0);
  p->pq.assign(norb + 1, 0);
  p->px2.assign(norb + 1, 0);
  p->pc.assign(norb + 1, 0);
  for (int b = 0; b < norb; ++b) {
    const OrbDev& d = p->orbs[b];
    const int64_t m1 = d.m[0], m2 = d.m[1], m3 = d.m[2];
    const int64_t R = contig_rows((int)m1, 1), R2 = contig_rows((int)m1, 2);
    p->pz[b + 1] = p->pz[b] + (int32_t)((m1 * m2 + kThreads - 1) / kThreads);
    p->py[b + 1] = p->py[b] + (int32_t)((m1 * m3 + kThreads - 1) / kThreads);
    p->px[b + 1] = p->px[b] + (int32_t)((m2 * m3 + R - 1) / R);
    p->px2[b + 1] = p->px2[b] + (int32_t)((m2 * m3 + R2 - 1) / R2);
    p->pc[b + 1] = p->pc[b] + (int32_t)((m1 * m2 * m3 + cg_tile_elems() - 1) / cg_tile_elems());
    p->pp[b + 1] = p->pp[b] + (int32_t)((m1 * m2 * m3 + kThreads - 1) / kThreads);
    p->pq[b + 1] = p->pq[b] + (int32_t)m3;
    if (p->pp[b + 1] < 0 || p->pz[b + 1] < 0 || p->px2[b + 1] < 0) {
      delete p;
      return fail(WVL_EINVAL, "too many tiles");
    }
  }
  p->nblk = p->shared ? (int)((p->Mrs + kThreads - 1) / kThreads) : 0;
  // plane-resident path: every orbital's (m1, m2) plane must fit the kernel
  {
    for (int b = 0; b < norb; ++b) {
      p->xy_m1 = std::max(p->xy_m1, p->orbs[b].m[0]);
      p->xy_m2 = std::max(p->xy_m2, p->orbs[b].m[1]);
    }
    // float64 uses the matrix cores when the plane fits their tiling
    const bool mx = xy_matrix_engine(prec, p->xy_m1, p->xy_m2) && !getenv("WVL_XY_VECTOR");
    bool ok = xy_supported(prec, p->xy_m1, p->xy_m2, mx);
    if (getenv("WVL_NO_PLANE_KERNEL") || p->bc_any) ok = false;
    if (const char* o = getenv("WVL_PLANE_OCCUPANCY")) p->xy_occ = atoi(o) == 2 ? 2 : 4;
    // compensated float32 keeps two windows of hi/lo pairs: fused, it drops
    // to one wave per SIMD and is slower than the two passes
    p->zfuse = prec != WVL_F32C && !getenv("WVL_NO_ZFUSE");
    p->use_xy = ok;
    p->xy_ok = !p->bc_any && (xy_supported(prec, p->xy_m1, p->xy_m2, mx) ||
                              xy_supported(prec, p->xy_m1, p->xy_m2, false));
    p->xy_engine = ok && mx ? 1 : 0;
    p->variant = ok ? 1 + p->xy_engine : 0;
    if (p->shared) {
      const int m3 = p->orbs[0].m[2];
      p->xy_G = std::max(1, std::min(8, (int)((int64_t)norb * m3 / 1024)));
      p->xy_ngroups = (norb + p->xy_G - 1) / p->xy_G;
      p->xy_blocks = p->xy_ngroups * m3;
    } else {
      p->xy_G = 1;
      p->xy_ngroups = 0;
      p->xy_blocks = p->pq[norb];
    }
  }
  // exact-product engine of the compensated form
  {
    bool ok = prec == WVL_F32C && uniform && !p->bc_any && !getenv("WVL_F32C_VECTOR") &&
              !getenv("WVL_NO_PLANE_KERNEL");
    if (ok) ok = oz_supported(p->orbs[0].m[0], p->orbs[0].m[1], p->orbs[0].m[2]);
    for (int b = 0; ok && b < norb; ++b) {
      const double* k = p->orbs[b].kscale;
      ok = k[0] == k[1] && k[1] == k[2];
    }
    p->oz_pc = ok;
    ok = ok && p->shared;
    p->oz_ok = ok;
    p->use_oz = ok;
    if (ok) p->variant = 3;
    if (const char* o = getenv("WVL_EXACT_OCCUPANCY_Z")) p->oz_occ_z = atoi(o) == 2 ? 2 : 4;
    p->pxz.assign(norb + 1, 0);
    for (int b = 0; b < norb; ++b) p->pxz[b + 1] = p->pxz[b] + p->orbs[b].m[1];
  }
  // persistent work order: z-pass tiles cost ~ m3 (one line per lane),
  // in-plane tiles (one plane) cost ~ m1 m2; largest first, ties by index
  {
    auto build = [&](std::vector<int32_t>& perm, std::vector<int32_t>& order,
                     const std::vector<int32_t>& pre, auto cost) {
      perm.resize(norb);
      for (int b = 0; b < norb; ++b) perm[b] = b;
      std::stable_sort(perm.begin(), perm.end(),
                       [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
      order.assign(norb + 1, 0);
      for (int r = 0; r < norb; ++r) order[r + 1] = order[r] + (pre[perm[r] + 1] - pre[perm[r]]);
    };
    build(p->perm_z, p->order_z, p->pz, [&](int b) { return (int64_t)p->orbs[b].m[2]; });
    build(p->perm_q, p->order_q, p->pq,
          [&](int b) { return (int64_t)p->orbs[b].m[0] * p->orbs[b].m[1]; });
    // pass-by-pass sequence: y tiles cost ~ m2, x tiles ~ their rows x m1,
    // pointwise tiles are all alike
    build(p->perm_y, p->order_y, p->py, [&](int b) { return (int64_t)p->orbs[b].m[1]; });
    build(p->perm_x, p->order_x, p->px, [&](int b) {
      const int m1 = p->orbs[b].m[0];
      return (int64_t)contig_rows(m1, 1) * m1;
    });
    {
      std::vector<int32_t> tmp;
      build(tmp, p->order_x2, p->px2, [&](int b) {
        const int m1 = p->orbs[b].m[0];
        return (int64_t)contig_rows(m1, 1) * m1;
      });
    }
    build(p->perm_p, p->order_p, p->pp, [&](int) { return (int64_t)0; });
    p->persistent = (flags & WVL_PERSISTENT) != 0;
    p->pgrid_pass = std::max(1, ctx->cus) * p->pgrid_mul;
  }
  // workspace layout
  size_t off = 0;
  // batch arrays: coefficients, or the real-space grid of isolated axes
  p->elems_rs = p->bc_any ? (int64_t)norb * p->Mrs : p->elems;
  const size_t arr = align256((size_t)std::max(p->elems, p->elems_rs) * esize(prec));
  p->o_A = off; off += arr;
  p->o_B = off; off += arr;
  p->o_S = off; off += arr;
  p->o_D = off; off += arr;      // fourth batch array: preconditioner, separate-pass form
  p->o_cg = off;                 // preconditioner: r.z, p.p, r.r tile partials, eps, scalars
  off += cg_bytes(p);
  p->o_ez = off; off += align256(sizeof(double) * std::max<int64_t>(p->pz[norb], (int64_t)norb * p->bc_tiles[2]));
  p->o_ey = off; off += align256(sizeof(double) * std::max<int64_t>(p->py[norb], (int64_t)norb * p->bc_tiles[1]));
  p->o_ex = off; off += align256(sizeof(double) * std::max<int64_t>(std::max(p->px[norb], p->px2[norb]),
                                                                   (int64_t)norb * p->bc_tiles[0]));
  p->o_pp = off;
  off += align256(sizeof(double) * (p->shared ? (size_t)norb * p->nblk : (size_t)p->pp[norb]));
  p->o_rv = off; off += align256(sizeof(double) * (size_t)std::max(p->nblk, 1));
  p->o_rho = off; off += align256(sizeof(double) * (size_t)(p->shared ? p->Mrs : 1));
  p->o_eorb = off; off += align256(sizeof(double) * 2 * (size_t)norb);
  if (p->dense) {
    p->o_syrk = off; off += align256(sizeof(double) * (size_t)syrk_partials(norb, p->M));
    p->o_L = off; off += align256(sizeof(double) * (size_t)norb * norb);
    p->o_Li = off; off += align256(sizeof(double) * (size_t)norb * norb);
  }
  if (p->xy_ok || p->oz_pc) {   // the plane path may be chosen later by the tuner
    if (p->shared) {
      p->o_rhop = off;
      off += align256(sizeof(double) * (size_t)p->xy_ngroups * p->M);
    }
    p->o_epl = off; off += align256(sizeof(double) * (size_t)p->pq[norb]);
    p->o_kpl = off; off += align256(sizeof(double) * (size_t)p->pq[norb]);
  }
  if (p->oz_ok) {   // potential as float pairs, plane exponents
    p->o_ozv = off; off += align256(sizeof(float) * 2 * (size_t)p->M);
    p->o_oze = off; off += align256(sizeof(int) * (size_t)p->orbs[0].m[2]);
  }
  if (p->oz_pc) {   // per-xz-plane kinetic sums
    p->o_kpl2 = off; off += align256(sizeof(double) * (size_t)p->pxz[norb]);
  }
  p->o_queue = off; off += align256(sizeof(int32_t) * kQueueCounters);   // work-queue counters
  p->ws = off;
  if (!ctx->dry) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = dev_malloc((void**)&p->d_orbs, sizeof(OrbDev) * norb);
    if (e == hipSuccess) e = dev_malloc((void**)&p->d_pz, sizeof(int32_t) * (norb + 1) * 19);
    if (e == hipSuccess) e = dev_malloc((void**)&p->d_info, sizeof(int) * 4);
    if (e != hipSuccess) {
      wvl_plan_destroy(p);
      return fail(WVL_ENOMEM, "plan allocation failed: %s", hipGetErrorString(e));
    }
    p->d_py = p->d_pz + (norb + 1);
    p->d_px = p->d_py + (norb + 1);
    p->d_pp = p->d_px + (norb + 1);
    p->d_pq = p->d_pp + (norb + 1);
    p->d_perm_z = p->d_pq + (norb + 1);
    p->d_order_z = p->d_perm_z + (norb + 1);
    p->d_perm_q = p->d_order_z + (norb + 1);
    p->d_order_q = p->d_perm_q + (norb + 1);
    p->d_px2 = p->d_order_q + (norb + 1);
    p->d_perm_y = p->d_px2 + (norb + 1);
    p->d_order_y = p->d_perm_y + (norb + 1);
    p->d_perm_x = p->d_order_y + (norb + 1);
    p->d_order_x = p->d_perm_x + (norb + 1);
    p->d_order_x2 = p->d_order_x + (norb + 1);
    p->d_perm_p = p->d_order_x2 + (norb + 1);
    p->d_order_p = p->d_perm_p + (norb + 1);
    p->d_pc = p->d_order_p + (norb + 1);
    p->d_pxz = p->d_pc + (norb + 1);
    std::vector<int32_t> all;
    all.insert(all.end(), p->pz.begin(), p->pz.end());
    all.insert(all.end(), p->py.begin(), p->py.end());
    all.insert(all.end(), p->px.begin(), p->px.end());
    all.insert(all.end(), p->pp.begin(), p->pp.end());
    all.insert(all.end(), p->pq.begin(), p->pq.end());
    for (auto* v : {&p->perm_z, &p->order_z, &p->perm_q, &p->order_q, &p->px2, &p->perm_y,
                    &p->order_y, &p->perm_x, &p->order_x, &p->order_x2, &p->perm_p, &p->order_p,
                    &p->pc, &p->pxz}) {
      all.insert(all.end(), v->begin(), v->end());
      all.resize(all.size() + (norb + 1 - v->size()), 0);
    }
    e = hipMemcpy(p->d_orbs, p->orbs.data(), sizeof(OrbDev) * norb, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_pz, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice);
    int zero[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpy(p->d_info, zero, sizeof zero, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      wvl_plan_destroy(p);
      return hipfail(e, "plan upload");
    }
  }
  if (p->bc_any && !ctx->dry) {
    std::vector<OrbDev> rs(p->orbs);
    for (int b = 0; b < norb; ++b) rs[b].off = (int64_t)b * p->Mrs;
    std::vector<int32_t> pb(3 * (size_t)(norb + 1));
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b <= norb; ++b) pb[(size_t)a * (norb + 1) + b] = b * p->bc_tiles[a];
    hipError_t e = dev_malloc((void**)&p->d_orbs_rs, sizeof(OrbDev) * norb);
    if (e == hipSuccess) e = dev_malloc((void**)&p->d_pb, sizeof(int32_t) * pb.size());
    if (e == hipSuccess)
      e = hipMemcpy(p->d_orbs_rs, rs.data(), sizeof(OrbDev) * norb, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_pb, pb.data(), sizeof(int32_t) * pb.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      wvl_plan_destroy(p);
      return fail(WVL_ENOMEM, "boundary-condition tables: %s", hipGetErrorString(e));
    }
  }
  if ((flags & WVL_AUTOTUNE) && !ctx->dry && !p->bc_any) {
    if (int r = autotune(p)) { wvl_plan_destroy(p); return r; }
  }
  *plan = p;
  return WVL_OK;
}

int wvl_plan_destroy(wvl_plan* p) {
  if (!p) return fail(WVL_EINVAL, "plan is NULL");
  if (!p->ctx->dry) {
    (void)hipSetDevice(p->ctx->device);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    for (auto& r : p->prof) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    if (p->ev_in) (void)hipEventDestroy(p->ev_in);
    if (p->ev_out) (void)hipEventDestroy(p->ev_out);
    if (p->gstream) (void)hipStreamDestroy(p->gstream);
    if (p->d_orbs) (void)hipFree(p->d_orbs);
    if (p->d_pz) (void)hipFree(p->d_pz);
    if (p->d_info) (void)hipFree(p->d_info);
    if (p->d_map_c) (void)hipFree(p->d_map_c);
    if (p->d_orbs_rs) (void)hipFree(p->d_orbs_rs);
    if (p->d_pb) (void)hipFree(p->d_pb);
  }
  delete p;
  return WVL_OK;
}

int wvl_plan_workspace(const wvl_plan* p, size_t* bytes) {
  if (int r = check_plan(p)) return r;
  if (!bytes) return fail(WVL_EINVAL, "bytes is NULL");
  *bytes = p->ws;
  return WVL_OK;
}

int wvl_plan_elements(const wvl_plan* p, int64_t* elems) {
  if (int r = check_plan(p)) return r;
  if (!elems) return fail(WVL_EINVAL, "elems is NULL");
  *elems = p->elems;
  return WVL_OK;
}

int wvl_plan_grid_points(const wvl_plan* p, int64_t* points) {
  if (int r = check_plan(p)) return r;
  if (!points) return fail(WVL_EINVAL, "points is NULL");
  if (!p->shared) return fail(WVL_EUNSUPPORTED, "plan has no shared grid");
  *points = p->Mrs;
  return WVL_OK;
}

int wvl_plan_tuning(const wvl_plan* p, int32_t* variant, double* times_ms, int32_t ntimes) {
  if (int r = check_plan(p)) return r;
  if (variant) *variant = p->variant;
  if (times_ms)
    for (int i = 0; i < ntimes; ++i) times_ms[i] = i < (int)p->tune_ms.size() ? p->tune_ms[i] : -1.0;
  return WVL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------
namespace {

struct Seq {
  wvl_plan* p;
  hipStream_t st;
  PassGeom gz, gy, gx, gp;
  int32_t* queue = nullptr;   // persistent launches: next free work-queue counter
  int32_t* queue_end = nullptr;
  Seq(wvl_plan* pl, hipStream_t s) : p(pl), st(s) {
    gz = PassGeom{p->d_orbs, p->d_pz, p->norb};
    gy = PassGeom{p->d_orbs, p->d_py, p->norb};
    gx = PassGeom{p->d_orbs, p->xdiv == 2 ? p->d_px2 : p->d_px, p->norb};
    gx.xdiv = p->xdiv;
    gp = PassGeom{p->d_orbs, p->d_pp, p->norb};
  }
  int ntiles(int axis) const {
    return axis == 1 ? (p->xdiv == 2 ? p->px2[p->norb] : p->px[p->norb])
         : axis == 2 ? p->py[p->norb] : p->pz[p->norb];
  }
  // persistent form of a launch over `n` tiles: work order and a fresh counter
  bool make_persistent(PassGeom& g, int n, const int32_t* order, const int32_t* perm) {
    if (!queue || queue >= queue_end) return false;
    g.order = order;
    g.perm = perm;
    g.queue = queue++;
    g.ntiles = n;
    g.grid = p->pgrid_pass;
    return true;
  }
  hipError_t pass(int op, int axis, const void* in, void* out, const void* k0 = nullptr,
                  double kmul = 1.0, double* ep = nullptr) {
    Mark mk(p, st, stage_of(op, axis));
    PassGeom g = axis == 1 ? gx : axis == 2 ? gy : gz;
    const int n = ntiles(axis);
    if (queue) {
      if (axis == 3) make_persistent(g, n, p->d_order_z, p->d_perm_z);
      else if (axis == 2) make_persistent(g, n, p->d_order_y, p->d_perm_y);
      else make_persistent(g, n, p->xdiv == 2 ? p->d_order_x2 : p->d_order_x, p->d_perm_x);
    }
    return launch_pass(p->prec, op, axis, g, n, in, out, k0, p->elems, kmul, ep, st);
  }
  hipError_t pot_orb(const void* psi, void* y, const double* V, double pot_scale, double* pp) {
    PassGeom g = gp;
    const int n = p->pp[p->norb];
    if (queue) make_persistent(g, n, p->d_order_p, p->d_perm_p);
    return launch_pot_orb(p->prec, g, n, psi, y, V, pot_scale, p->elems, pp, st);
  }
  // out = W_z^T t + (kmul K_z c + kxy), one launch
  hipError_t zfinal(const void* t, const void* c, const void* kxy, void* out, double kmul,
                    double* ep) {
    Mark mk(p, st, ST_ZFIN);
    PassGeom g = gz;
    const int n = p->pz[p->norb];
    if (queue) make_persistent(g, n, p->d_order_z, p->d_perm_z);
    return launch_zfinal(p->prec, g, n, t, c, kxy, out, p->elems, kmul, ep, st);
  }
  // 3D separable operator: z pass in -> out, y pass out -> tmp, x pass tmp -> out
  hipError_t op3(int op, const void* in, void* out, void* tmp) {
    hipError_t e = pass(op, 3, in, out);
    if (e == hipSuccess) e = pass(op, 2, out, tmp);
    if (e == hipSuccess) e = pass(op, 1, tmp, out);
    return e;
  }
};

#define WVL_CHK(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return hipfail(_e, "kernel launch"); \
  } while (0)

// ---------------------------------------------------------------------------
// Isolated / surface boundary conditions (Sec. 3.1): pass-by-pass sequence on
// arrays whose length along an isolated axis changes (m coefficients, m + 29
// real-space points).  Real-space arrays in the workspace have the plane
// stride elems_rs (compensated float32); coefficient arrays p->elems.
// ---------------------------------------------------------------------------
struct Shape { int n[3]; };   // lengths along axes 1, 2, 3

hipError_t bc_pass(wvl_plan* p, hipStream_t st, int op, int axis, Shape& sh, const void* in,
                   void* out, const void* k0, int64_t plane_in, int64_t plane_out,
                   int64_t plane_k0, double kmul, double* ep) {
  Mark mk(p, st, stage_of(op, axis));
  const int a = axis - 1;
  const bool iso = p->bc_free[a];
  const int m = p->orbs[0].m[a];
  BcPass g{};
  g.orbs = p->d_orbs;
  g.orbs_n = p->norb;
  g.n1 = sh.n[0];
  g.n2 = sh.n[1];
  g.n3 = sh.n[2];
  g.n_in = sh.n[a];
  // global position of output 0 minus that of input 0: the real-space grid
  // of an isolated axis starts 14 fine points before the coefficients
  if (op == OP_CW) { g.n_out = iso ? m + kBcExtra : m; g.d = iso ? -14 : 0; }
  else if (op == OP_CWT) { g.n_out = m; g.d = iso ? 14 : 0; }
  else { g.n_out = m; g.d = 0; }
  g.periodic = iso ? 0 : 1;
  Shape o = sh;
  o.n[a] = g.n_out;
  g.vol_in = (int64_t)sh.n[0] * sh.n[1] * sh.n[2];
  g.vol_out = (int64_t)o.n[0] * o.n[1] * o.n[2];
  if (axis == 1) {
    g.rows_per_tile = bc_rows_per_tile(op, g.n_out);
    g.tiles = (sh.n[1] * sh.n[2] + g.rows_per_tile - 1) / g.rows_per_tile;
  } else {
    const int64_t lines = axis == 3 ? (int64_t)sh.n[0] * sh.n[1] : (int64_t)sh.n[0] * sh.n[2];
    g.tiles = (int)((lines + kThreads - 1) / kThreads);
  }
  g.plane_k0 = plane_k0;
  sh = o;
  return launch_bc_pass(p->prec, op, axis, g, in, out, k0, plane_in, plane_out, kmul, ep, st);
}

// psi = W3 c on the real-space grid, into A (plane elems_rs)
int bc_point_values(wvl_plan* p, hipStream_t st, const void* c, void* A, void* B) {
  const int64_t prs = p->elems_rs;
  Shape sh{{p->orbs[0].m[0], p->orbs[0].m[1], p->orbs[0].m[2]}};
  WVL_CHK(bc_pass(p, st, OP_CW, 3, sh, c, A, nullptr, p->elems, prs, 0, 1.0, nullptr));
  WVL_CHK(bc_pass(p, st, OP_CW, 2, sh, A, B, nullptr, prs, prs, 0, 1.0, nullptr));
  WVL_CHK(bc_pass(p, st, OP_CW, 1, sh, B, A, nullptr, prs, prs, 0, 1.0, nullptr));
  return WVL_OK;
}

// (K_x + K_y + K_z) c + k0 with the kinetic energies <c, K_a c> per tile
int bc_kinetic(wvl_plan* p, hipStream_t st, const void* c, const void* k0, int64_t plane_k0,
               void* tmp, int64_t plane_tmp, void* out, int64_t plane_out, double kmul,
               double* ez, double* ey, double* ex) {
  Shape sh{{p->orbs[0].m[0], p->orbs[0].m[1], p->orbs[0].m[2]}};
  const Shape c_sh = sh;
  WVL_CHK(bc_pass(p, st, OP_CK, 3, sh, c, tmp, k0, p->elems, plane_tmp, plane_k0, kmul, ez));
  sh = c_sh;
  WVL_CHK(bc_pass(p, st, OP_CK, 2, sh, c, tmp, tmp, p->elems, plane_tmp, plane_tmp, kmul, ey));
  sh = c_sh;
  WVL_CHK(bc_pass(p, st, OP_CK, 1, sh, c, out, tmp, p->elems, plane_out, plane_tmp, kmul, ex));
  return WVL_OK;
}

int hpsi_bc(wvl_plan* p, hipStream_t st, const void* c, const double* V, double pot_scale,
            double kin_scale, void* hpsi, double* rho, double* e_loc, double* e_kin, double* e_orb,
            void* ws) {
  void* A = wsp(ws, p->o_A);
  void* B = wsp(ws, p->o_B);
  void* S = wsp(ws, p->o_S);
  double* ez = (double*)wsp(ws, p->o_ez);
  double* ey = (double*)wsp(ws, p->o_ey);
  double* ex = (double*)wsp(ws, p->o_ex);
  double* pp = (double*)wsp(ws, p->o_pp);
  double* rv = (double*)wsp(ws, p->o_rv);
  double* eorb = e_orb ? e_orb : (double*)wsp(ws, p->o_eorb);
  const bool want_e = e_loc || e_kin || e_orb;
  const int64_t prs = p->elems_rs;
  // steps 2 + 3a: psi on the real-space grid
  if (int r = bc_point_values(p, st, c, A, B)) return r;
  // step 3b and the density: y = pot_scale V psi in place
  {
    Mark mk(p, st, ST_POT);
    WVL_CHK(launch_pot_shared(p->prec, p->d_orbs_rs, p->norb, p->Mrs, A, A, V, pot_scale, prs, rho,
                              0, want_e ? rv : nullptr, e_orb ? pp : nullptr, st));
  }
  // steps 3c + 6: back onto the coefficients
  Shape sh{{p->Mr[0], p->Mr[1], p->Mr[2]}};
  WVL_CHK(bc_pass(p, st, OP_CWT, 1, sh, A, B, nullptr, prs, prs, 0, 1.0, nullptr));
  WVL_CHK(bc_pass(p, st, OP_CWT, 2, sh, B, A, nullptr, prs, prs, 0, 1.0, nullptr));
  WVL_CHK(bc_pass(p, st, OP_CWT, 3, sh, A, B, nullptr, prs, prs, 0, 1.0, nullptr));
  // steps 4 + 5: the kinetic operator on the coefficients, accumulated onto B
  if (int r = bc_kinetic(p, st, c, B, prs, S, prs, hpsi, p->elems, kin_scale,
                         want_e ? ez : nullptr, want_e ? ey : nullptr, want_e ? ex : nullptr))
    return r;
  if (want_e) {
    Mark mk(p, st, ST_ENERGY);
    const int32_t* pbx = p->d_pb;
    const int32_t* pby = p->d_pb + (p->norb + 1);
    const int32_t* pbz = p->d_pb + 2 * (p->norb + 1);
    WVL_CHK(launch_orb_sums(p->d_orbs, p->norb, pbz, pby, pbx, ez, ey, ex, pp, e_orb ? 2 : 0,
                            p->d_pp, p->nblk, eorb, st));
    if (e_loc || e_kin)
      WVL_CHK(launch_totals(p->d_orbs, p->norb, eorb, rv, p->nblk, e_loc, e_kin, st));
  }
  return WVL_OK;
}

// Local H*psi of the compensated form with exact digit products (wvl_oz.hip):
// potential as float pairs; u = W_z c; the in-plane kernel (psi, rho, e_pot,
// t, kxy); the density reduction; Hc = W_z^T t + kin_scale k (K_z c + kxy).
int hpsi_oz(wvl_plan* p, hipStream_t st, const void* c, const double* V, double pot_scale,
            double kin_scale, void* hpsi, double* rho, double* e_loc, double* e_kin, double* e_orb,
            void* ws) {
  const bool want_e = e_loc || e_kin || e_orb;
  double* rhop = (double*)wsp(ws, p->o_rhop);
  double* rv = (double*)wsp(ws, p->o_rv);
  double* eorb = e_orb ? e_orb : (double*)wsp(ws, p->o_eorb);
  const OzLds l = oz_lds(p->orbs[0].m[0], p->orbs[0].m[1], p->orbs[0].m[2]);
  OzArgs a{};
  a.orbs = p->d_orbs;
  a.norb = p->norb;
  a.m1 = p->orbs[0].m[0];
  a.m2 = p->orbs[0].m[1];
  a.m3 = p->orbs[0].m[2];
  a.c = (const float*)c;
  a.out = (float*)hpsi;
  a.u = (float*)wsp(ws, p->o_A);
  a.t = (float*)wsp(ws, p->o_B);
  a.kxy = (float*)wsp(ws, p->o_S);
  a.plane = p->elems;
  float* vhl = (float*)wsp(ws, p->o_ozv);
  int* vexp = (int*)wsp(ws, p->o_oze);
  a.vhl = vhl;
  a.vexp = vexp;
  a.M = p->M;
  int pe = 0;
  if (pot_scale != 0.0) (void)frexp(pot_scale, &pe);   // |pot_scale| <= 2^pe
  a.pexp = pe;
  a.ps_hi = (float)pot_scale;
  a.ps_lo = (float)(pot_scale - (double)a.ps_hi);
  a.ps_scaled = pot_scale != 1.0;
  a.kin_mul = kin_scale;
  a.rho_part = rhop;
  a.ngroups = p->xy_ngroups;
  a.G = p->xy_G;
  a.epot = (double*)wsp(ws, p->o_epl);
  a.pq = p->d_pq;
  a.ekin = (double*)wsp(ws, p->o_kpl2);
  a.dxy = l.dxy;
  a.dz = l.dz;
  {
    Mark mk(p, st, ST_POT);
    WVL_CHK(launch_oz_vprep(V, a.m1 * a.m2, a.m3, vhl, p->M, vexp, st));
  }
  {
    Mark mk(p, st, stage_of(OP_CW, 3));
    WVL_CHK(launch_oz_z(a, st));
  }
  {
    Mark mk(p, st, ST_XY);
    WVL_CHK(launch_oz_xy(a, st));
  }
  if (rho || want_e) {
    Mark mk(p, st, ST_RHO);
    WVL_CHK(launch_rho_reduce(rhop, p->xy_ngroups, p->M, V, rho, want_e ? rv : nullptr, st));
  }
  {
    Mark mk(p, st, ST_ZFIN);
    WVL_CHK(launch_oz_zfinal(a, p->oz_occ_z, st));
  }
  if (want_e) {
    Mark mk(p, st, ST_ENERGY);
    // kinetic: per xz-plane sums; potential: per z-plane sums
    WVL_CHK(launch_orb_sums(p->d_orbs, p->norb, p->d_pxz, nullptr, nullptr, a.ekin, nullptr,
                            nullptr, a.epot, 1, p->d_pq, 0, eorb, st));
    if (e_loc || e_kin)
      WVL_CHK(launch_totals(p->d_orbs, p->norb, eorb, rv, p->nblk, e_loc, e_kin, st));
  }
  return WVL_OK;
}

// The local H*psi launch sequence (Sec. 2.4 steps 2-6 with the density of
// Sec. 2.5 and the float64 energies).  hpsi may be c itself: then the last z
// step runs as two passes (the fused one would overwrite c at the start of a
// z line before its periodic wrap reads it back).
int hpsi_sequence(wvl_plan* p, hipStream_t st, const void* c, const double* V, double pot_scale,
                  double kin_scale, void* hpsi, double* rho, double* e_loc, double* e_kin,
                  double* e_orb, void* ws) {
  if (p->bc_any)
    return hpsi_bc(p, st, c, V, pot_scale, kin_scale, hpsi, rho, e_loc, e_kin, e_orb, ws);
  if (p->use_oz)
    return hpsi_oz(p, st, c, V, pot_scale, kin_scale, hpsi, rho, e_loc, e_kin, e_orb, ws);
  Seq q(p, st);
  void* A = wsp(ws, p->o_A);
  void* B = wsp(ws, p->o_B);
  void* S = wsp(ws, p->o_S);
  double* ez = (double*)wsp(ws, p->o_ez);
  double* ey = (double*)wsp(ws, p->o_ey);
  double* ex = (double*)wsp(ws, p->o_ex);
  double* pp = (double*)wsp(ws, p->o_pp);
  double* rv = (double*)wsp(ws, p->o_rv);
  double* eorb = e_orb ? e_orb : (double*)wsp(ws, p->o_eorb);
  const bool want_e = e_loc || e_kin || e_orb;
  if (p->persistent) {
    int32_t* queue = (int32_t*)wsp(ws, p->o_queue);
    WVL_CHK(launch_fill_int(queue, kQueueCounters, st));
    q.queue = queue;
    q.queue_end = queue + kQueueCounters;
  }
  if (p->use_xy) {
    // z pass: u = W_z c; planes: psi, rho, y, t = W_y^T W_x^T y, kxy;
    // z passes: kxy += K_z c, then Hc = W_z^T t + kxy
    double* epl = (double*)wsp(ws, p->o_epl);
    double* kpl = (double*)wsp(ws, p->o_kpl);
    double* rhop = p->shared ? (double*)wsp(ws, p->o_rhop) : nullptr;
    WVL_CHK(q.pass(OP_CW, 3, c, A));
    {
      XyArgs xa;
      xa.orbs = p->d_orbs;
      xa.pq = p->d_pq;
      xa.norb = p->norb;
      xa.shared = p->shared ? 1 : 0;
      xa.ngroups = p->xy_ngroups;
      xa.G = p->xy_G;
      xa.M = p->M;
      xa.u = A;
      xa.c = c;
      xa.t = B;
      xa.kxy = S;
      xa.V = V;
      xa.pot_scale = pot_scale;
      xa.kin_mul = kin_scale;
      xa.plane = p->elems;
      xa.rho_part = rhop;
      xa.epot = epl;
      xa.ekin = kpl;
      xa.occupancy = p->xy_occ;
      xa.engine = p->xy_engine;
      xa.rho_lds = 0;
      xa.order = nullptr;
      xa.perm = nullptr;
      xa.queue = nullptr;
      xa.ntiles = p->xy_blocks;
      int nblocks = p->xy_blocks;
      if (q.queue && !p->shared && q.queue < q.queue_end) {
        xa.order = p->d_order_q;
        xa.perm = p->d_perm_q;
        xa.queue = q.queue++;
        const size_t lds = xy_lds_bytes(p->prec, p->xy_m1, p->xy_m2, p->xy_engine != 0);
        const int per_cu = std::max(1, std::min(p->xy_occ / 2, (int)(p->ctx->lds_per_block / lds)));
        nblocks = std::min(nblocks, std::max(1, p->ctx->cus) * per_cu);
      }
      if (p->shared && p->xy_engine) {
        // matrix-core engine: one launch, each workgroup runs its group's
        // orbitals in turn
        Mark mk(p, st, ST_XY);
        xa.slot = -1;
        WVL_CHK(launch_xy(p->prec, xa, p->xy_m1, p->xy_m2, p->xy_blocks, st));
      } else if (p->shared) {
        for (int slot = 0; slot < p->xy_G; ++slot) {
          Mark mk(p, st, ST_XY);
          xa.slot = slot;
          WVL_CHK(launch_xy(p->prec, xa, p->xy_m1, p->xy_m2, p->xy_blocks, st));
        }
      } else {
        Mark mk(p, st, ST_XY);
        xa.slot = 0;
        WVL_CHK(launch_xy(p->prec, xa, p->xy_m1, p->xy_m2, nblocks, st));
      }
    }
    if (p->shared && (rho || want_e)) {
      Mark mk(p, st, ST_RHO);
      WVL_CHK(launch_rho_reduce(rhop, p->xy_ngroups, p->M, V, rho, want_e ? rv : nullptr, st));
    }
    if (p->zfuse && hpsi != c) {
      WVL_CHK(q.zfinal(B, c, S, hpsi, kin_scale, want_e ? ez : nullptr));
    } else {
      WVL_CHK(q.pass(OP_CK, 3, c, S, S, kin_scale, want_e ? ez : nullptr));
      WVL_CHK(q.pass(OP_CWT, 3, B, hpsi, S));
    }
    if (want_e) {
      Mark mk(p, st, ST_ENERGY);
      // kinetic: z-pass tiles + per-plane in-plane sums; potential: per plane
      WVL_CHK(launch_orb_sums(p->d_orbs, p->norb, p->d_pz, p->d_pq, nullptr, ez, kpl, nullptr, epl,
                              1, p->d_pq, 0, eorb, st));
      if (e_loc || e_kin)
        WVL_CHK(launch_totals(p->d_orbs, p->norb, eorb, rv, p->shared ? p->nblk : 0, e_loc, e_kin, st));
    }
    return WVL_OK;
  }
  // steps 2 + 3a with the combined filter (synthesis then magic filter per
  // axis): psi = W3 c (z: c -> A, y: A -> B, x: B -> B)
  WVL_CHK(q.pass(OP_CW, 3, c, A));
  WVL_CHK(q.pass(OP_CW, 2, A, B));
  WVL_CHK(q.pass(OP_CW, 1, B, B));
  // step 3b and density: y = pot_scale V psi in place
  {
    Mark mk(p, st, ST_POT);
    if (p->shared) {
      WVL_CHK(launch_pot_shared(p->prec, p->d_orbs, p->norb, p->M, B, B, V, pot_scale, p->elems,
                                rho, 0, want_e ? rv : nullptr, e_orb ? pp : nullptr, st));
    } else {
      WVL_CHK(q.pot_orb(B, B, V, pot_scale, want_e ? pp : nullptr));
    }
  }
  // steps 3c + 6 combined (transposed magic filter then analysis): W3^T y
  WVL_CHK(q.pass(OP_CWT, 3, B, A));
  WVL_CHK(q.pass(OP_CWT, 2, A, B));
  WVL_CHK(q.pass(OP_CWT, 1, B, B));
  // steps 4 + 5: the kinetic operator on the coefficients, A Kin S per axis,
  // accumulated onto W3^T y (the K_0 initialisation of the kinetic recursion)
  WVL_CHK(q.pass(OP_CK, 3, c, A, B, kin_scale, want_e ? ez : nullptr));
  WVL_CHK(q.pass(OP_CK, 2, c, A, A, kin_scale, want_e ? ey : nullptr));
  WVL_CHK(q.pass(OP_CK, 1, c, hpsi, A, kin_scale, want_e ? ex : nullptr));
  (void)S;
  if (want_e) {
    Mark mk(p, st, ST_ENERGY);
    const int pot_mode = p->shared ? (e_orb ? 2 : 0) : 1;
    WVL_CHK(launch_orb_sums(p->d_orbs, p->norb, p->d_pz, p->d_py,
                            p->xdiv == 2 ? p->d_px2 : p->d_px, ez, ey, ex, pp, pot_mode,
                            p->d_pp, p->nblk, eorb, st));
    if (e_loc || e_kin)
      WVL_CHK(launch_totals(p->d_orbs, p->norb, eorb, rv, p->shared ? p->nblk : 0, e_loc, e_kin, st));
  }
  return WVL_OK;
}

// Launch candidates of wvl_local_hpsi, timed on the plan's own batch (zero
// data: no kernel's work depends on values).  Candidate k = 3 * seq + shape:
//   seq 0: one 1D pass per axis and operator;
//   seq 1: plane-resident kernel, 4 waves per SIMD, default engine;
//   seq 2: plane-resident kernel, 2 waves per SIMD, default engine;
//   seq 3: plane-resident kernel, 4 waves per SIMD, vector FMA engine
//          (float64 only, where the matrix-core engine is the default);
//   shape 0: default tiles (axis-1 tiles as many rows as fit in LDS;
//            persistent launches of 8 workgroups per CU);
//   shape 1: axis-1 tiles of half as many rows (seq 0 only: the other
//            sequences have no axis-1 pass);
//   shape 2: persistent launches of 4 workgroups per CU (persistent plans).
// Unavailable candidates get -1.  The fastest one is kept.
struct Cand { bool xy; int occ, engine, xdiv, pmul; bool oz; };

void apply_cand(wvl_plan* p, const Cand& c) {
  p->use_oz = c.oz;
  p->use_xy = c.xy;
  p->xy_occ = c.occ;
  p->xy_engine = c.engine;
  p->xdiv = c.xdiv;
  p->pgrid_mul = c.pmul;
  p->pgrid_pass = std::max(1, p->ctx->cus) * c.pmul;
  p->variant = c.oz ? 3 : c.xy ? 1 + c.engine : 0;
}

int autotune(wvl_plan* p) {
  const bool mx = xy_matrix_engine(p->prec, p->xy_m1, p->xy_m2);
  const bool plane_ok = xy_supported(p->prec, p->xy_m1, p->xy_m2, mx) && !getenv("WVL_NO_PLANE_KERNEL");
  const bool vec_ok = xy_supported(p->prec, p->xy_m1, p->xy_m2, false) && !getenv("WVL_NO_PLANE_KERNEL");
  const Cand seqs[5] = {{false, 4, 0, 1, 8, false}, {true, 4, mx ? 1 : 0, 1, 8, false},
                        {true, 2, mx ? 1 : 0, 1, 8, false}, {true, 4, 0, 1, 8, false},
                        {false, 4, 0, 1, 8, true}};
  const bool seq_ok[5] = {true, plane_ok, plane_ok, mx && vec_ok, p->oz_ok};
  const size_t es = p->prec == WVL_F32 ? 4 : 8;
  const size_t arr = (size_t)p->elems * (p->prec == WVL_F32C ? 8 : es);
  const size_t vbytes = sizeof(double) * (size_t)(p->shared ? p->Mrs : std::max<int64_t>(p->vlen, 1));
  void *c = nullptr, *out = nullptr, *ws = nullptr, *V = nullptr, *e = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t err = dev_malloc(&c, arr);
  if (err == hipSuccess) err = dev_malloc(&out, arr);
  if (err == hipSuccess) err = dev_malloc(&ws, p->ws);
  if (err == hipSuccess) err = dev_malloc(&V, vbytes);
  if (err == hipSuccess) err = dev_malloc(&e, 4 * sizeof(double));
  if (err == hipSuccess) err = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (err == hipSuccess) err = hipEventCreate(&t0);
  if (err == hipSuccess) err = hipEventCreate(&t1);
  if (err == hipSuccess) err = hipMemsetAsync(c, 0, arr, st);
  if (err == hipSuccess) err = hipMemsetAsync(V, 0, vbytes, st);
  int status = WVL_OK;
  if (err != hipSuccess) status = hipfail(err, "autotune buffers");
  const Cand keep{p->use_xy, p->xy_occ, p->xy_engine, p->xdiv, p->pgrid_mul, p->use_oz};
  int best = -1;
  double best_ms = 0.0;
  p->tune_ms.assign(kTuneCands, -1.0);
  for (int k = 0; k < kTuneCands && status == WVL_OK; ++k) {
    const int seq = k / 3, shape = k % 3;
    if (!seq_ok[seq]) continue;
    if (shape == 1 && seq != 0) continue;
    if (shape == 2 && (!p->persistent || seq == 4)) continue;
    Cand cd = seqs[seq];
    if (shape == 1) cd.xdiv = 2;
    if (shape == 2) cd.pmul = 4;
    apply_cand(p, cd);
    double* ed = (double*)e;
    status = hpsi_sequence(p, st, c, (const double*)V, 1.0, 1.0, out, nullptr, ed, ed + 1,
                           nullptr, ws);   // warm-up
    if (status != WVL_OK) break;
    constexpr int kReps = 3;
    err = hipEventRecord(t0, st);
    for (int r = 0; r < kReps && status == WVL_OK && err == hipSuccess; ++r)
      status = hpsi_sequence(p, st, c, (const double*)V, 1.0, 1.0, out, nullptr, ed, ed + 1,
                             nullptr, ws);
    if (status != WVL_OK) break;
    if (err == hipSuccess) err = hipEventRecord(t1, st);
    if (err == hipSuccess) err = hipEventSynchronize(t1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, t0, t1);
    if (err != hipSuccess) { status = hipfail(err, "autotune timing"); break; }
    p->tune_ms[k] = ms / kReps;
    if (best < 0 || p->tune_ms[k] < best_ms) { best = k; best_ms = p->tune_ms[k]; }
  }
  if (best >= 0 && status == WVL_OK) {
    Cand cd = seqs[best / 3];
    if (best % 3 == 1) cd.xdiv = 2;
    if (best % 3 == 2) cd.pmul = 4;
    apply_cand(p, cd);
    p->tune_best = best;
  } else {
    apply_cand(p, keep);
  }
  if (st) (void)hipStreamSynchronize(st);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (st) (void)hipStreamDestroy(st);
  for (void* q : {c, out, ws, V, e})
    if (q) (void)hipFree(q);
  return status;
}

}  // namespace

extern "C" {

int wvl_synthesis(wvl_plan* p, const void* c, void* s, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!c || !s || !ws) return fail(WVL_EINVAL, "wvl_synthesis: NULL pointer");
  if (int r = check_aligned("wvl_synthesis", {c, s})) return r;
  if (int r = check_disjoint(p, c, s, "wvl_synthesis")) return r;
  if (int r = check_periodic(p, "wvl_synthesis")) return r;
  if (int r = check_gpu(p)) return r;
  Seq q(p, (hipStream_t)stream);
  WVL_CHK(q.op3(OP_SYN, c, s, wsp(ws, p->o_A)));
  return WVL_OK;
}

int wvl_analysis(wvl_plan* p, const void* s, void* c, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!c || !s || !ws) return fail(WVL_EINVAL, "wvl_analysis: NULL pointer");
  if (int r = check_aligned("wvl_analysis", {c, s})) return r;
  if (int r = check_disjoint(p, s, c, "wvl_analysis")) return r;
  if (int r = check_periodic(p, "wvl_analysis")) return r;
  if (int r = check_gpu(p)) return r;
  Seq q(p, (hipStream_t)stream);
  WVL_CHK(q.op3(OP_ANA, s, c, wsp(ws, p->o_A)));
  return WVL_OK;
}

int wvl_magic_filter(wvl_plan* p, const void* in, void* out, int transpose, void* ws,
                     void* stream) {
  if (int r = check_plan(p)) return r;
  if (!in || !out || !ws) return fail(WVL_EINVAL, "wvl_magic_filter: NULL pointer");
  if (int r = check_aligned("wvl_magic_filter", {in, out})) return r;
  if (int r = check_disjoint(p, in, out, "wvl_magic_filter")) return r;
  if (int r = check_periodic(p, "wvl_magic_filter")) return r;
  if (int r = check_gpu(p)) return r;
  Seq q(p, (hipStream_t)stream);
  WVL_CHK(q.op3(transpose ? OP_MFT : OP_MF, in, out, wsp(ws, p->o_A)));
  return WVL_OK;
}

int wvl_kinetic(wvl_plan* p, const void* s, const void* k0, void* out, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!s || !out || !ws) return fail(WVL_EINVAL, "wvl_kinetic: NULL pointer");
  if (int r = check_aligned("wvl_kinetic", {s, k0, out})) return r;
  if (int r = check_disjoint(p, s, out, "wvl_kinetic")) return r;
  if (int r = check_periodic(p, "wvl_kinetic")) return r;
  if (k0 && overlap(k0, batch_bytes(p), s, batch_bytes(p)))
    return fail(WVL_EINVAL, "wvl_kinetic: k0 overlaps s");
  if (k0 && k0 != out && overlap(k0, batch_bytes(p), out, batch_bytes(p)))
    return fail(WVL_EINVAL, "wvl_kinetic: k0 overlaps out without being out");
  if (int r = check_gpu(p)) return r;
  Seq q(p, (hipStream_t)stream);
  WVL_CHK(q.pass(OP_KIN, 3, s, out, k0));
  WVL_CHK(q.pass(OP_KIN, 2, s, out, out));
  WVL_CHK(q.pass(OP_KIN, 1, s, out, out));
  return WVL_OK;
}

int wvl_local_density(wvl_plan* p, const void* c, double* rho, int accumulate, void* ws,
                      void* stream) {
  if (int r = check_plan(p)) return r;
  if (!c || !rho || !ws) return fail(WVL_EINVAL, "wvl_local_density: NULL pointer");
  if (int r = check_aligned("wvl_local_density", {c})) return r;
  if (!p->shared) return fail(WVL_EUNSUPPORTED, "wvl_local_density needs a WVL_SHARED_V plan");
  if (int r = check_gpu(p)) return r;
  hipStream_t st = (hipStream_t)stream;
  Seq q(p, st);
  void* A = wsp(ws, p->o_A);
  void* B = wsp(ws, p->o_B);
  if (p->bc_any) {
    if (int r = bc_point_values(p, st, c, A, B)) return r;
    WVL_CHK(launch_pot_shared(p->prec, p->d_orbs_rs, p->norb, p->Mrs, A, nullptr, nullptr, 1.0,
                              p->elems_rs, rho, accumulate, nullptr, nullptr, st));
    return WVL_OK;
  }
  WVL_CHK(q.pass(OP_SYN, 3, c, A));
  WVL_CHK(q.pass(OP_SYN, 2, A, B));
  WVL_CHK(q.pass(OP_SYN, 1, B, B));
  WVL_CHK(q.pass(OP_MF, 3, B, A));
  WVL_CHK(q.pass(OP_MF, 2, A, B));
  WVL_CHK(q.pass(OP_MF, 1, B, B));
  WVL_CHK(launch_pot_shared(p->prec, p->d_orbs, p->norb, p->M, B, nullptr, nullptr, 1.0, p->elems,
                            rho, accumulate, nullptr, nullptr, st));
  return WVL_OK;
}

int wvl_local_hpsi(wvl_plan* p, const void* c, const double* V, double pot_scale,
                   double kin_scale, void* hpsi, double* rho, double* e_loc, double* e_kin,
                   double* e_orb, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!c || !V || !hpsi || !ws) return fail(WVL_EINVAL, "wvl_local_hpsi: NULL pointer");
  if (int r = check_aligned("wvl_local_hpsi", {c, hpsi})) return r;
  if (rho && !p->shared) return fail(WVL_EUNSUPPORTED, "rho needs a WVL_SHARED_V plan");
  if (!isfinite(pot_scale) || !isfinite(kin_scale))
    return fail(WVL_EINVAL, "wvl_local_hpsi: scales must be finite");
  if (hpsi != c && overlap(c, batch_bytes(p), hpsi, batch_bytes(p)))
    return fail(WVL_EINVAL, "wvl_local_hpsi: hpsi overlaps c without being c");
  if (int r = check_gpu(p)) return r;
  hipStream_t st = (hipStream_t)stream;
  if (!(p->flags & WVL_USE_GRAPH))
    return hpsi_sequence(p, st, c, V, pot_scale, kin_scale, hpsi, rho, e_loc, e_kin, e_orb, ws);
  // graph path: record once per pointer set on a private stream, replay after
  GraphKey key{};
  key.p[0] = c; key.p[1] = V; key.p[2] = hpsi; key.p[3] = rho; key.p[4] = e_loc;
  key.p[5] = e_kin; key.p[6] = e_orb; key.p[7] = ws;
  key.s[0] = pot_scale; key.s[1] = kin_scale;
  if (!p->gstream) {
    WVL_HIP(hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
    WVL_HIP(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
    WVL_HIP(hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming));
  }
  if (!p->gexec || !(key == p->gkey)) {
    if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
    hipGraph_t g;
    WVL_HIP(hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal));
    p->capturing = true;
    int r = hpsi_sequence(p, p->gstream, c, V, pot_scale, kin_scale, hpsi, rho, e_loc, e_kin,
                          e_orb, ws);
    p->capturing = false;
    hipError_t e = hipStreamEndCapture(p->gstream, &g);
    if (r != WVL_OK) { if (e == hipSuccess) (void)hipGraphDestroy(g); return r; }
    if (e != hipSuccess) return hipfail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { p->gexec = nullptr; return hipfail(e, "hipGraphInstantiate"); }
    p->gkey = key;
  }
  WVL_HIP(hipEventRecord(p->ev_in, st));
  WVL_HIP(hipStreamWaitEvent(p->gstream, p->ev_in, 0));
  WVL_HIP(hipGraphLaunch(p->gexec, p->gstream));
  WVL_HIP(hipEventRecord(p->ev_out, p->gstream));
  WVL_HIP(hipStreamWaitEvent(st, p->ev_out, 0));
  return WVL_OK;
}

int wvl_energy_gradient(wvl_plan* p, const void* c, const double* V, double g_loc, double g_kin,
                        void* grad, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!c || !V || !grad || !ws) return fail(WVL_EINVAL, "wvl_energy_gradient: NULL pointer");
  if (int r = check_aligned("wvl_energy_gradient", {c, grad})) return r;
  if (!isfinite(g_loc) || !isfinite(g_kin))
    return fail(WVL_EINVAL, "wvl_energy_gradient: weights must be finite");
  if (grad != c && overlap(c, batch_bytes(p), grad, batch_bytes(p)))
    return fail(WVL_EINVAL, "wvl_energy_gradient: grad overlaps c without being c");
  if (int r = check_gpu(p)) return r;
  hipStream_t st = (hipStream_t)stream;
  // 2 f_b (g_loc Hloc + g_kin Kin) c_b: with one occupation for every orbital
  // the weights fold into the two operator scales, otherwise the orbitals are
  // scaled by f_b afterwards
  const double f = p->occ_uniform ? p->orbs[0].occ : 1.0;
  if (int r = hpsi_sequence(p, st, c, V, 2.0 * f * g_loc, 2.0 * f * g_kin, grad, nullptr, nullptr,
                            nullptr, nullptr, ws))
    return r;
  if (!p->occ_uniform) {
    PassGeom g{p->d_orbs, p->d_pp, p->norb};
    hipError_t e = launch_scale_occ(p->prec, g, p->pp[p->norb], grad, 1.0, p->elems, st);
    if (e != hipSuccess) return hipfail(e, "occupation weights");
  }
  return WVL_OK;
}

// Operator form of the preconditioner's fused (combined-filter) step:
//   0 one combined-filter pass per axis;
//   1 the plane-resident form: z pass, then both in-plane passes with the
//     plane of p in LDS (periodic plans whose planes fit the in-plane kernel);
//   2 the same two launches with the exact digit products (compensated
//     uniform periodic plans that the engine covers).
static int precond_form(const wvl_plan* p, uint32_t mode) {
  if ((mode & (WVL_PRECOND_SEPARATE | WVL_PRECOND_PASSES)) || p->bc_any) return 0;
  if (p->oz_pc) return 2;
  const bool mx = xy_matrix_engine(p->prec, p->xy_m1, p->xy_m2) && !getenv("WVL_XY_VECTOR");
  return p->xy_ok && xy_supported(p->prec, p->xy_m1, p->xy_m2, mx) ? 1 : 0;
}

int wvl_precondition(wvl_plan* p, const void* g, const double* eps, int32_t iters, uint32_t mode,
                     void* gt, double* res, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!g || !eps || !gt || !ws) return fail(WVL_EINVAL, "wvl_precondition: NULL pointer");
  if (int r = check_aligned("wvl_precondition", {g, gt})) return r;
  if (iters < 0 || iters > 10000) return fail(WVL_EINVAL, "wvl_precondition: iters = %d", iters);
  if (mode & ~(uint32_t)(WVL_PRECOND_SEPARATE | WVL_PRECOND_PASSES))
    return fail(WVL_EINVAL, "wvl_precondition: unknown mode bits 0x%x", mode);
  if ((mode & WVL_PRECOND_SEPARATE) && (mode & WVL_PRECOND_PASSES))
    return fail(WVL_EINVAL, "wvl_precondition: WVL_PRECOND_SEPARATE and WVL_PRECOND_PASSES exclude each other");
  if (p->bc_any && (mode & WVL_PRECOND_SEPARATE))
    return fail(WVL_EUNSUPPORTED, "wvl_precondition: the separate-pass form is periodic only");
  for (int b = 0; b < p->norb; ++b)
    if (!(eps[b] < 0.0) || !isfinite(eps[b]))
      return fail(WVL_EINVAL, "wvl_precondition: eps[%d] = %g must be negative and finite", b,
                  eps[b]);
  if (int r = check_disjoint(p, g, gt, "wvl_precondition")) return r;
  if (int r = check_gpu(p)) return r;
  hipStream_t st = (hipStream_t)stream;
  Seq q(p, st);   // ordinary (not persistent) pass launches
  void* R = wsp(ws, p->o_A);
  void* Pv = wsp(ws, p->o_B);
  void* Q = wsp(ws, p->o_S);
  void* D = wsp(ws, p->o_D);
  const CgLayout cl = cg_layout(p);
  double* prz = (double*)wsp(ws, p->o_cg + cl.rz);
  double* ppp = (double*)wsp(ws, p->o_cg + cl.pp);
  double* prr = (double*)wsp(ws, p->o_cg + cl.rr);
  double* eps_d = (double*)wsp(ws, p->o_cg + cl.eps);
  void* sc = wsp(ws, p->o_cg + cl.sc);
  double* ez = (double*)wsp(ws, p->o_ez);
  double* ey = (double*)wsp(ws, p->o_ey);
  double* ex = (double*)wsp(ws, p->o_ex);
  const PassGeom gp{p->d_orbs, p->d_pc, p->norb};
  const int nt = p->pc[p->norb];
  const int64_t plane = p->elems;
  const bool separate = (mode & WVL_PRECOND_SEPARATE) != 0;
  const bool helm_mx = xy_matrix_engine(p->prec, p->xy_m1, p->xy_m2) && !getenv("WVL_XY_VECTOR");
  const int form = precond_form(p, mode);
  const bool exact = form == 2, plane_form = form == 1;
  double* kpl = plane_form || exact ? (double*)wsp(ws, p->o_kpl) : nullptr;
  OzHelmArgs oa{};
  if (exact) {
    const OzLds l = oz_lds(p->orbs[0].m[0], p->orbs[0].m[1], p->orbs[0].m[2]);
    oa.orbs = p->d_orbs;
    oa.norb = p->norb;
    oa.m1 = p->orbs[0].m[0];
    oa.m2 = p->orbs[0].m[1];
    oa.m3 = p->orbs[0].m[2];
    oa.p = (const float*)Pv;
    oa.q = (float*)Q;
    oa.plane = plane;
    oa.ez = (double*)wsp(ws, p->o_kpl2);
    oa.exy = kpl;
    oa.dxy = l.dxy;
    oa.dz = l.dz;
  }
  WVL_HIP(hipMemcpyAsync(eps_d, eps, sizeof(double) * p->norb, hipMemcpyHostToDevice, st));
  WVL_CHK(launch_cg_init(p->prec, gp, nt, g, gt, R, Pv, eps_d, plane, prz, ppp, prr, st));
  for (int it = 0; it < iters; ++it) {
    // q = (A Kin S - eps) p, with the kinetic energy partials p.Kin p
    if (p->bc_any) {
      if (int r = bc_kinetic(p, st, Pv, nullptr, plane, Q, plane, Q, plane, 1.0, ez, ey, ex)) return r;
    } else if (exact) {
      // the same with the exact digit products: k K_z p over xz-planes,
      // then k (K_x + K_y) p added plane by plane
      Mark mk(p, st, ST_HELM);
      WVL_CHK(launch_oz_helm(oa, st));
    } else if (plane_form) {
      // K_z p by the z pass, then (K_x + K_y) p added plane by plane
      WVL_CHK(q.pass(OP_CK, 3, Pv, Q, nullptr, 1.0, ez));
      Mark mk(p, st, ST_HELM);
      HelmArgs ha{p->d_orbs, p->d_pq, p->norb, Pv, Q, plane, kpl};
      WVL_CHK(launch_helm_xy(p->prec, ha, p->xy_m1, p->xy_m2, p->pq[p->norb], helm_mx, st));
    } else if (!separate) {
      // combined filter (analysis o kinetic o synthesis) per axis, on the
      // coefficients; q = Kin p here, the shift is applied in the update
      WVL_CHK(q.pass(OP_CK, 3, Pv, Q, nullptr, 1.0, ez));
      WVL_CHK(q.pass(OP_CK, 2, Pv, Q, Q, 1.0, ey));
      WVL_CHK(q.pass(OP_CK, 1, Pv, Q, Q, 1.0, ex));
    } else {
      // the separate operations: s = S p, K = Kin s + K_0 with K_0 = -eps s
      // (Sec. 3.4), q = A K
      WVL_CHK(q.op3(OP_SYN, Pv, Q, D));
      WVL_CHK(launch_cg_shift(p->prec, gp, nt, Q, D, eps_d, plane, st));
      WVL_CHK(q.pass(OP_KIN, 3, Q, D, D, 1.0, ez));
      WVL_CHK(q.pass(OP_KIN, 2, Q, D, D, 1.0, ey));
      WVL_CHK(q.pass(OP_KIN, 1, Q, D, D, 1.0, ex));
      WVL_CHK(q.op3(OP_ANA, D, Q, D));
    }
    {
      Mark mk(p, st, ST_CG);
      if (p->bc_any)
        WVL_CHK(launch_cg_alpha(p->norb, p->d_pb + 2 * (p->norb + 1), p->d_pb + (p->norb + 1), p->d_pb,
                                p->d_pc, ez, ey, ex, prz, ppp, eps_d, sc, st));
      else if (exact)
        WVL_CHK(launch_cg_alpha(p->norb, p->d_pxz, p->d_pq, nullptr, p->d_pc, oa.ez, kpl, nullptr,
                                prz, ppp, eps_d, sc, st));
      else if (plane_form)
        WVL_CHK(launch_cg_alpha(p->norb, p->d_pz, p->d_pq, nullptr, p->d_pc, ez, kpl, nullptr, prz,
                                ppp, eps_d, sc, st));
      else
        WVL_CHK(launch_cg_alpha(p->norb, p->d_pz, p->d_py, p->xdiv == 2 ? p->d_px2 : p->d_px,
                                p->d_pc, ez, ey, ex, prz, ppp, eps_d, sc, st));
      WVL_CHK(launch_cg_update1(p->prec, gp, nt, gt, R, Pv, Q, eps_d, separate ? 0 : 1, sc, plane,
                                prz, prr, st));
      WVL_CHK(launch_cg_beta(p->norb, p->d_pc, prz, sc, st));
      WVL_CHK(launch_cg_update2(p->prec, gp, nt, R, Pv, eps_d, sc, plane, ppp, st));
    }
  }
  if (res) WVL_CHK(launch_cg_res(p->norb, p->d_pc, prr, res, st));
  return WVL_OK;
}

// ---------------------------------------------------------------------------
// Compressed storage (Sec. 2.1; steps 1 and 7 of Sec. 2.4)
// ---------------------------------------------------------------------------
static int check_segments(const int32_t* seg, int32_t nseg, int64_t npts, const char* what,
                          int64_t* count) {
  if (nseg < 0) return fail(WVL_EINVAL, "%s: negative segment count", what);
  if (nseg > 0 && !seg) return fail(WVL_EINVAL, "%s: NULL segments", what);
  int64_t prev = 0, n = 0;
  for (int32_t k = 0; k < nseg; ++k) {
    const int64_t a = seg[2 * k], b = seg[2 * k + 1];
    if (a < prev || b <= a || b > npts)
      return fail(WVL_EINVAL, "%s: segment %d [%lld, %lld) out of order or outside [0, %lld)", what,
                  k, (long long)a, (long long)b, (long long)npts);
    n += b - a;
    prev = b;
  }
  *count = n;
  return WVL_OK;
}

int wvl_plan_set_regions(wvl_plan* p, const int32_t* seg_c, int32_t nseg_c, const int32_t* seg_f,
                         int32_t nseg_f) {
  if (int r = check_plan(p)) return r;
  if (p->M == 0) return fail(WVL_EUNSUPPORTED, "regions need every orbital on the same grid");
  const int64_t npts = p->M / 8;
  int64_t nvc = 0, nvf = 0;
  if (int r = check_segments(seg_c, nseg_c, npts, "coarse region", &nvc)) return r;
  if (int r = check_segments(seg_f, nseg_f, npts, "fine region", &nvf)) return r;
  if (nvc + 7 * nvf > ((int64_t)1 << 31) - 1) return fail(WVL_EINVAL, "regions too large");
  if (int r = check_gpu(p)) return r;
  std::vector<int32_t> host((size_t)(2 * npts + nvc + nvf), -1);
  int32_t* map_c = host.data();
  int32_t* map_f = map_c + npts;
  int32_t* list_c = map_f + npts;
  int32_t* list_f = list_c + nvc;
  int64_t k = 0;
  for (int32_t s = 0; s < nseg_c; ++s)
    for (int32_t q = seg_c[2 * s]; q < seg_c[2 * s + 1]; ++q) { map_c[q] = (int32_t)k; list_c[k++] = q; }
  k = 0;
  for (int32_t s = 0; s < nseg_f; ++s)
    for (int32_t q = seg_f[2 * s]; q < seg_f[2 * s + 1]; ++q) { map_f[q] = (int32_t)k; list_f[k++] = q; }
  if (p->d_map_c) { WVL_HIP(hipFree(p->d_map_c)); p->d_map_c = nullptr; }
  void* d = nullptr;
  hipError_t e = dev_malloc(&d, sizeof(int32_t) * host.size());
  if (e != hipSuccess) return fail(WVL_ENOMEM, "region maps: %s", hipGetErrorString(e));
  e = hipMemcpy(d, host.data(), sizeof(int32_t) * host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(d); return hipfail(e, "region upload"); }
  p->d_map_c = (int32_t*)d;
  p->d_map_f = p->d_map_c + npts;
  p->d_list_c = p->d_map_f + npts;
  p->d_list_f = p->d_list_c + nvc;
  p->nvc = nvc;
  p->nvf = nvf;
  return WVL_OK;
}

int wvl_plan_compressed_size(const wvl_plan* p, int64_t* nvctr_c, int64_t* nvctr_f) {
  if (int r = check_plan(p)) return r;
  if (!nvctr_c || !nvctr_f) return fail(WVL_EINVAL, "NULL output");
  if (p->nvc < 0) return fail(WVL_EUNSUPPORTED, "no regions set (wvl_plan_set_regions)");
  *nvctr_c = p->nvc;
  *nvctr_f = p->nvf;
  return WVL_OK;
}

static int check_compressed(const wvl_plan* p, const char* what) {
  if (p->nvc < 0) return fail(WVL_EUNSUPPORTED, "%s: no regions set (wvl_plan_set_regions)", what);
  return WVL_OK;
}

// bytes of one compressed batch array (both planes for WVL_F32C)
static size_t cbatch_bytes(const wvl_plan* p) {
  return (size_t)((p->nvc + 7 * p->nvf) * p->norb) * (p->prec == WVL_F32 ? 4 : 8);
}

int wvl_decompress(wvl_plan* p, const void* psi_c, void* c, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!psi_c || !c) return fail(WVL_EINVAL, "wvl_decompress: NULL pointer");
  if (int r = check_aligned("wvl_decompress", {c})) return r;
  if (int r = check_compressed(p, "wvl_decompress")) return r;
  if (overlap(psi_c, cbatch_bytes(p), c, batch_bytes(p)))
    return fail(WVL_EINVAL, "wvl_decompress: output overlaps input");
  if (int r = check_gpu(p)) return r;
  const int64_t L = p->nvc + 7 * p->nvf;
  WVL_CHK(launch_decompress(p->prec, p->d_orbs, p->norb, p->M, p->d_map_c, p->d_map_f, p->nvc, L,
                            psi_c, L * p->norb, c, p->elems, (hipStream_t)stream));
  return WVL_OK;
}

int wvl_compress(wvl_plan* p, const void* c, void* psi_c, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!psi_c || !c) return fail(WVL_EINVAL, "wvl_compress: NULL pointer");
  if (int r = check_aligned("wvl_compress", {c})) return r;
  if (int r = check_compressed(p, "wvl_compress")) return r;
  if (overlap(psi_c, cbatch_bytes(p), c, batch_bytes(p)))
    return fail(WVL_EINVAL, "wvl_compress: output overlaps input");
  if (int r = check_gpu(p)) return r;
  const int64_t L = p->nvc + 7 * p->nvf;
  WVL_CHK(launch_compress(p->prec, p->d_orbs, p->norb, p->d_list_c, p->d_list_f, p->nvc, L, c,
                          p->elems, psi_c, L * p->norb, (hipStream_t)stream));
  return WVL_OK;
}

int wvl_local_hpsi_compressed(wvl_plan* p, const void* psi_c, const double* V, double pot_scale,
                              double kin_scale, void* hpsi_c, double* rho, double* e_loc,
                              double* e_kin, double* e_orb, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!psi_c || !V || !hpsi_c || !ws) return fail(WVL_EINVAL, "wvl_local_hpsi_compressed: NULL pointer");
  if (int r = check_compressed(p, "wvl_local_hpsi_compressed")) return r;
  if (rho && !p->shared) return fail(WVL_EUNSUPPORTED, "rho needs a WVL_SHARED_V plan");
  if (!isfinite(pot_scale) || !isfinite(kin_scale))
    return fail(WVL_EINVAL, "wvl_local_hpsi_compressed: scales must be finite");
  if (hpsi_c != psi_c && overlap(psi_c, cbatch_bytes(p), hpsi_c, cbatch_bytes(p)))
    return fail(WVL_EINVAL, "wvl_local_hpsi_compressed: hpsi_c overlaps psi_c without being it");
  if (int r = check_gpu(p)) return r;
  hipStream_t st = (hipStream_t)stream;
  const int64_t L = p->nvc + 7 * p->nvf;
  void* full = wsp(ws, p->o_D);
  // step 1: unpack onto the whole grid; steps 2-6 in place; step 7: pack
  WVL_CHK(launch_decompress(p->prec, p->d_orbs, p->norb, p->M, p->d_map_c, p->d_map_f, p->nvc, L,
                            psi_c, L * p->norb, full, p->elems, st));
  if (int r = hpsi_sequence(p, st, full, V, pot_scale, kin_scale, full, rho, e_loc, e_kin, e_orb, ws))
    return r;
  WVL_CHK(launch_compress(p->prec, p->d_orbs, p->norb, p->d_list_c, p->d_list_f, p->nvc, L, full,
                          p->elems, hpsi_c, L * p->norb, st));
  return WVL_OK;
}

int wvl_plan_query(const wvl_plan* p, int32_t what, int64_t* value) {
  if (int r = check_plan(p)) return r;
  if (!value) return fail(WVL_EINVAL, "value is NULL");
  switch (what) {
    case WVL_Q_VARIANT: *value = p->variant; break;
    case WVL_Q_GROUP: *value = p->use_xy && p->shared ? p->xy_G : 0; break;
    case WVL_Q_PERSISTENT: *value = p->persistent ? 1 : 0; break;
    case WVL_Q_XDIV: *value = p->xdiv; break;
    case WVL_Q_PGRID: *value = p->pgrid_mul; break;
    case WVL_Q_TUNE_BEST: *value = p->tune_best; break;
    case WVL_Q_FUSED_Z: *value = p->use_xy && p->zfuse ? 1 : 0; break;
    case WVL_Q_PRECOND_FORM: *value = precond_form(p, 0); break;
    default: return fail(WVL_EINVAL, "unknown query %d", what);
  }
  return WVL_OK;
}

int wvl_overlap(wvl_plan* p, const void* c, double* S, void* ws, void* stream) {
  if (int r = check_plan(p)) return r;
  if (!c || !S || !ws) return fail(WVL_EINVAL, "wvl_overlap: NULL pointer");
  if (int r = check_aligned("wvl_overlap", {c})) return r;
  if (!p->dense) return fail(WVL_EUNSUPPORTED, "wvl_overlap needs a dense uniform batch");
  if (int r = check_gpu(p)) return r;
  hipStream_t st = (hipStream_t)stream;
  Mark mk(p, st, ST_OVERLAP);
  hipError_t e = launch_overlap_p(p->prec, c, p->elems, p->norb, p->M, S,
                                  (double*)wsp(ws, p->o_syrk), st);
  if (e != hipSuccess) return hipfail(e, "overlap");
  return WVL_OK;
}

}  // extern "C"

// Overlap, Cholesky and X <- L^{-1} X with the scratch arrays given (SYRK
// slice partials, L, L^{-1}).
static int orthonormalize_into(wvl_plan* p, void* c, double* S, double* L, double* syrk, double* Lw,
                               double* Li, hipStream_t st) {
  const size_t nn = sizeof(double) * (size_t)p->norb * p->norb;
  hipError_t e;
  {
    Mark mk(p, st, ST_OVERLAP);
    e = launch_overlap_p(p->prec, c, p->elems, p->norb, p->M, Lw, syrk, st);
  }
  if (e != hipSuccess) return hipfail(e, "overlap");
  if (S) WVL_HIP(hipMemcpyAsync(S, Lw, nn, hipMemcpyDeviceToDevice, st));
  {
    Mark mk(p, st, ST_CHOL);
    e = launch_cholesky_inv(Lw, Li, p->norb, p->d_info, st);
  }
  if (e != hipSuccess) return hipfail(e, "cholesky");
  if (L) {
    e = launch_chol_factor(Lw, Li, p->norb, L, st);
    if (e != hipSuccess) return hipfail(e, "cholesky factor");
  }
  {
    Mark mk(p, st, ST_TRMM);
    e = launch_trmm_rows_p(p->prec, Li, c, c, p->elems, p->norb, p->M, st);
  }
  if (e != hipSuccess) return hipfail(e, "trmm");
  return WVL_OK;
}

static int check_orthonormalize(const wvl_plan* p, const void* c, const char* what) {
  if (int r = check_plan(p)) return r;
  if (!c) return fail(WVL_EINVAL, "%s: NULL pointer", what);
  if (int r = check_aligned(what, {c})) return r;
  if (!p->dense) return fail(WVL_EUNSUPPORTED, "%s needs a dense uniform batch", what);
  if (p->norb > 256) return fail(WVL_EUNSUPPORTED, "%s supports up to 256 orbitals", what);
  return WVL_OK;
}

// ---------------------------------------------------------------------------
// Entry point for callers that cannot allocate (graph capture, serving loops):
// its scratch memory is a static device array of the library, one per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel or a copy: that name is a host-side stand-in, so every use goes
// through the device address that hipGetSymbolAddress returns, looked up once
// per device when a context is created there.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)80 << 20;   // 80 MiB per GPU
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `device` (the current device); once per device
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(WVL_EUNSUPPORTED, "device %d", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return WVL_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hipfail(e, "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[device] = ptr;
  return WVL_OK;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

extern "C" {

int wvl_orthonormalize(wvl_plan* p, void* c, double* S, double* L, void* ws, void* stream) {
  if (int r = check_orthonormalize(p, c, "wvl_orthonormalize")) return r;
  if (!ws) return fail(WVL_EINVAL, "wvl_orthonormalize: NULL workspace");
  if (int r = check_gpu(p)) return r;
  return orthonormalize_into(p, c, S, L, (double*)wsp(ws, p->o_syrk), (double*)wsp(ws, p->o_L),
                             (double*)wsp(ws, p->o_Li),
                             (hipStream_t)stream);
}

int wvl_orthonormalize_noalloc(wvl_plan* p, void* c, double* S, double* L, void* stream) {
  if (int r = check_orthonormalize(p, c, "wvl_orthonormalize_noalloc")) return r;
  // scratch layout: SYRK slice partials, then L and L^{-1} (n x n each),
  // every part 256-byte aligned
  const size_t nn = align256(sizeof(double) * (size_t)p->norb * p->norb);
  const size_t syrk = align256(sizeof(double) * (size_t)syrk_partials(p->norb, p->M));
  const size_t need = syrk + 2 * nn;
  if (need > kScratchBytes)
    return fail(WVL_EUNSUPPORTED,
                "wvl_orthonormalize_noalloc: needs %zu bytes of scratch, the library holds %zu",
                need, kScratchBytes);
  if (int r = check_gpu(p)) return r;
  char* base = (char*)scratch_ptr(p->ctx->device);
  if (!base) return fail(WVL_EHIP, "wvl_orthonormalize_noalloc: scratch not set up on device %d",
                         p->ctx->device);
  return orthonormalize_into(p, c, S, L, (double*)base, (double*)(base + syrk),
                             (double*)(base + syrk + nn),
                             (hipStream_t)stream);
}

int wvl_convert(wvl_ctx* ctx, const void* src, int32_t sp, void* dst, int32_t dp, int64_t n,
                void* stream) {
  if (!ctx) return fail(WVL_EINVAL, "ctx is NULL");
  if (!src || !dst) return fail(WVL_EINVAL, "wvl_convert: NULL pointer");
  if (sp < 0 || sp > 2 || dp < 0 || dp > 2) return fail(WVL_EINVAL, "wvl_convert: bad precision");
  if (n < 0) return fail(WVL_EINVAL, "wvl_convert: negative count");
  if (src == dst) return fail(WVL_EINVAL, "wvl_convert: src and dst overlap");
  if (ctx->dry) return fail(WVL_ENODEV, "dry context: no GPU");
  WVL_HIP(hipSetDevice(ctx->device));
  hipError_t e = launch_convert(src, sp, dst, dp, n, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(e, "convert");
  return WVL_OK;
}

int wvl_plan_sync(wvl_plan* p, void* stream) {
  if (int r = check_plan(p)) return r;
  if (int r = check_gpu(p)) return r;
  WVL_HIP(hipStreamSynchronize((hipStream_t)stream));
  int info[4];
  WVL_HIP(hipMemcpy(info, p->d_info, sizeof info, hipMemcpyDeviceToHost));
  if (info[0] != 0) {
    int zero[4] = {0, 0, 0, 0};
    (void)hipMemcpy(p->d_info, zero, sizeof zero, hipMemcpyHostToDevice);
    return fail(WVL_EINVAL, "overlap matrix not positive definite (pivot %d)", info[0] - 1);
  }
  return WVL_OK;
}

int wvl_plan_profile(wvl_plan* p, int32_t capacity) {
  if (int r = check_plan(p)) return r;
  if (capacity < 0 || capacity > (1 << 20)) return fail(WVL_EINVAL, "profile capacity out of range");
  p->prof_cap = capacity;
  p->prof_used = 0;
  return WVL_OK;
}

int wvl_plan_profile_read(wvl_plan* p, int32_t* stage, double* ms, int32_t max, int32_t* count) {
  if (int r = check_plan(p)) return r;
  if (!count || max < 0 || (max > 0 && (!stage || !ms)))
    return fail(WVL_EINVAL, "wvl_plan_profile_read: bad arguments");
  if (int r = check_gpu(p)) return r;
  const int n = std::min(max, p->prof_used);
  for (int i = 0; i < n; ++i) {
    WVL_HIP(hipEventSynchronize(p->prof[i].b));
    float t = 0.f;
    WVL_HIP(hipEventElapsedTime(&t, p->prof[i].a, p->prof[i].b));
    stage[i] = p->prof[i].stage;
    ms[i] = t;
  }
  *count = n;
  p->prof_used = 0;
  return WVL_OK;
}

const char* wvl_stage_name(int32_t stage) {
  if (stage < 0 || stage >= ST_NSTAGE) return "unknown";
  return kStageNames[stage];
}

}  // extern "C"
