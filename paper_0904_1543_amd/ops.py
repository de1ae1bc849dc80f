"""torch-facing wrapper of libwvl: device memory, streams and plans.

PyTorch only provides device memory (tensors) and the current HIP stream;
every arithmetic step runs in libwvl's kernels through :mod:`lib`.

Batch tensors are packed buffers (orbital b at element offset off_b):
  f64  -> torch.float64, shape (elems,)
  f32  -> torch.float32, shape (elems,)
  f32c -> torch.float32, shape (2, elems): hi plane, lo plane (value = hi + lo)
"""

import ctypes

import numpy as np
import torch

from . import lib

PRECS = {"f64": lib.WVL_F64, "f32": lib.WVL_F32, "f32c": lib.WVL_F32C}

_CTX = {}


def context(device=0):
    if device not in _CTX:
        h = ctypes.c_void_p()
        lib.wvl_create(ctypes.byref(h), device)
        _CTX[device] = h
    return _CTX[device]


def stream_handle(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def fine_shape(dims):
    n1, n2, n3 = dims
    return (2 * n3, 2 * n2, 2 * n1)


class Plan:
    """A batch of orbitals with given coarse dims (n1, n2, n3) per orbital."""

    def __init__(self, dims, prec="f64", shared_v=True, hgrid=(1.0, 1.0, 1.0), occ=2.0,
                 graph=False, persistent=False, autotune=False, device=0, dry=False,
                 bc="periodic"):
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.norb = len(self.dims)
        self.prec = prec
        self.pid = PRECS[prec]
        self.device = device
        self.dry = dry
        self.shared_v = shared_v
        self.M = [int(np.prod(fine_shape(d))) for d in self.dims]
        offs = np.concatenate([[0], np.cumsum(self.M)[:-1]]).astype(np.int64)
        self.offsets = offs
        self.v_offsets = offs.copy() if not shared_v else np.zeros_like(offs)
        occs = np.broadcast_to(np.asarray(occ, dtype=np.float64), (self.norb,))
        hg = np.broadcast_to(np.asarray(hgrid, dtype=np.float64), (self.norb, 3)) \
            if np.ndim(hgrid) != 1 else np.tile(np.asarray(hgrid, dtype=np.float64), (self.norb, 1))
        arr = (lib.wvl_orbital * self.norb)()
        for b, d in enumerate(self.dims):
            arr[b].n[0], arr[b].n[1], arr[b].n[2] = d
            arr[b].reserved = 0
            arr[b].off = int(offs[b])
            arr[b].v_off = int(self.v_offsets[b])
            arr[b].hgrid[0], arr[b].hgrid[1], arr[b].hgrid[2] = (float(x) for x in hg[b])
            arr[b].occ = float(occs[b])
        self.occ = np.array(occs, dtype=np.float64)
        flags = (lib.WVL_SHARED_V if shared_v else 0) | (lib.WVL_USE_GRAPH if graph else 0) | \
            (lib.WVL_PERSISTENT if persistent else 0) | (lib.WVL_AUTOTUNE if autotune else 0) | \
            {"periodic": 0, "free": lib.WVL_FREE_BC, "surface": lib.WVL_SURFACE_BC}[bc]
        self.bc = bc
        self._arr = arr
        ctx = ctypes.c_void_p()
        if dry:
            lib.wvl_create(ctypes.byref(ctx), -1)
            self._own_ctx = ctx
        else:
            ctx = context(device)
            self._own_ctx = None
        self.ctx = ctx
        h = ctypes.c_void_p()
        lib.wvl_plan_create(ctx, arr, self.norb, self.pid, flags, ctypes.byref(h))
        self.h = h
        wsb = ctypes.c_size_t()
        lib.wvl_plan_workspace(h, ctypes.byref(wsb))
        el = ctypes.c_int64()
        lib.wvl_plan_elements(h, ctypes.byref(el))
        self.ws_bytes = wsb.value
        self.elems = el.value
        # points of V and rho (the real-space grid of a shared potential)
        self.grid_points = self.M[0]
        if shared_v:
            gp = ctypes.c_int64()
            lib.wvl_plan_grid_points(h, ctypes.byref(gp))
            self.grid_points = gp.value
        self.ws = None
        if not dry:
            self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8,
                                  device=f"cuda:{device}")

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and self.h.value:
                lib.raw("wvl_plan_destroy")(self.h)
                self.h = None
            if getattr(self, "_own_ctx", None) is not None:
                lib.raw("wvl_destroy")(self._own_ctx)
        except Exception:
            pass

    # ------------------------------------------------------------------ buffers
    @property
    def dev(self):
        return f"cuda:{self.device}"

    def empty(self):
        if self.prec == "f64":
            return torch.empty(self.elems, dtype=torch.float64, device=self.dev)
        if self.prec == "f32":
            return torch.empty(self.elems, dtype=torch.float32, device=self.dev)
        return torch.empty((2, self.elems), dtype=torch.float32, device=self.dev)

    def convert(self, src, src_prec, dst_prec, count):
        dst = {"f64": lambda: torch.empty(count, dtype=torch.float64, device=self.dev),
               "f32": lambda: torch.empty(count, dtype=torch.float32, device=self.dev),
               "f32c": lambda: torch.empty((2, count), dtype=torch.float32, device=self.dev)}[dst_prec]()
        lib.wvl_convert(self.ctx, ptr(src), PRECS[src_prec], ptr(dst), PRECS[dst_prec], count,
                        stream_handle())
        return dst

    def pack(self, arrays):
        """float64 host arrays (one per orbital, or a (B, m3, m2, m1) array) ->
        packed device tensor in the plan precision (conversion on the GPU)."""
        flat = np.empty(self.elems, dtype=np.float64)
        for b in range(self.norb):
            flat[self.offsets[b]:self.offsets[b] + self.M[b]] = np.asarray(arrays[b]).ravel()
        t64 = torch.from_numpy(flat).to(self.dev)
        if self.prec == "f64":
            return t64
        return self.convert(t64, "f64", self.prec, self.elems)

    def to_f64(self, t):
        if self.prec == "f64":
            return t
        return self.convert(t, self.prec, "f64", self.elems)

    def unpack(self, t):
        flat = self.to_f64(t).cpu().numpy()
        return [flat[self.offsets[b]:self.offsets[b] + self.M[b]].reshape(fine_shape(self.dims[b]))
                for b in range(self.norb)]

    def pack_potential(self, V):
        if self.shared_v:
            return torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64).ravel()).to(self.dev)
        flat = np.empty(self.elems, dtype=np.float64)
        for b in range(self.norb):
            flat[self.v_offsets[b]:self.v_offsets[b] + self.M[b]] = np.asarray(V[b]).ravel()
        return torch.from_numpy(flat).to(self.dev)

    # ------------------------------------------------------------------ ops
    def synthesis(self, c, out=None):
        out = self.empty() if out is None else out
        lib.wvl_synthesis(self.h, ptr(c), ptr(out), ptr(self.ws), stream_handle())
        return out

    def analysis(self, s, out=None):
        out = self.empty() if out is None else out
        lib.wvl_analysis(self.h, ptr(s), ptr(out), ptr(self.ws), stream_handle())
        return out

    def magic_filter(self, x, transpose=False, out=None):
        out = self.empty() if out is None else out
        lib.wvl_magic_filter(self.h, ptr(x), ptr(out), int(bool(transpose)), ptr(self.ws),
                             stream_handle())
        return out

    def kinetic(self, s, k0=None, out=None):
        out = self.empty() if out is None else out
        lib.wvl_kinetic(self.h, ptr(s), ptr(k0), ptr(out), ptr(self.ws), stream_handle())
        return out

    def local_density(self, c, rho=None, accumulate=False):
        npts = self.grid_points
        if rho is None:
            rho = torch.empty(npts, dtype=torch.float64, device=self.dev)
        lib.wvl_local_density(self.h, ptr(c), ptr(rho), int(bool(accumulate)), ptr(self.ws),
                              stream_handle())
        return rho

    def local_hpsi(self, c, V, pot_scale=1.0, kin_scale=1.0, out=None, rho=True, energies=True,
                   per_orbital=False):
        out = self.empty() if out is None else out
        r = torch.empty(self.grid_points, dtype=torch.float64, device=self.dev) \
            if (rho and self.shared_v) else None
        e = torch.empty(2, dtype=torch.float64, device=self.dev) if energies else None
        eo = torch.empty(2 * self.norb, dtype=torch.float64, device=self.dev) if per_orbital else None
        e_loc = ctypes.c_void_p(e.data_ptr()) if e is not None else None
        e_kin = ctypes.c_void_p(e.data_ptr() + 8) if e is not None else None
        lib.wvl_local_hpsi(self.h, ptr(c), ptr(V), float(pot_scale), float(kin_scale), ptr(out),
                           ptr(r), e_loc, e_kin, ptr(eo), ptr(self.ws), stream_handle())
        return dict(hpsi=out, rho=r, energies=e, e_orb=eo)

    def energy_gradient(self, c, V, g_loc=1.0, g_kin=1.0, out=None):
        """2 f_b (g_loc Hloc + g_kin Kin) c_b for every orbital (on the device)."""
        out = self.empty() if out is None else out
        lib.wvl_energy_gradient(self.h, ptr(c), ptr(V), float(g_loc), float(g_kin), ptr(out),
                                ptr(self.ws), stream_handle())
        return out

    def precondition(self, g, eps, iters, separate=False, out=None, residuals=False, form=None):
        """Preconditioned gradients: `iters` PCG steps on (-1/2 nabla^2 - eps_b) x = g_b
        for every orbital (eps: one negative value per orbital, host side).
        form: None (default: fused plane kernel when it fits), "passes"
        (combined filter, one pass per axis) or "separate"."""
        if form == "separate":
            separate = True
        out = self.empty() if out is None else out
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (self.norb,)))
        res = torch.empty(self.norb, dtype=torch.float64, device=self.dev) if residuals else None
        lib.wvl_precondition(self.h, ptr(g), e.ctypes.data_as(lib.DP), int(iters),
                             lib.WVL_PRECOND_SEPARATE if separate else
                             (lib.WVL_PRECOND_PASSES if form == "passes" else 0), ptr(out), ptr(res),
                             ptr(self.ws), stream_handle())
        return (out, res) if residuals else out

    # ------------------------------------------------------------ compressed form
    def set_regions(self, seg_c, seg_f):
        """Coarse and fine regions as (k, 2) int32 segment arrays [start, end)."""
        sc = np.ascontiguousarray(np.asarray(seg_c, dtype=np.int32).reshape(-1, 2))
        sf = np.ascontiguousarray(np.asarray(seg_f, dtype=np.int32).reshape(-1, 2))
        I32P = ctypes.POINTER(ctypes.c_int32)
        lib.wvl_plan_set_regions(self.h, sc.ctypes.data_as(I32P), len(sc),
                                 sf.ctypes.data_as(I32P), len(sf))
        a, b = ctypes.c_int64(), ctypes.c_int64()
        lib.wvl_plan_compressed_size(self.h, ctypes.byref(a), ctypes.byref(b))
        self.nvctr = (a.value, b.value)
        self.clen = a.value + 7 * b.value
        return self.nvctr

    def empty_compressed(self):
        n = self.clen * self.norb
        if self.prec == "f64":
            return torch.empty(n, dtype=torch.float64, device=self.dev)
        if self.prec == "f32":
            return torch.empty(n, dtype=torch.float32, device=self.dev)
        return torch.empty((2, n), dtype=torch.float32, device=self.dev)

    def pack_compressed(self, vectors):
        """float64 host vectors (one per orbital) -> compressed batch tensor."""
        t64 = torch.from_numpy(np.concatenate([np.asarray(v, dtype=np.float64).ravel()
                                               for v in vectors])).to(self.dev)
        if self.prec == "f64":
            return t64
        return self.convert(t64, "f64", self.prec, self.clen * self.norb)

    def unpack_compressed(self, t):
        flat = (t if self.prec == "f64" else
                self.convert(t, self.prec, "f64", self.clen * self.norb)).cpu().numpy()
        return [flat[b * self.clen:(b + 1) * self.clen] for b in range(self.norb)]

    def decompress(self, psi_c, out=None):
        out = self.empty() if out is None else out
        lib.wvl_decompress(self.h, ptr(psi_c), ptr(out), stream_handle())
        return out

    def compress(self, c, out=None):
        out = self.empty_compressed() if out is None else out
        lib.wvl_compress(self.h, ptr(c), ptr(out), stream_handle())
        return out

    def local_hpsi_compressed(self, psi_c, V, pot_scale=1.0, kin_scale=1.0, out=None, rho=True,
                              energies=True, per_orbital=False):
        out = self.empty_compressed() if out is None else out
        r = torch.empty(self.grid_points, dtype=torch.float64, device=self.dev) \
            if (rho and self.shared_v) else None
        e = torch.empty(2, dtype=torch.float64, device=self.dev) if energies else None
        eo = torch.empty(2 * self.norb, dtype=torch.float64, device=self.dev) if per_orbital else None
        e_loc = ctypes.c_void_p(e.data_ptr()) if e is not None else None
        e_kin = ctypes.c_void_p(e.data_ptr() + 8) if e is not None else None
        lib.wvl_local_hpsi_compressed(self.h, ptr(psi_c), ptr(V), float(pot_scale), float(kin_scale),
                                      ptr(out), ptr(r), e_loc, e_kin, ptr(eo), ptr(self.ws),
                                      stream_handle())
        return dict(hpsi=out, rho=r, energies=e, e_orb=eo)

    def query(self, what):
        """A plan property (lib.WVL_Q_*)."""
        v = ctypes.c_int64()
        lib.wvl_plan_query(self.h, int(what), ctypes.byref(v))
        return v.value

    def overlap(self, c):
        S = torch.empty((self.norb, self.norb), dtype=torch.float64, device=self.dev)
        lib.wvl_overlap(self.h, ptr(c), ptr(S), ptr(self.ws), stream_handle())
        return S

    def orthonormalize(self, c):
        S = torch.empty((self.norb, self.norb), dtype=torch.float64, device=self.dev)
        L = torch.empty((self.norb, self.norb), dtype=torch.float64, device=self.dev)
        lib.wvl_orthonormalize(self.h, ptr(c), ptr(S), ptr(L), ptr(self.ws), stream_handle())
        return S, L

    def sync(self):
        lib.wvl_plan_sync(self.h, stream_handle())

    def profile(self, capacity):
        lib.wvl_plan_profile(self.h, int(capacity))

    def profile_read(self, maxrec=1 << 16):
        st = (ctypes.c_int32 * maxrec)()
        ms = (ctypes.c_double * maxrec)()
        n = ctypes.c_int32()
        lib.wvl_plan_profile_read(self.h, st, ms, maxrec, ctypes.byref(n))
        return [(lib.wvl_stage_name(st[i]), ms[i]) for i in range(n.value)]
