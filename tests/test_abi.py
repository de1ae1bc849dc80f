"""C-ABI contract on the host (no GPU needed): the library loads, exports every
symbol that include/wvl.h declares, and checks its arguments before touching
the GPU (dry contexts answer WVL_ENODEV only after the checks passed)."""

import ctypes
import os
import re

import pytest

from paper_0904_1543_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "wvl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wvl_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib._lib, n), n
    assert set(names) == set(lib.EXPORTS)


def test_version_and_error_text():
    assert "gfx950" in lib.wvl_version()
    rc = lib.raw("wvl_create")(None, 0)
    assert rc == lib.WVL_EINVAL
    assert "ctx" in lib.wvl_last_error()


def _orbs(dims, offs=None, hgrid=(1.0, 1.0, 1.0), occ=2.0):
    arr = (lib.wvl_orbital * len(dims))()
    off = 0
    for b, d in enumerate(dims):
        arr[b].n[0], arr[b].n[1], arr[b].n[2] = d
        arr[b].off = off if offs is None else offs[b]
        arr[b].v_off = 0
        arr[b].hgrid[0], arr[b].hgrid[1], arr[b].hgrid[2] = hgrid
        arr[b].occ = occ
        off += 8 * d[0] * d[1] * d[2]
    return arr


@pytest.fixture()
def dry():
    ctx = ctypes.c_void_p()
    assert lib.raw("wvl_create")(ctypes.byref(ctx), -1) == lib.WVL_OK
    yield ctx
    lib.raw("wvl_destroy")(ctx)


def _plan(ctx, dims, prec=0, flags=1, **kw):
    h = ctypes.c_void_p()
    rc = lib.raw("wvl_plan_create")(ctx, _orbs(dims, **kw), len(dims), prec, flags, ctypes.byref(h))
    return rc, h


def test_no_gpu_gives_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert lib.raw("wvl_create")(ctypes.byref(ctx), 0) == lib.WVL_ENODEV
    assert "GPU" in lib.wvl_last_error()


def test_plan_argument_checks(dry):
    assert _plan(dry, [(4, 4, 4)], prec=7)[0] == lib.WVL_EINVAL
    assert _plan(dry, [(1, 4, 4)])[0] == lib.WVL_EINVAL                     # n < 2
    assert _plan(dry, [(4, 4, 4)], flags=64)[0] == lib.WVL_EINVAL           # unknown flag
    assert _plan(dry, [(4, 4, 4)], hgrid=(1.0, -1.0, 1.0))[0] == lib.WVL_EINVAL
    assert _plan(dry, [(4, 4, 4), (4, 4, 4)], offs=[0, 100])[0] == lib.WVL_EINVAL  # overlap
    assert _plan(dry, [(4, 4, 4), (4, 6, 4)], flags=1)[0] == lib.WVL_EINVAL  # shared V, uneven
    h = ctypes.c_void_p()
    assert lib.raw("wvl_plan_create")(dry, _orbs([(4, 4, 4)]), 0, 0, 1, ctypes.byref(h)) == lib.WVL_EINVAL
    assert lib.raw("wvl_plan_create")(None, _orbs([(4, 4, 4)]), 1, 0, 1, ctypes.byref(h)) == lib.WVL_EINVAL
    rc, p = _plan(dry, [(4, 4, 4), (4, 6, 4)], flags=0)
    assert rc == lib.WVL_OK
    lib.wvl_plan_destroy(p)


def test_plan_sizes(dry):
    rc, p = _plan(dry, [(16, 16, 16)] * 3, prec=2)
    assert rc == lib.WVL_OK
    el = ctypes.c_int64()
    lib.wvl_plan_elements(p, ctypes.byref(el))
    assert el.value == 3 * 32 ** 3
    ws = ctypes.c_size_t()
    lib.wvl_plan_workspace(p, ctypes.byref(ws))
    assert ws.value >= 3 * 8 * el.value      # three work arrays of hi+lo planes
    pts = ctypes.c_int64()
    lib.wvl_plan_grid_points(p, ctypes.byref(pts))
    assert pts.value == 32 ** 3
    lib.wvl_plan_destroy(p)


def test_calls_check_arguments_before_gpu(dry):
    rc, p = _plan(dry, [(4, 4, 4)] * 2)
    assert rc == lib.WVL_OK
    a, b, ws = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    f = lib.raw
    # NULL pointers and aliasing -> EINVAL
    assert f("wvl_synthesis")(p, None, b, ws, None) == lib.WVL_EINVAL
    assert f("wvl_synthesis")(p, a, a, ws, None) == lib.WVL_EINVAL
    assert f("wvl_analysis")(p, a, b, None, None) == lib.WVL_EINVAL
    assert f("wvl_magic_filter")(p, a, a, 0, ws, None) == lib.WVL_EINVAL
    assert f("wvl_kinetic")(p, a, None, a, ws, None) == lib.WVL_EINVAL
    assert f("wvl_kinetic")(p, a, a, b, ws, None) == lib.WVL_EINVAL
    assert f("wvl_local_hpsi")(p, a, None, 1.0, 1.0, b, None, None, None, None, ws, None) == lib.WVL_EINVAL
    assert f("wvl_local_hpsi")(p, a, a, float("nan"), 1.0, b, None, None, None, None, ws, None) == lib.WVL_EINVAL
    assert f("wvl_synthesis")(None, a, b, ws, None) == lib.WVL_EINVAL
    # valid arguments on a dry plan -> ENODEV
    assert f("wvl_synthesis")(p, a, b, ws, None) == lib.WVL_ENODEV
    assert f("wvl_kinetic")(p, a, None, b, ws, None) == lib.WVL_ENODEV
    assert f("wvl_local_density")(p, a, b, 0, ws, None) == lib.WVL_ENODEV
    assert f("wvl_local_hpsi")(p, a, b, 1.0, 1.0, ws, None, None, None, None, ws, None) == lib.WVL_ENODEV
    assert f("wvl_overlap")(p, a, b, ws, None) == lib.WVL_ENODEV
    assert f("wvl_convert")(dry, a, 0, b, 2, 10, None) == lib.WVL_ENODEV
    assert f("wvl_convert")(dry, a, 0, a, 2, 10, None) == lib.WVL_EINVAL
    assert f("wvl_convert")(dry, a, 0, b, 5, 10, None) == lib.WVL_EINVAL
    lib.wvl_plan_destroy(p)


def test_unsupported_combinations(dry):
    rc, p = _plan(dry, [(4, 4, 4), (4, 6, 4)], flags=0)    # uneven, per-orbital V
    a, b, ws = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    assert lib.raw("wvl_local_density")(p, a, b, 0, ws, None) == lib.WVL_EUNSUPPORTED
    assert lib.raw("wvl_overlap")(p, a, b, ws, None) == lib.WVL_EUNSUPPORTED
    assert lib.raw("wvl_local_hpsi")(p, a, a, 1.0, 1.0, b, b, None, None, None, ws, None) == \
        lib.WVL_EUNSUPPORTED   # rho needs a shared potential
    lib.wvl_plan_destroy(p)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_partial_overlap_is_rejected(dry, prec):
    """Batch arrays of 2 x 8^3 elements (8 KiB in float64 and compensated
    float32, 4 KiB in float32): an output that starts inside its input is
    rejected; hpsi (or the gradient) equal to c is allowed."""
    rc, p = _plan(dry, [(4, 4, 4)] * 2, prec=prec)
    assert rc == lib.WVL_OK
    f = lib.raw
    a, V, ws = 0x100000, ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    A = ctypes.c_void_p(a)
    inside = ctypes.c_void_p(a + 16)
    nbytes = 2 * 512 * (4 if prec == 1 else 8)
    after = ctypes.c_void_p(a + nbytes)      # first byte past the array: disjoint
    hpsi = f("wvl_local_hpsi")
    assert hpsi(p, A, V, 1.0, 1.0, inside, None, None, None, None, ws, None) == lib.WVL_EINVAL
    assert "overlaps" in lib.wvl_last_error()
    assert hpsi(p, A, V, 1.0, 1.0, A, None, None, None, None, ws, None) == lib.WVL_ENODEV
    assert hpsi(p, A, V, 1.0, 1.0, after, None, None, None, None, ws, None) == lib.WVL_ENODEV
    grad = f("wvl_energy_gradient")
    assert grad(p, A, V, 1.0, 1.0, inside, ws, None) == lib.WVL_EINVAL
    assert grad(p, A, V, 1.0, 1.0, A, ws, None) == lib.WVL_ENODEV
    assert f("wvl_synthesis")(p, A, inside, ws, None) == lib.WVL_EINVAL
    assert f("wvl_analysis")(p, inside, A, ws, None) == lib.WVL_EINVAL
    assert f("wvl_magic_filter")(p, A, inside, 1, ws, None) == lib.WVL_EINVAL
    out = ctypes.c_void_p(0x400000)
    k0_inside_out = ctypes.c_void_p(0x400000 + 16)
    assert f("wvl_kinetic")(p, A, k0_inside_out, out, ws, None) == lib.WVL_EINVAL
    assert f("wvl_kinetic")(p, A, out, out, ws, None) == lib.WVL_ENODEV
    assert f("wvl_kinetic")(p, A, inside, out, ws, None) == lib.WVL_EINVAL
    lib.wvl_plan_destroy(p)


def test_misaligned_batch_arrays_are_rejected(dry):
    """Batch arrays must start on a 16-byte boundary (every entry point that
    takes one checks it before any GPU work)."""
    rc, p = _plan(dry, [(4, 4, 4)] * 2)
    assert rc == lib.WVL_OK
    f = lib.raw
    A, V, ws = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    out = ctypes.c_void_p(0x400000)
    odd = ctypes.c_void_p(0x500008)
    S = ctypes.c_void_p(0x600000)
    eps = (ctypes.c_double * 2)(-0.5, -0.2)
    calls = {
        "wvl_synthesis": lambda x, y: f("wvl_synthesis")(p, x, y, ws, None),
        "wvl_analysis": lambda x, y: f("wvl_analysis")(p, x, y, ws, None),
        "wvl_magic_filter": lambda x, y: f("wvl_magic_filter")(p, x, y, 0, ws, None),
        "wvl_kinetic": lambda x, y: f("wvl_kinetic")(p, x, None, y, ws, None),
        "wvl_local_hpsi": lambda x, y: f("wvl_local_hpsi")(p, x, V, 1.0, 1.0, y, None, None,
                                                           None, None, ws, None),
        "wvl_energy_gradient": lambda x, y: f("wvl_energy_gradient")(p, x, V, 1.0, 1.0, y, ws,
                                                                     None),
        "wvl_precondition": lambda x, y: f("wvl_precondition")(p, x, eps, 2, 0, y, None, ws, None),
    }
    for name, call in calls.items():
        for x, y in ((odd, out), (A, odd)):
            assert call(x, y) == lib.WVL_EINVAL, name
            assert "16-byte aligned" in lib.wvl_last_error(), name
        assert call(A, out) == lib.WVL_ENODEV, name
    assert f("wvl_local_density")(p, odd, S, 0, ws, None) == lib.WVL_EINVAL
    assert f("wvl_overlap")(p, odd, S, ws, None) == lib.WVL_EINVAL
    assert f("wvl_orthonormalize")(p, odd, S, S, ws, None) == lib.WVL_EINVAL
    lib.wvl_plan_destroy(p)


def test_plan_queries(dry):
    rc, p = _plan(dry, [(8, 6, 32)] * 33)        # fine (16, 12, 64): G = 2
    assert rc == lib.WVL_OK
    v = ctypes.c_int64()
    q = lib.raw("wvl_plan_query")
    assert q(p, lib.WVL_Q_VARIANT, ctypes.byref(v)) == lib.WVL_OK and v.value == 2
    assert q(p, lib.WVL_Q_GROUP, ctypes.byref(v)) == lib.WVL_OK and v.value == 2
    assert q(p, lib.WVL_Q_PERSISTENT, ctypes.byref(v)) == lib.WVL_OK and v.value == 0
    assert q(p, lib.WVL_Q_XDIV, ctypes.byref(v)) == lib.WVL_OK and v.value == 1
    assert q(p, lib.WVL_Q_PGRID, ctypes.byref(v)) == lib.WVL_OK and v.value == 8
    assert q(p, lib.WVL_Q_TUNE_BEST, ctypes.byref(v)) == lib.WVL_OK and v.value == -1
    assert q(p, lib.WVL_Q_FUSED_Z, ctypes.byref(v)) == lib.WVL_OK and v.value == 1
    assert q(p, 99, ctypes.byref(v)) == lib.WVL_EINVAL
    assert q(p, lib.WVL_Q_GROUP, None) == lib.WVL_EINVAL
    lib.wvl_plan_destroy(p)
    rc, p = _plan(dry, [(8, 6, 32)] * 33, prec=2, flags=4)   # per-orbital V, persistent
    assert q(p, lib.WVL_Q_VARIANT, ctypes.byref(v)) == lib.WVL_OK and v.value == 1
    assert q(p, lib.WVL_Q_GROUP, ctypes.byref(v)) == lib.WVL_OK and v.value == 0
    assert q(p, lib.WVL_Q_PERSISTENT, ctypes.byref(v)) == lib.WVL_OK and v.value == 1
    assert q(p, lib.WVL_Q_FUSED_Z, ctypes.byref(v)) == lib.WVL_OK and v.value == 0
    lib.wvl_plan_destroy(p)


def test_noalloc_orthonormalize_checks(dry):
    """Arguments and sizes are checked before any GPU work."""
    f = lib.raw("wvl_orthonormalize_noalloc")
    a = ctypes.c_void_p(0x100000)
    rc, p = _plan(dry, [(4, 4, 4)] * 257)
    assert rc == lib.WVL_OK
    assert f(p, a, None, None, None) == lib.WVL_EUNSUPPORTED      # more than 256 orbitals
    lib.wvl_plan_destroy(p)
    rc, p = _plan(dry, [(4, 4, 4)] * 3)
    assert f(p, None, None, None, None) == lib.WVL_EINVAL
    assert f(None, a, None, None, None) == lib.WVL_EINVAL
    assert f(p, a, None, None, None) == lib.WVL_ENODEV             # valid, but no GPU
    lib.wvl_plan_destroy(p)


def test_precondition_checks(dry):
    rc, p = _plan(dry, [(4, 4, 4)] * 2)
    f = lib.raw("wvl_precondition")
    a, b, ws = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    good = (ctypes.c_double * 2)(-0.5, -0.2)
    bad = (ctypes.c_double * 2)(-0.5, 0.0)
    assert f(p, a, good, 3, 0, b, None, ws, None) == lib.WVL_ENODEV
    assert f(p, a, bad, 3, 0, b, None, ws, None) == lib.WVL_EINVAL       # eps must be < 0
    assert "eps[1]" in lib.wvl_last_error()
    assert f(p, a, good, -1, 0, b, None, ws, None) == lib.WVL_EINVAL     # iters
    assert f(p, a, good, 3, 4, b, None, ws, None) == lib.WVL_EINVAL      # unknown mode
    assert f(p, a, None, 3, 0, b, None, ws, None) == lib.WVL_EINVAL
    assert f(p, a, good, 3, 0, a, None, ws, None) == lib.WVL_EINVAL      # gt overlaps g
    lib.wvl_plan_destroy(p)


def test_region_checks(dry):
    rc, p = _plan(dry, [(4, 4, 4)] * 2)          # 64 coarse points
    f = lib.raw("wvl_plan_set_regions")
    I32 = ctypes.c_int32

    def segs(*pairs):
        flat = [v for pq in pairs for v in pq]
        return (I32 * max(1, len(flat)))(*flat), len(pairs)

    good, n = segs((0, 5), (8, 20))
    assert f(p, good, n, good, n) == lib.WVL_ENODEV                     # valid: no GPU
    for bad in (segs((5, 5)), segs((0, 65)), segs((8, 20), (0, 5)), segs((0, 10), (9, 12)),
                segs((-1, 3))):
        assert f(p, bad[0], bad[1], good, n) == lib.WVL_EINVAL
    assert f(p, None, 1, good, n) == lib.WVL_EINVAL
    a, b = ctypes.c_int64(), ctypes.c_int64()
    assert lib.raw("wvl_plan_compressed_size")(p, ctypes.byref(a), ctypes.byref(b)) == \
        lib.WVL_EUNSUPPORTED                                             # no regions yet
    x, y = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000)
    assert lib.raw("wvl_decompress")(p, x, y, None) == lib.WVL_EUNSUPPORTED
    lib.wvl_plan_destroy(p)
    rc, p = _plan(dry, [(4, 4, 4), (4, 6, 4)], flags=0)                 # uneven batch
    assert f(p, good, n, good, n) == lib.WVL_EUNSUPPORTED
    lib.wvl_plan_destroy(p)


def test_boundary_condition_plans(dry):
    a, b, ws = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    assert _plan(dry, [(4, 4, 4)] * 2, flags=1 | 16 | 32)[0] == lib.WVL_EINVAL     # both
    assert _plan(dry, [(4, 4, 4)] * 2, flags=16)[0] == lib.WVL_EUNSUPPORTED       # no shared V
    assert _plan(dry, [(4, 4, 4), (4, 6, 4)], flags=16)[0] == lib.WVL_EUNSUPPORTED
    for flag, shape in ((16, (37, 37, 37)), (32, (8, 37, 8))):
        rc, p = _plan(dry, [(4, 4, 4)] * 2, flags=1 | flag)
        assert rc == lib.WVL_OK
        pts = ctypes.c_int64()
        lib.wvl_plan_grid_points(p, ctypes.byref(pts))
        assert pts.value == shape[0] * shape[1] * shape[2]        # m + 29 on isolated axes
        assert lib.raw("wvl_synthesis")(p, a, b, ws, None) == lib.WVL_EUNSUPPORTED
        assert lib.raw("wvl_kinetic")(p, a, None, b, ws, None) == lib.WVL_EUNSUPPORTED
        assert lib.raw("wvl_local_hpsi")(p, a, b, 1.0, 1.0, ws, None, None, None, None, ws,
                                          None) == lib.WVL_ENODEV
        eps = (ctypes.c_double * 2)(-0.5, -0.2)
        assert lib.raw("wvl_precondition")(p, a, eps, 3, 1, b, None, ws, None) == \
            lib.WVL_EUNSUPPORTED                                   # separate form: periodic only
        lib.wvl_plan_destroy(p)


def test_exact_product_engine_selection(dry, monkeypatch):
    """Compensated plans take the exact digit-product engine (variant 3) when
    it applies: shared potential, fine lengths multiples of 16, planes of at
    most 36 tiles, isotropic spacing; otherwise the vector engine."""
    q = lib.raw("wvl_plan_query")
    v = ctypes.c_int64()

    def variant(dims, flags=1, **kw):
        rc, p = _plan(dry, dims, prec=2, flags=flags, **kw)
        assert rc == lib.WVL_OK
        assert q(p, lib.WVL_Q_VARIANT, ctypes.byref(v)) == lib.WVL_OK
        lib.wvl_plan_destroy(p)
        return v.value

    assert variant([(48, 48, 48)] * 4) == 3                  # fine 96^3: 36 tiles a plane
    assert variant([(8, 24, 16)] * 3) == 3                   # fine (32, 48, 16)
    assert variant([(20, 18, 17)] * 2) == 1                  # lengths not multiples of 16
    assert variant([(56, 48, 48)] * 2) == 1                  # 112 x 96 planes: 42 tiles
    assert variant([(48, 48, 48)] * 2, flags=0) == 1         # one potential per orbital
    assert variant([(16, 16, 16)] * 2, hgrid=(1.0, 0.9, 1.0)) == 1
    assert variant([(16, 16, 16)] * 2, hgrid=(0.8, 0.8, 0.8)) == 3
    monkeypatch.setenv("WVL_F32C_VECTOR", "1")
    assert variant([(48, 48, 48)] * 4) == 1
    monkeypatch.delenv("WVL_F32C_VECTOR")
    monkeypatch.setenv("WVL_NO_PLANE_KERNEL", "1")
    assert variant([(48, 48, 48)] * 4) == 0


def test_precondition_form_selection(dry, monkeypatch):
    """The preconditioner's default operator form: exact digit products for
    compensated plans the engine covers (a shared potential is not needed),
    the plane-resident vector form for other planes that fit, else passes."""
    q = lib.raw("wvl_plan_query")
    v = ctypes.c_int64()

    def form(dims, prec=2, flags=1, **kw):
        rc, p = _plan(dry, dims, prec=prec, flags=flags, **kw)
        assert rc == lib.WVL_OK
        assert q(p, lib.WVL_Q_PRECOND_FORM, ctypes.byref(v)) == lib.WVL_OK
        lib.wvl_plan_destroy(p)
        return v.value

    assert form([(48, 48, 48)] * 4) == 2
    assert form([(48, 48, 48)] * 2, flags=0) == 2            # one potential per orbital
    assert form([(8, 24, 16)] * 3, hgrid=(0.8, 0.8, 0.8)) == 2
    assert form([(16, 16, 16)] * 2, hgrid=(1.0, 0.9, 1.0)) == 1
    assert form([(20, 18, 17)] * 2) == 1                     # lengths not multiples of 16
    assert form([(48, 48, 48)] * 4, prec=0) == 1
    assert form([(16, 16, 16)] * 2, flags=1 | lib.WVL_FREE_BC) == 0
    monkeypatch.setenv("WVL_F32C_VECTOR", "1")
    assert form([(48, 48, 48)] * 4) == 1
    monkeypatch.delenv("WVL_F32C_VECTOR")
