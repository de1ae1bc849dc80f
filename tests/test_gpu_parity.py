"""GPU parity: every C-ABI operation against the float64 oracle, element by
element, on seeded inputs, in the three precisions.

Bounds (normwise relative error ||gpu - oracle|| / ||oracle|| per result):
float64 1e-12, plain float32 2e-6, compensated float32 (hi + lo) 1e-10.
Shapes cover several tiles with ragged tails, lines shorter than the filters
(fine length 4 < 16 taps: the periodic wrap applies several times), and an
uneven batch with one potential per orbital.
"""

import numpy as np
import pytest
import torch

from oracle import wavelet as W
from paper_0904_1543_amd import inputs
from paper_0904_1543_amd import ops
from parity_helpers import assert_close

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6, "f32c": 1e-10}
PRECS = ["f64", "f32", "f32c"]
CASES = {
    "small": (3, (8, 6, 5)),      # fine (10, 12, 16)
    "tiny": (2, (2, 3, 4)),       # fine (8, 6, 4): lines shorter than the filters
    "ragged": (2, (20, 18, 17)),  # fine (34, 36, 40): several ragged tiles per pass
}


def setup(case, prec, seed=5, potential="uniform"):
    norb, dims = CASES[case]
    cs = inputs.random_case(seed, norb, dims, potential=potential)
    plan = ops.Plan(cs["dims"], prec=prec)
    return cs, plan


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(CASES))
def test_transforms(case, prec):
    cs, plan = setup(case, prec)
    C = cs["C"]
    c = plan.pack(C)
    tol = TOL[prec]
    s = plan.synthesis(c)
    assert_close(plan.unpack(s), [W.synthesis(x) for x in C], tol)
    a = plan.analysis(c)
    assert_close(plan.unpack(a), [W.analysis(x) for x in C], tol)
    mf = plan.magic_filter(c)
    assert_close(plan.unpack(mf), [W.magic_filter(x) for x in C], tol)
    mft = plan.magic_filter(c, transpose=True)
    assert_close(plan.unpack(mft), [W.magic_filter_t(x) for x in C], tol)
    # round trip on the GPU
    back = plan.analysis(s)
    assert_close(plan.unpack(back), list(C), 4 * tol)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["small", "ragged", "tiny"])
def test_kinetic(case, prec):
    norb, dims = CASES[case]
    cs = inputs.random_case(8, norb, dims)
    hg = (1.0, 0.7, 1.3)
    plan = ops.Plan(cs["dims"], prec=prec, hgrid=hg)
    C = cs["C"]
    K0 = [np.cos(x) for x in C]
    c, k0 = plan.pack(C), plan.pack(K0)
    out = plan.kinetic(c)
    assert_close(plan.unpack(out), [W.kinetic(x, hg) for x in C], TOL[prec])
    out2 = plan.kinetic(c, k0)
    assert_close(plan.unpack(out2), [W.kinetic(x, hg, k0=k) for x, k in zip(C, K0)], TOL[prec])
    # k0 may be the output buffer itself (accumulate in place)
    acc = plan.pack(K0)
    plan.kinetic(c, acc, out=acc)
    assert_close(plan.unpack(acc), [W.kinetic(x, hg, k0=k) for x, k in zip(C, K0)], TOL[prec])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(CASES))
def test_local_density(case, prec):
    cs, plan = setup(case, prec)
    c = plan.pack(cs["C"])
    rho = plan.local_density(c).cpu().numpy()
    ref = W.local_density(cs["C"], cs["occ"]).ravel()
    assert_close(rho, ref, TOL[prec])
    # accumulate
    rho2 = plan.local_density(c, rho=torch.from_numpy(ref.copy()).cuda(), accumulate=True)
    assert_close(rho2.cpu().numpy(), 2 * ref, TOL[prec])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(CASES))
def test_local_hpsi(case, prec):
    cs, plan = setup(case, prec, potential="gauss16")
    C, V, occ = cs["C"], cs["V"], cs["occ"]
    c = plan.pack(C)
    Vt = plan.pack_potential(V)
    r = plan.local_hpsi(c, Vt, per_orbital=True)
    ref = W.local_hpsi(C, V, occ)
    tol = TOL[prec]
    assert_close(plan.unpack(r["hpsi"]), list(ref["hpsi"]), tol)
    assert_close(r["rho"].cpu().numpy(), ref["rho"].ravel(), tol)
    e = r["energies"].cpu().numpy()
    assert abs(e[0] - ref["e_loc"]) <= tol * abs(ref["e_loc"])
    assert abs(e[1] - ref["e_kin"]) <= tol * abs(ref["e_kin"])
    eo = r["e_orb"].cpu().numpy()
    assert_close(eo[: plan.norb], ref["e_loc_orb"], tol)
    assert_close(eo[plan.norb:], ref["e_kin_orb"], tol)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["small", "tiny"])
def test_local_hpsi_pass_by_pass_variant(case, prec, monkeypatch):
    """The variant with one 1D pass per axis (used when a plane does not fit
    in LDS) gives the same result."""
    monkeypatch.setenv("WVL_NO_PLANE_KERNEL", "1")
    cs, plan = setup(case, prec, potential="gauss16")
    assert _variant(plan) == 0
    C, V, occ = cs["C"], cs["V"], cs["occ"]
    r = plan.local_hpsi(plan.pack(C), plan.pack_potential(V), per_orbital=True)
    ref = W.local_hpsi(C, V, occ)
    assert_close(plan.unpack(r["hpsi"]), list(ref["hpsi"]), TOL[prec])
    assert_close(r["rho"].cpu().numpy(), ref["rho"].ravel(), TOL[prec])
    e = r["energies"].cpu().numpy()
    assert abs(e[0] - ref["e_loc"]) <= TOL[prec] * abs(ref["e_loc"])
    assert abs(e[1] - ref["e_kin"]) <= TOL[prec] * abs(ref["e_kin"])


def _variant(plan):
    from paper_0904_1543_amd import lib
    import ctypes
    v = ctypes.c_int32()
    lib.wvl_plan_tuning(plan.h, ctypes.byref(v), None, 0)
    return v.value


@pytest.mark.parametrize("prec,expect", [("f64", 2), ("f32", 1), ("f32c", 1)])
def test_plane_kernel_is_the_default(prec, expect):
    """float64 runs its in-plane passes on the matrix cores, the other
    precisions on the vector units."""
    cs, plan = setup("ragged", prec)
    assert _variant(plan) == expect


@pytest.mark.parametrize("case", list(CASES))
def test_local_hpsi_f64_vector_engine(case, monkeypatch):
    """The vector-FMA form of the float64 in-plane passes gives the same
    result as the oracle (and as the matrix-core form)."""
    monkeypatch.setenv("WVL_XY_VECTOR", "1")
    cs, plan = setup(case, "f64", potential="gauss16")
    assert _variant(plan) == 1
    C, V, occ = cs["C"], cs["V"], cs["occ"]
    r = plan.local_hpsi(plan.pack(C), plan.pack_potential(V), per_orbital=True)
    ref = W.local_hpsi(C, V, occ)
    assert_close(plan.unpack(r["hpsi"]), list(ref["hpsi"]), TOL["f64"])
    assert_close(r["rho"].cpu().numpy(), ref["rho"].ravel(), TOL["f64"])
    eo = r["e_orb"].cpu().numpy()
    assert_close(eo[: plan.norb], ref["e_loc_orb"], TOL["f64"])
    assert_close(eo[plan.norb:], ref["e_kin_orb"], TOL["f64"])


@pytest.mark.parametrize("dims", [(16, 16, 3), (33, 31, 2), (48, 41, 2), (64, 64, 2)])
def test_local_hpsi_f64_plane_sizes(dims):
    """Planes that are whole multiples of the 16 x 16 matrix tiles, ragged
    ones, and the largest supported plane (128 x 128 fine)."""
    cs = inputs.random_case(21, 2, dims, potential="gauss16")
    plan = ops.Plan(cs["dims"], prec="f64")
    assert _variant(plan) == 2
    C, V, occ = cs["C"], cs["V"], cs["occ"]
    r = plan.local_hpsi(plan.pack(C), plan.pack_potential(V), per_orbital=True)
    ref = W.local_hpsi(C, V, occ)
    assert_close(plan.unpack(r["hpsi"]), list(ref["hpsi"]), TOL["f64"])
    e = r["energies"].cpu().numpy()
    assert abs(e[0] - ref["e_loc"]) <= TOL["f64"] * abs(ref["e_loc"])
    assert abs(e[1] - ref["e_kin"]) <= TOL["f64"] * abs(ref["e_kin"])


@pytest.mark.parametrize("prec", PRECS)
def test_local_hpsi_scaled(prec):
    """pot_scale / kin_scale weight the two parts: H' = a Hloc + b Kin."""
    cs, plan = setup("small", prec, seed=9)
    C, V, occ = cs["C"], cs["V"], cs["occ"]
    c, Vt = plan.pack(C), plan.pack_potential(V)
    r = plan.local_hpsi(c, Vt, pot_scale=0.3, kin_scale=-1.7)
    ref = []
    for x in C:
        s = W.synthesis(x)
        y = 0.3 * V * W.magic_filter(s)
        ref.append(W.analysis(W.magic_filter_t(y) - 1.7 * W.kinetic(s)))
    assert_close(plan.unpack(r["hpsi"]), ref, TOL[prec])
    # energies are those of the unweighted operators
    full = W.local_hpsi(C, V, occ)
    e = r["energies"].cpu().numpy()
    assert abs(e[1] - full["e_kin"]) <= TOL[prec] * abs(full["e_kin"])


@pytest.mark.parametrize("prec", PRECS)
def test_uneven_batch_per_orbital_potential(prec):
    cs = inputs.random_uneven_case(31, 5, lo=2, hi=11)
    plan = ops.Plan(cs["dims"], prec=prec, shared_v=False)
    c = plan.pack(cs["C"])
    Vt = plan.pack_potential(cs["V"])
    r = plan.local_hpsi(c, Vt, rho=False, per_orbital=True)
    got = plan.unpack(r["hpsi"])
    ref = [W.local_hpsi_orbital(x, v)[0] for x, v in zip(cs["C"], cs["V"])]
    assert_close(got, ref, TOL[prec])
    eo = r["e_orb"].cpu().numpy()
    ref_e = W.local_hpsi(cs["C"], cs["V"], cs["occ"], shared_v=False)
    assert_close(eo[: plan.norb], ref_e["e_loc_orb"], TOL[prec])
    assert_close(eo[plan.norb:], ref_e["e_kin_orb"], TOL[prec])
    e = r["energies"].cpu().numpy()
    assert abs(e[0] - float(np.dot(cs["occ"], ref_e["e_loc_orb"]))) <= TOL[prec] * abs(e[0])
    # the other operations on the uneven batch
    s = plan.synthesis(c)
    assert_close(plan.unpack(s), [W.synthesis(x) for x in cs["C"]], TOL[prec])


def test_float64_runs_are_bitwise_reproducible():
    cs, plan = setup("ragged", "f64", potential="gauss16")
    c, Vt = plan.pack(cs["C"]), plan.pack_potential(cs["V"])
    r1 = plan.local_hpsi(c, Vt)
    r2 = plan.local_hpsi(c, Vt)
    assert torch.equal(r1["hpsi"], r2["hpsi"])
    assert torch.equal(r1["rho"], r2["rho"])
    assert torch.equal(r1["energies"], r2["energies"])


def test_every_output_element_is_written():
    cs, plan = setup("ragged", "f64", potential="gauss16")
    c, Vt = plan.pack(cs["C"]), plan.pack_potential(cs["V"])
    out = torch.full_like(c, float("nan"))
    plan.local_hpsi(c, Vt, out=out)
    assert not torch.isnan(out).any()
    for fn in (plan.synthesis, plan.analysis, plan.magic_filter):
        o = torch.full_like(c, float("nan"))
        fn(c, out=o)
        assert not torch.isnan(o).any()


def test_graph_replay_matches_eager():
    cs = inputs.random_case(12, 3, (8, 6, 5), potential="gauss16")
    eager = ops.Plan(cs["dims"], prec="f64")
    graph = ops.Plan(cs["dims"], prec="f64", graph=True)
    c, Vt = eager.pack(cs["C"]), eager.pack_potential(cs["V"])
    ref = eager.local_hpsi(c, Vt)
    out = graph.empty()
    rho = torch.empty_like(ref["rho"])
    en = torch.empty(2, dtype=torch.float64, device="cuda:0")
    import ctypes
    from paper_0904_1543_amd import lib
    for rep in range(4):
        out.fill_(float("nan"))
        rho.zero_()
        lib.wvl_local_hpsi(graph.h, ops.ptr(c), ops.ptr(Vt), 1.0, 1.0, ops.ptr(out), ops.ptr(rho),
                           ctypes.c_void_p(en.data_ptr()), ctypes.c_void_p(en.data_ptr() + 8), None,
                           ops.ptr(graph.ws), ops.stream_handle())
        torch.cuda.synchronize()
        assert torch.equal(out, ref["hpsi"]), rep
        assert torch.equal(rho, ref["rho"]), rep
        assert torch.equal(en, ref["energies"]), rep
        _ = (c * 2.0).sum().item()   # unrelated eager work between replays


@pytest.mark.parametrize("prec", PRECS)
def test_fused_last_z_pass_is_bitwise_equal(prec, monkeypatch):
    """The fused last z step (W_z^T t + K_z c + kxy in one launch) keeps the
    association of the two separate passes: same bits, same energies."""
    cs = inputs.random_case(61, 3, (20, 18, 17), potential="gauss16")
    fused = ops.Plan(cs["dims"], prec=prec)
    monkeypatch.setenv("WVL_NO_ZFUSE", "1")
    split = ops.Plan(cs["dims"], prec=prec)
    c, Vt = fused.pack(cs["C"]), fused.pack_potential(cs["V"])
    a = fused.local_hpsi(c, Vt, pot_scale=0.7, kin_scale=1.3, per_orbital=True)
    b = split.local_hpsi(c, Vt, pot_scale=0.7, kin_scale=1.3, per_orbital=True)
    assert torch.equal(a["hpsi"], b["hpsi"])
    assert torch.equal(a["e_orb"], b["e_orb"])
    assert torch.equal(a["energies"], b["energies"])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("form", ["default", "pass_by_pass", "vector_engine", "persistent"])
def test_local_hpsi_in_place(prec, form, monkeypatch):
    """hpsi = c: the result replaces the coefficients.  The fused last z step
    would read the periodic wrap of c after overwriting it, so the library
    runs that step as two passes here; every launch sequence is checked."""
    if form == "vector_engine" and prec != "f64":
        pytest.skip("the vector engine is the default for this precision")
    if form == "pass_by_pass":
        monkeypatch.setenv("WVL_NO_PLANE_KERNEL", "1")
    if form == "vector_engine":
        monkeypatch.setenv("WVL_XY_VECTOR", "1")
    norb, dims = CASES["ragged"]
    cs = inputs.random_case(61, norb, dims, potential="gauss16")
    plan = ops.Plan(cs["dims"], prec=prec, persistent=(form == "persistent"))
    C, V, occ = cs["C"], cs["V"], cs["occ"]
    c = plan.pack(C)
    Vt = plan.pack_potential(V)
    out_sep = plan.local_hpsi(c, Vt, per_orbital=True)
    r = plan.local_hpsi(c, Vt, out=c, per_orbital=True)
    assert r["hpsi"].data_ptr() == c.data_ptr()
    ref = W.local_hpsi(C, V, occ)
    tol = TOL[prec]
    assert_close(plan.unpack(c), list(ref["hpsi"]), tol, "in-place hpsi")
    assert_close(r["rho"].cpu().numpy(), ref["rho"].ravel(), tol, "rho")
    eo = r["e_orb"].cpu().numpy()
    assert_close(eo[plan.norb:], ref["e_kin_orb"], tol, "e_kin per orbital")
    # the separate-output call agrees with the in-place one
    assert_close(plan.unpack(c), plan.unpack(out_sep["hpsi"]), tol, "in place vs separate")


@pytest.mark.parametrize("prec", PRECS)
def test_energy_gradient_with_occupations(prec):
    """wvl_energy_gradient applies 2 f_b on the device, for unequal f_b."""
    norb, dims = CASES["small"]
    cs = inputs.random_case(62, norb, dims, potential="gauss16")
    occ = np.array([2.0, 0.5, 1.25])
    plan = ops.Plan(cs["dims"], prec=prec, occ=occ)
    c = plan.pack(cs["C"])
    g = plan.energy_gradient(c, plan.pack_potential(cs["V"]), g_loc=0.75, g_kin=-1.5)
    ref = []
    for x, f in zip(cs["C"], occ):
        s = W.synthesis(x)
        hl = W.analysis(W.magic_filter_t(cs["V"] * W.magic_filter(s)))
        hk = W.analysis(W.kinetic(s))
        ref.append(2.0 * f * (0.75 * hl - 1.5 * hk))
    assert_close(plan.unpack(g), ref, TOL[prec], "energy gradient")
