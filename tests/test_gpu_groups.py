"""The plane kernel's density groups: with a shared potential, the orbitals of
a batch are split into groups of G whose density partials are accumulated in
orbital order, then summed over groups.  Every case here has G > 1 (asserted
from the plan) and a ragged last group, and compares rho, the total E_loc,
E_kin, H*psi and the per-orbital energies with the float64 oracle, for the
matrix-core and vector engines and the three precisions (Sec. 2.5, Eq.
"density")."""

import pytest

from oracle import wavelet as W
from paper_0904_1543_amd import inputs, lib, ops
from parity_helpers import TOL, assert_close, assert_scalar

pytestmark = pytest.mark.gpu

# (orbitals, coarse dims): fine (16, 12, 64), norb * m3 / 1024 -> G
CASES = {"G2": (33, (8, 6, 32)), "G4": (67, (8, 6, 32)), "G8": (137, (8, 6, 32))}
EXPECT_G = {"G2": 2, "G4": 4, "G8": 8}


@pytest.fixture(scope="module")
def refs():
    out = {}
    for name, (norb, dims) in CASES.items():
        cs = inputs.random_case(70 + norb, norb, dims, potential="gauss16")
        out[name] = (cs, W.local_hpsi(cs["C"], cs["V"], cs["occ"]))
    return out


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("form", ["f64", "f64_vector", "f64_occ2", "f64_occ2_mem", "f32", "f32c"])
def test_grouped_density_and_energies(refs, case, form, monkeypatch):
    prec = form.split("_")[0]
    if form == "f64_vector":
        monkeypatch.setenv("WVL_XY_VECTOR", "1")
    if form.startswith("f64_occ2"):   # 2 waves per SIMD: the group's density plane kept in LDS
        monkeypatch.setenv("WVL_PLANE_OCCUPANCY", "2")
    if form == "f64_occ2_mem":        # ... or, at the same occupancy, in memory
        monkeypatch.setenv("WVL_NO_RHO_LDS", "1")
    cs, ref = refs[case]
    plan = ops.Plan(cs["dims"], prec=prec)
    assert plan.query(lib.WVL_Q_GROUP) == EXPECT_G[case]
    assert plan.query(lib.WVL_Q_VARIANT) == (2 if form.startswith("f64") and form != "f64_vector"
                                             else 1)
    r = plan.local_hpsi(plan.pack(cs["C"]), plan.pack_potential(cs["V"]), per_orbital=True)
    tol = TOL[prec]
    assert_close(r["rho"].cpu().numpy(), ref["rho"].ravel(), tol, "rho")
    e = r["energies"].cpu().numpy()
    assert_scalar(e[0], ref["e_loc"], tol, "E_loc")
    assert_scalar(e[1], ref["e_kin"], tol, "E_kin")
    assert_close(plan.unpack(r["hpsi"]), list(ref["hpsi"]), tol, "hpsi")
    eo = r["e_orb"].cpu().numpy()
    assert_close(eo[: plan.norb], ref["e_loc_orb"], tol, "e_pot per orbital")
    assert_close(eo[plan.norb:], ref["e_kin_orb"], tol, "e_kin per orbital")
