"""GPU parity of the compressed storage (Sec. 2.1) and of the local
Hamiltonian on compressed orbitals (steps 1-7 of Sec. 2.4) against the float64
oracle, in the three precisions, on synthetic sphere regions (atoms-like
coarse and fine regions of a periodic box)."""

import numpy as np
import pytest

from oracle import compress as CP
from oracle import wavelet as W
from paper_0904_1543_amd import inputs, ops
from parity_helpers import TOL, assert_close, assert_scalar

pytestmark = pytest.mark.gpu

CASES = {"small": (3, (8, 6, 7)), "ragged": (2, (20, 18, 17)), "tiny": (2, (2, 3, 4))}


def _setup(case, prec, seed=120):
    norb, dims = CASES[case]
    cs = inputs.random_case(seed, norb, dims, potential="gauss16")
    seg_c, seg_f = inputs.sphere_regions(seed + 1, dims, natoms=3, rc=0.35, rf=0.18)
    plan = ops.Plan(cs["dims"], prec=prec)
    nvc, nvf = plan.set_regions(seg_c, seg_f)
    assert nvc == len(CP.region_points(seg_c)) and nvf == len(CP.region_points(seg_f))
    vecs = [CP.compress(c, seg_c, seg_f, dims) for c in cs["C"]]
    return cs, dims, seg_c, seg_f, plan, vecs


@pytest.mark.parametrize("prec", ["f64", "f32", "f32c"])
@pytest.mark.parametrize("case", list(CASES))
def test_decompress_compress(case, prec):
    cs, dims, seg_c, seg_f, plan, vecs = _setup(case, prec)
    psi_c = plan.pack_compressed(vecs)
    full = plan.unpack(plan.decompress(psi_c))
    ref = [CP.decompress(v, seg_c, seg_f, dims) for v in vecs]
    # the values as the plan stores them: float32, or the hi + lo pair
    if prec == "f32":
        ref = [r.astype(np.float32).astype(np.float64) for r in ref]
    if prec == "f32c":
        ref = [sum(p.astype(np.float64) for p in inputs.split_hilo(r)) for r in ref]
    for g, r in zip(full, ref):
        assert np.array_equal(g, r)            # pure data movement: exact
    back = plan.unpack_compressed(plan.compress(plan.pack(cs["C"])))
    refc = [CP.compress(c, seg_c, seg_f, dims) for c in cs["C"]]
    assert_close(back, refc, TOL[prec], "compress")


@pytest.mark.parametrize("prec", ["f64", "f32", "f32c"])
@pytest.mark.parametrize("case", list(CASES))
def test_local_hpsi_compressed(case, prec):
    cs, dims, seg_c, seg_f, plan, vecs = _setup(case, prec)
    psi_c = plan.pack_compressed(vecs)
    r = plan.local_hpsi_compressed(psi_c, plan.pack_potential(cs["V"]), per_orbital=True)
    tol = TOL[prec]
    ref = [CP.local_hpsi_compressed(v, cs["V"], seg_c, seg_f, dims) for v in vecs]
    assert_close(plan.unpack_compressed(r["hpsi"]), [h for h, _ in ref], tol, "compressed H psi")
    rho = sum(f * psi * psi for f, (_, psi) in zip(cs["occ"], ref))
    assert_close(r["rho"].cpu().numpy(), rho.ravel(), tol, "rho")
    assert_scalar(r["energies"][0].item(), float(np.sum(cs["V"] * rho)), tol, "E_loc")
    full = [CP.decompress(v, seg_c, seg_f, dims) for v in vecs]
    ekin = [float(np.sum(W.synthesis(c) * W.kinetic(W.synthesis(c)))) for c in full]
    assert_close(r["e_orb"].cpu().numpy()[plan.norb:], np.array(ekin), tol, "e_kin per orbital")
    # in place: hpsi_c = psi_c
    plan.local_hpsi_compressed(psi_c, plan.pack_potential(cs["V"]), out=psi_c)
    assert_close(plan.unpack_compressed(psi_c), [h for h, _ in ref], tol, "in place")


def test_whole_box_regions_equal_full_hamiltonian():
    norb, dims = 2, (10, 9, 8)
    cs = inputs.random_case(130, norb, dims, potential="gauss16")
    n1, n2, n3 = dims
    full = np.array([[0, n1 * n2 * n3]], dtype=np.int32)
    plan = ops.Plan(cs["dims"], prec="f64")
    plan.set_regions(full, full)
    vecs = [CP.compress(c, full, full, dims) for c in cs["C"]]
    r = plan.local_hpsi_compressed(plan.pack_compressed(vecs), plan.pack_potential(cs["V"]))
    h = plan.local_hpsi(plan.pack(cs["C"]), plan.pack_potential(cs["V"]))
    got = [CP.decompress(v, full, full, dims) for v in plan.unpack_compressed(r["hpsi"])]
    assert_close(got, plan.unpack(h["hpsi"]), 1e-15, "whole box vs full grid")
