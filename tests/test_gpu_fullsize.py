"""Parity at the benchmark's full size and launch configuration: 256
orbitals of coarse 48^3 (fine 96^3) with the shared 16-Gaussian potential.

The oracle cannot run the whole batch in a test, so sampled orbitals are
checked one by one (local H*psi and their per-orbital energies), and the
orthonormalisation through properties that hold at any size: L against the
Cholesky factor of the overlap computed on the host, and the orthonormality
of the result.
"""

import numpy as np
import pytest
import torch

from oracle import wavelet as W
from parity_helpers import assert_close
from paper_0904_1543_amd import inputs, ops

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32c": 1e-10}
SAMPLE = [0, 97, 255]


@pytest.fixture(scope="module")
def c3():
    return inputs.workload(3)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_sampled_orbitals_full_batch(c3, prec):
    plan = ops.Plan(c3["dims"], prec=prec)
    c = plan.pack(c3["C"])
    r = plan.local_hpsi(c, plan.pack_potential(c3["V"]), per_orbital=True)
    got = plan.to_f64(r["hpsi"])
    eo = r["e_orb"].cpu().numpy()
    ref = W.local_hpsi(c3["C"][SAMPLE], c3["V"], c3["occ"][SAMPLE])
    M = plan.M[0]
    for i, b in enumerate(SAMPLE):
        g = got[b * M:(b + 1) * M].cpu().numpy()
        assert_close(g, ref["hpsi"][i], TOL[prec], b)
        assert abs(eo[b] - ref["e_loc_orb"][i]) <= TOL[prec] * abs(ref["e_loc_orb"][i]), b
        n = plan.norb
        assert abs(eo[n + b] - ref["e_kin_orb"][i]) <= TOL[prec] * abs(ref["e_kin_orb"][i]), b


def test_orthonormalize_full_batch(c3):
    plan = ops.Plan(c3["dims"], prec="f64")
    c = plan.pack(c3["C"])
    S_gpu, L_gpu = plan.orthonormalize(c)
    plan.sync()
    X = c3["C"].reshape(len(c3["C"]), -1)
    S = X @ X.T
    L = np.linalg.cholesky(S)
    assert_close(S_gpu.cpu().numpy(), S, 1e-13)
    assert_close(np.tril(L_gpu.cpu().numpy()), L, 1e-12)
    # the orthonormalised batch has the identity as its overlap
    S2 = plan.overlap(c).cpu().numpy()
    assert np.max(np.abs(S2 - np.eye(plan.norb))) < 1e-12
    del c
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def c3_density(c3):
    """rho = sum_b f_b psi_b^2 and E_loc = sum_r V rho over all 256 orbitals,
    from the oracle in a pool of host threads over orbitals (summed in
    orbital order)."""
    from concurrent.futures import ThreadPoolExecutor
    import os
    C, occ = c3["C"], c3["occ"]
    rho = None
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        for b, psi in enumerate(ex.map(W.point_values, C)):
            rho = occ[b] * psi * psi if rho is None else rho + occ[b] * psi * psi
    return rho, float(np.sum(c3["V"] * rho))


@pytest.mark.parametrize("prec", ["f64", "f32", "f32c"])
def test_density_and_e_loc_full_batch(c3, c3_density, prec):
    """The bench's batch (density groups of 8 orbitals in the plane kernel):
    rho and the total E_loc against the oracle over every orbital."""
    from paper_0904_1543_amd import lib
    from parity_helpers import assert_scalar
    tol = {"f64": 1e-12, "f32": 2e-6, "f32c": 1e-10}[prec]
    plan = ops.Plan(c3["dims"], prec=prec)
    assert plan.query(lib.WVL_Q_GROUP) == 8
    r = plan.local_hpsi(plan.pack(c3["C"]), plan.pack_potential(c3["V"]))
    rho_ref, eloc_ref = c3_density
    assert_close(r["rho"].cpu().numpy(), rho_ref.ravel(), tol, "rho")
    assert_scalar(r["energies"][0].item(), eloc_ref, tol, "E_loc")
    del r
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_precondition_full_batch_sampled(c3, prec):
    """The preconditioner on the 256 x 96^3 batch: sampled orbitals against
    the oracle running the same 3 conjugate-gradient steps."""
    from oracle import precond as PC
    eps = -inputs.rng_for(31).uniform(0.1, 1.0, size=len(c3["dims"]))
    plan = ops.Plan(c3["dims"], prec=prec)
    gt = plan.to_f64(plan.precondition(plan.pack(c3["C"]), eps, 3))
    M = plan.M[0]
    tol = TOL[prec]
    for b in (0, 200):
        ref, _ = PC.pcg(c3["C"][b], eps[b], 3)
        assert_close(gt[b * M:(b + 1) * M].cpu().numpy(), ref, tol, f"orbital {b}")
    del gt
    torch.cuda.empty_cache()
