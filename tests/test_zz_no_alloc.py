"""The no-allocation orthonormalisation (scratch in a static device array of
the library) against the workspace entry point it mirrors, through the C ABI:
two calls in a row, the second on a smaller batch, each compared bit for bit
with wvl_orthonormalize on the same input and, to the parity bound, with the
float64 oracle (S = X X^T, S = L L^T, X <- L^{-1} X; Sec. 5 step VIII)."""

import ctypes

import numpy as np
import pytest
import torch

from oracle import wavelet as W
from paper_0904_1543_amd import inputs, lib, ops
from parity_helpers import TOL, assert_close

pytestmark = pytest.mark.gpu


def _orthonormalize(plan, c, noalloc):
    n = plan.norb
    S = torch.full((n, n), float("nan"), dtype=torch.float64, device=plan.dev)
    L = torch.full((n, n), float("nan"), dtype=torch.float64, device=plan.dev)
    if noalloc:
        rc = lib.raw("wvl_orthonormalize_noalloc")(plan.h, ops.ptr(c), ops.ptr(S), ops.ptr(L),
                                                   ops.stream_handle())
    else:
        rc = lib.raw("wvl_orthonormalize")(plan.h, ops.ptr(c), ops.ptr(S), ops.ptr(L),
                                           ops.ptr(plan.ws), ops.stream_handle())
    assert rc == lib.WVL_OK, lib.wvl_last_error()
    plan.sync()
    return S, L


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_noalloc_matches_workspace_entry_point(prec):
    # second call smaller: fewer orbitals on a smaller grid
    for seed, (norb, dims) in enumerate([(200, (12, 10, 9)), (37, (6, 5, 4))]):
        cs = inputs.random_case(90 + seed, norb, dims)
        print(f"[no-alloc] {prec} call {seed}: {norb} orbitals, coarse {dims}", flush=True)
        plan = ops.Plan(cs["dims"], prec=prec)
        c_ref = plan.pack(cs["C"])
        c_new = c_ref.clone()
        S_ref, L_ref = _orthonormalize(plan, c_ref, noalloc=False)
        S_new, L_new = _orthonormalize(plan, c_new, noalloc=True)
        # same kernels, same reduction order: identical results
        assert torch.equal(S_new, S_ref)
        assert torch.equal(torch.tril(L_new), torch.tril(L_ref))
        assert torch.equal(c_new, c_ref)
        # and within the parity bound of the oracle
        Xn, L = W.cholesky_orthonormalize(cs["C"])
        assert_close(np.tril(L_new.cpu().numpy()), L, 1e-12, "L")
        assert_close(plan.unpack(c_new), list(Xn), max(TOL[prec], 1e-12), "orthonormalised batch")
