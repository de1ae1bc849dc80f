"""Pins of the preconditioner oracle (Sec. 2, Eq. "precon") against mathematics.

* brute force: H_eps equals the dense matrix A3 K3 S3 - eps I assembled entry
  by entry from the 1D filter definitions (explicit loops, np.kron), and the
  Jacobi diagonal equals that matrix's diagonal;
* the linear algebra of CG: with enough steps PCG reaches numpy's dense
  solution; the error in the energy norm of H_eps decreases at every step
  (a property of conjugate gradients, preconditioned or not); the first step
  is the exact line minimiser along the preconditioned residual; the
  recurrence residual equals g - H_eps x;
* the operator: symmetric positive definite for eps < 0, and the K_0 = -eps s
  form of the kinetic recursion (Sec. 3.4) equals A Kin S - eps I.
"""

import numpy as np
import pytest

from oracle import filters as OF
from oracle import precond as PC
from oracle import wavelet as W
from paper_0904_1543_amd import inputs
from test_oracle_ops import dense_ops

SHAPES = [(8, 8, 8), (10, 6, 8)]
HG = (1.0, 0.8, 1.25)


@pytest.fixture(scope="module")
def F():
    return OF.filters(8)


def _dense_helmholtz(shape, eps, F):
    S3, A3, _, K3 = dense_ops(shape, F, HG)
    return A3 @ K3 @ S3 - eps * np.eye(S3.shape[0])


def _vec(seed, shape):
    rng = inputs.rng_for(seed)
    x = rng.standard_normal(shape)
    return x / np.linalg.norm(x)


@pytest.mark.parametrize("shape", SHAPES)
def test_operator_equals_dense_matrix(F, shape):
    eps = -0.37
    H = _dense_helmholtz(shape, eps, F)
    for seed in (1, 2):
        x = _vec(seed, shape)
        got = PC.helmholtz(x, eps, HG).ravel()
        assert np.max(np.abs(got - H @ x.ravel())) < 1e-13
    assert np.max(np.abs(H - H.T)) < 1e-13                       # symmetric
    assert np.min(np.linalg.eigvalsh(H)) > 0.36                   # >= -eps: Kin is PSD
    assert np.max(np.abs(PC.helmholtz_diagonal(shape, eps, HG).ravel() - np.diag(H))) < 1e-13


def test_diagonal_depends_only_on_the_parities():
    """The kinetic diagonal is a function of (scaling or wavelet) per axis:
    two values per axis on a periodic line."""
    d = PC.kinetic_diagonal_1d(24, 0.9)
    assert np.allclose(d[0::2], d[0], rtol=0, atol=1e-14)
    assert np.allclose(d[1::2], d[1], rtol=0, atol=1e-14)
    assert d[1] > d[0] > 0       # wavelets carry the high frequencies


@pytest.mark.parametrize("shape", SHAPES)
def test_pcg_reaches_the_dense_solution(F, shape):
    eps = -0.5
    H = _dense_helmholtz(shape, eps, F)
    g = _vec(3, shape)
    ref = np.linalg.solve(H, g.ravel())
    x, res = PC.pcg(g, eps, 120, HG)
    assert np.linalg.norm(x.ravel() - ref) / np.linalg.norm(ref) < 1e-11
    assert res < 1e-11
    # the recurrence residual is the true residual
    x5, res5 = PC.pcg(g, eps, 5, HG)
    assert abs(res5 - np.linalg.norm(g.ravel() - H @ x5.ravel())) < 1e-12


def test_energy_norm_error_decreases(F):
    shape, eps = (8, 8, 8), -0.3
    H = _dense_helmholtz(shape, eps, F)
    g = _vec(4, shape)
    ref = np.linalg.solve(H, g.ravel())
    _, _, xs = PC.pcg(g, eps, 25, HG, history=True)
    errs = [float((x.ravel() - ref) @ H @ (x.ravel() - ref)) for x in xs]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6 * errs[0]


def test_first_step_is_the_line_minimiser(F):
    """x_1 = alpha z_0 minimises the energy (1/2) x.Hx - g.x along z_0 = M^-1 g."""
    shape, eps = (10, 6, 8), -0.8
    H = _dense_helmholtz(shape, eps, F)
    g = _vec(5, shape).ravel()
    z0 = g / np.diag(H)
    a_star = (g @ z0) / (z0 @ H @ z0)
    x1, _ = PC.pcg(g.reshape(shape), eps, 1, HG)
    assert np.max(np.abs(x1.ravel() - a_star * z0)) < 1e-14


def test_zero_steps_and_zero_gradient():
    g = _vec(6, (8, 8, 8))
    x, res = PC.pcg(g, -0.4, 0)
    assert not np.any(x) and abs(res - 1.0) < 1e-15
    x, res = PC.pcg(np.zeros((8, 8, 8)), -0.4, 4)
    assert not np.any(x) and res == 0.0


def test_k0_form_of_the_kinetic_recursion():
    """A (Kin s - eps s) = A Kin S c - eps c since A S = I (Sec. 3.4, last sentence)."""
    c = _vec(7, (12, 10, 8))
    eps = -0.6
    lhs = PC.helmholtz(c, eps, HG)
    rhs = W.analysis(W.kinetic(W.synthesis(c), HG)) - eps * c
    assert np.max(np.abs(lhs - rhs)) < 1e-14


@pytest.mark.parametrize("bc", ["free", "surface"])
def test_pcg_with_isolated_axes_reaches_the_dense_solution(F, bc):
    """The Helmholtz operator of isolated / surface conditions: its dense
    matrix (explicit-loop 1D matrices, zero potential) against PCG."""
    from test_oracle_boundary import dense_hamiltonian
    from oracle import boundary as BCo
    dims, eps = (3, 2, 3), -0.45
    shape = inputs.fine_shape(dims)
    H = dense_hamiltonian(dims, bc, np.zeros(BCo.real_space_shape(dims, bc)), F, HG)
    H = H - eps * np.eye(H.shape[0])
    assert np.max(np.abs(PC.helmholtz_diagonal(shape, eps, HG, bc).ravel() - np.diag(H))) < 1e-13
    g = _vec(12, shape)
    ref = np.linalg.solve(H, g.ravel())
    x, res = PC.pcg(g, eps, 150, HG, bc=bc)
    assert np.linalg.norm(x.ravel() - ref) / np.linalg.norm(ref) < 1e-11
