"""Pins of the isolated / surface boundary-condition oracle (Sec. 3.1).

* brute force: every free 1D operator equals a rectangular matrix assembled
  entry by entry from its definition (explicit loops over coefficients and
  taps), and the 3D local Hamiltonian with free and surface conditions equals
  the Kronecker product of those matrices (and the periodic circulants along
  periodic axes); the result is symmetric;
* exact identities: the free synthesis is an isometry whose adjoint, the
  analysis, inverts it (the coarse basis functions are exact combinations of
  fine ones on the infinite line); the free magic filter and its transpose
  are adjoint;
* locality: an orbital whose coefficients vanish near the faces of the box
  sees no boundary, so free, surface and periodic conditions give the same
  H c and the same point values inside the box.
"""

import numpy as np
import pytest

from oracle import boundary as BC
from oracle import filters as OF
from oracle import wavelet as W
from paper_0904_1543_amd import inputs
from test_oracle_ops import dense_analysis, dense_conv, dense_synthesis


@pytest.fixture(scope="module")
def F():
    return OF.filters(8)


def free_synthesis_matrix(m, F):
    """(m + 14) x m: column 2i -> h_j at row 2i + j + 7, column 2i + 1 -> g_j."""
    M = np.zeros((m + 14, m))
    for i in range(m // 2):
        for k in range(len(F["h"])):
            j = F["lo"] + k
            M[2 * i + j + 7, 2 * i] += F["h"][k]
            M[2 * i + j + 7, 2 * i + 1] += F["g"][k]
    return M


def free_conv_matrix(nout, out_lo, nin, in_lo, w, lo):
    """out[K] = sum_l w_l x[K - l] for global positions K = out_lo.., x at in_lo.."""
    M = np.zeros((nout, nin))
    for a in range(nout):
        for k, wl in enumerate(w):
            b = out_lo + a - (lo + k) - in_lo
            if 0 <= b < nin:
                M[a, b] += wl
    return M


def dense_1d(m, F, free, h=1.0):
    """(S, A, Omega, T) of one axis: periodic circulants or free rectangles."""
    t = -F["r"] / (2 * h * h)
    if not free:
        return (dense_synthesis(m, F["h"], F["g"], F["lo"]),
                dense_analysis(m, F["h"], F["g"], F["lo"]),
                dense_conv(m, F["omega"], F["omega_lo"]), dense_conv(m, t, F["r_lo"]))
    S = free_synthesis_matrix(m, F)
    O = free_conv_matrix(m + 29, -14, m + 14, -7, F["omega"], F["omega_lo"])
    T = free_conv_matrix(m + 14, -7, m + 14, -7, t, F["r_lo"])
    return S, S.T, O, T


def along(x, M, axis):
    """Apply the matrix M along numpy axis `axis` of x."""
    return np.moveaxis(np.tensordot(M, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)


def apply3(x, mats):
    """mats[a - 1] along paper axis a (axis 1 = last numpy axis)."""
    for a, M in enumerate(mats):
        x = along(x, M, -1 - a)
    return x


def dense_hamiltonian(dims, bc, V, F, hg=(1.0, 1.0, 1.0)):
    """H column by column: A (Omega^T diag(V) Omega + K) S with the 1D
    matrices applied along their axes (K: the sum of the 1D kinetic
    matrices, each along its axis)."""
    n1, n2, n3 = dims
    ops = [dense_1d(2 * n, F, BC.BCS[bc][a] == "f", hg[a]) for a, n in enumerate((n1, n2, n3))]
    S = [o[0] for o in ops]
    A = [o[1] for o in ops]
    O = [o[2] for o in ops]
    T = [o[3] for o in ops]
    shape = inputs.fine_shape(dims)
    n = int(np.prod(shape))
    H = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        s = apply3(e.reshape(shape), S)
        y = V * apply3(s, O)
        k = apply3(y, [M.T for M in O])
        for a in range(3):
            k = k + along(s, T[a], -1 - a)
        H[:, j] = apply3(k, A).ravel()
    return H


@pytest.mark.parametrize("m", [4, 10])
def test_free_1d_operators_equal_their_matrices(F, m):
    rng = inputs.rng_for(m)
    x = rng.standard_normal(m)
    S, A, O, T = dense_1d(m, F, True, 0.8)
    s = BC.synthesis_1d_free(x, -1)
    assert np.max(np.abs(s - S @ x)) < 1e-15
    assert np.max(np.abs(BC.analysis_1d_free(s, -1) - A @ s)) < 1e-15
    psi = BC.magic_filter_1d_free(s, -1)
    assert np.max(np.abs(psi - O @ s)) < 1e-15
    y = rng.standard_normal(m + 29)
    assert np.max(np.abs(BC.magic_filter_t_1d_free(y, -1) - O.T @ y)) < 1e-15
    assert np.max(np.abs(BC.kinetic_1d_free(s, -1, 0.8) - T @ s)) < 1e-14


@pytest.mark.parametrize("bc", ["free", "surface"])
def test_hamiltonian_equals_kronecker_matrix(F, bc):
    dims = (2, 3, 2)
    hg = (1.0, 0.9, 1.1)
    V = inputs.potential_gauss(inputs.rng_for(3), BC.real_space_shape(dims, bc))
    H = dense_hamiltonian(dims, bc, V, F, hg)
    assert np.max(np.abs(H - H.T)) < 1e-13
    rng = inputs.rng_for(4)
    for _ in range(2):
        c = rng.standard_normal(inputs.fine_shape(dims))
        h = BC.local_hpsi_orbital(c, V, bc, hg)[0]
        assert np.max(np.abs(h.ravel() - H @ c.ravel())) < 1e-13


def test_free_synthesis_is_an_isometry_inverted_by_the_analysis():
    c = inputs.rng_for(5).standard_normal(inputs.fine_shape((5, 4, 6)))
    s = BC.synthesis(c, "free")
    assert s.shape == tuple(n + 14 for n in c.shape)
    assert abs(np.linalg.norm(s) - np.linalg.norm(c)) < 1e-13
    assert np.max(np.abs(BC.analysis(s, "free") - c)) < 1e-14


def test_free_magic_filter_adjoint():
    rng = inputs.rng_for(6)
    s = rng.standard_normal((20, 18, 24))
    y = rng.standard_normal((35, 33, 39))
    lhs = np.sum(BC.magic_filter(s, "free") * y)
    rhs = np.sum(s * BC.magic_filter_t(y, "free"))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("bc", ["free", "surface"])
def test_no_boundary_seen_away_from_the_faces(bc):
    """Coefficients only in coarse points 16..19 of 36 per axis: synthesis,
    magic filter, its transpose and the analysis spread them by at most 32
    fine points, so nothing wraps and every condition gives the same H c."""
    dims = (36, 36, 36)
    m = 72
    rng = inputs.rng_for(7)
    c = np.zeros((m, m, m))
    c[32:40, 32:40, 32:40] = rng.standard_normal((8, 8, 8))
    Vp = inputs.potential_gauss(rng, (m, m, m))
    # the same potential on the box, embedded in the larger real-space grid
    Vb = np.zeros(BC.real_space_shape(dims, bc))
    sl = tuple(slice(14, 14 + m) if BC.BCS[bc][2 - k] == "f" else slice(0, m) for k in range(3))
    Vb[sl] = Vp
    hp, psip, _ = W.local_hpsi_orbital(c, Vp)
    hb, psib, _ = BC.local_hpsi_orbital(c, Vb, bc)
    # equal up to the rounding of differently ordered sums
    assert np.max(np.abs(hb - hp)) < 1e-14 * np.max(np.abs(hp))
    assert np.max(np.abs(psib[sl] - psip)) < 1e-14 * np.max(np.abs(psip))
    assert abs(np.sum(psib ** 2) - np.sum(psip ** 2)) < 1e-13 * np.sum(psip ** 2)
