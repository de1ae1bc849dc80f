"""Pins of the oracle's operators against mathematics.

* brute force: every 3D operator equals a dense matrix assembled entry by
  entry from the 1D definitions (explicit loops) and combined with np.kron;
* Fourier: analysis of the exact fine coefficients of a plane wave gives its
  exact coarse scaling and wavelet coefficients (phi-hat, psi-hat from the
  infinite product), the magic filter returns its point values, and the
  kinetic energy of a cosine is (1/2) int |f'|^2, to the order of the filters;
* invariants: orthogonality of the transform, adjointness, the density and
  energy identities, exact central differences of quadratic functionals,
  orthonormality after the Cholesky step.
"""

import math

import mpmath as mp
import numpy as np
import pytest

from oracle import filters as OF
from oracle import wavelet as W
from paper_0904_1543_amd import inputs


@pytest.fixture(scope="module")
def F():
    return OF.filters(8)


# ---------------------------------------------------------------- dense 1D matrices

def dense_conv(m, w, lo):
    M = np.zeros((m, m))
    for I in range(m):
        for k, wl in enumerate(w):
            l = lo + k
            M[I, (I - l) % m] += wl
    return M


def dense_synthesis(m, h, g, lo):
    M = np.zeros((m, m))
    for i in range(m // 2):
        for k in range(len(h)):
            j = lo + k
            M[(2 * i + j) % m, 2 * i] += h[k]
            M[(2 * i + j) % m, 2 * i + 1] += g[k]
    return M


def dense_analysis(m, h, g, lo):
    M = np.zeros((m, m))
    for i in range(m // 2):
        for k in range(len(h)):
            j = lo + k
            M[2 * i, (2 * i + j) % m] += h[k]
            M[2 * i + 1, (2 * i + j) % m] += g[k]
    return M


def kron3(M3, M2, M1):
    return np.kron(M3, np.kron(M2, M1))


def dense_ops(shape, F, hgrid=(1.0, 1.0, 1.0)):
    m3, m2, m1 = shape
    S = [dense_synthesis(m, F["h"], F["g"], F["lo"]) for m in (m1, m2, m3)]
    A = [dense_analysis(m, F["h"], F["g"], F["lo"]) for m in (m1, m2, m3)]
    O = [dense_conv(m, F["omega"], F["omega_lo"]) for m in (m1, m2, m3)]
    T = [dense_conv(m, -F["r"] / (2 * hh * hh), F["r_lo"]) for m, hh in zip((m1, m2, m3), hgrid)]
    I = [np.eye(m) for m in (m1, m2, m3)]
    S3 = kron3(S[2], S[1], S[0])
    A3 = kron3(A[2], A[1], A[0])
    O3 = kron3(O[2], O[1], O[0])
    K3 = kron3(T[2], I[1], I[0]) + kron3(I[2], T[1], I[0]) + kron3(I[2], I[1], T[0])
    return S3, A3, O3, K3


SHAPES = [(8, 8, 8), (10, 6, 8), (4, 12, 6)]


@pytest.mark.parametrize("shape", SHAPES)
def test_3d_operators_equal_dense_kronecker(shape, F):
    rng = np.random.default_rng(11)
    S3, A3, O3, K3 = dense_ops(shape, F, hgrid=(1.0, 0.7, 1.3))
    x = rng.standard_normal(shape)
    xv = x.ravel()
    assert np.allclose(W.synthesis(x).ravel(), S3 @ xv, atol=1e-13, rtol=0)
    assert np.allclose(W.analysis(x).ravel(), A3 @ xv, atol=1e-13, rtol=0)
    assert np.allclose(W.magic_filter(x).ravel(), O3 @ xv, atol=1e-13, rtol=0)
    assert np.allclose(W.magic_filter_t(x).ravel(), O3.T @ xv, atol=1e-13, rtol=0)
    assert np.allclose(W.kinetic(x, (1.0, 0.7, 1.3)).ravel(), K3 @ xv, atol=1e-12, rtol=0)
    # analysis is the transpose of synthesis
    assert np.allclose(A3, S3.T, atol=1e-15)
    # the full local Hamiltonian
    V = rng.uniform(-1, 0, shape)
    H = A3 @ (O3.T @ np.diag(V.ravel()) @ O3 + K3) @ S3
    Hc, _, _ = W.local_hpsi_orbital(x, V, (1.0, 0.7, 1.3))
    assert np.allclose(Hc.ravel(), H @ xv, atol=1e-12, rtol=0)
    assert np.allclose(H, H.T, atol=1e-12)
    # kinetic operator is positive semidefinite
    ev = np.linalg.eigvalsh(0.5 * (K3 + K3.T))
    assert ev.min() > -1e-12


def test_3d_hamiltonian_dense_16cubed(F):
    """Brute force at fine 16^3 (4096 x 4096) for the whole local H."""
    shape = (16, 16, 16)
    S3, A3, O3, K3 = dense_ops(shape, F)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(shape)
    V = rng.uniform(-1, 0, shape)
    Hx = A3 @ (O3.T @ (V.ravel() * (O3 @ (S3 @ x.ravel()))) + K3 @ (S3 @ x.ravel()))
    Hc, _, _ = W.local_hpsi_orbital(x, V)
    assert np.max(np.abs(Hc.ravel() - Hx)) < 1e-12


# ---------------------------------------------------------------- orthogonal transform

@pytest.mark.parametrize("shape", [(8, 8, 8), (32, 16, 24), (6, 4, 10)])
def test_analysis_inverts_synthesis(shape):
    rng = np.random.default_rng(3)
    c = rng.standard_normal(shape)
    s = W.synthesis(c)
    assert np.max(np.abs(W.analysis(s) - c)) < 1e-13
    assert np.max(np.abs(W.synthesis(W.analysis(c)) - c)) < 1e-13
    assert abs(np.linalg.norm(s) - np.linalg.norm(c)) < 1e-13 * np.linalg.norm(c)


def test_constant_scaling_input():
    """Only scaling components, all equal to C: s = C / (2 sqrt2) everywhere
    (sum_{j even} h_j = sum_{j odd} h_j = 1/sqrt2 along each axis)."""
    c = np.zeros((16, 12, 8))
    c[0::2, 0::2, 0::2] = 3.0
    s = W.synthesis(c)
    assert np.max(np.abs(s - 3.0 / (2 * math.sqrt(2)))) < 1e-14


def test_synthesised_wavelet_has_vanishing_moments():
    m = 64
    x = np.zeros(m)
    x[2 * 16 + 1] = 1.0       # one wavelet coefficient, away from the wrap
    s = W.synthesis_1d(x, 0)
    k = np.arange(m, dtype=np.float64)
    for p in range(8):
        assert abs(np.sum(s * (k - 32) ** p)) < 1e-9 * 10 ** p
    assert abs(np.sum(s * (k - 32) ** 8)) > 1e-3


# ---------------------------------------------------------------- Fourier pins

def _phi_hat(h, lo, xi, terms=70):
    p = mp.mpc(1)
    for k in range(1, terms + 1):
        t = xi / mp.mpf(2) ** k
        p *= mp.fsum(hj * mp.expj(t * (lo + i)) for i, hj in enumerate(h)) / mp.sqrt(2)
    return p


def _psi_hat(h, g, lo, xi):
    t = xi / 2
    m1 = mp.fsum(gj * mp.expj(t * (lo + i)) for i, gj in enumerate(g)) / mp.sqrt(2)
    return m1 * _phi_hat(h, lo, t)


def test_analysis_of_plane_wave_is_exact():
    """f(x) = cos(xi x): exact fine coefficients s_k = Re(e^{i xi k} Phi(xi));
    exact coarse coefficients c_i = sqrt2 Re(e^{2 i xi i} Phi(2 xi)) and
    d_i = sqrt2 Re(e^{2 i xi i} Psi(2 xi)) (orthonormal basis, spacing 2)."""
    Fm = OF.filters_mp(8)
    m, kk = 32, 3
    with mp.workdps(30):
        xi = 2 * mp.pi * kk / m
        ph1 = complex(_phi_hat(Fm["h"], Fm["lo"], xi))
        ph2 = complex(_phi_hat(Fm["h"], Fm["lo"], 2 * xi))
        ps2 = complex(_psi_hat(Fm["h"], Fm["g"], Fm["lo"], 2 * xi))
    xif = float(xi)
    k = np.arange(m)
    s = np.real(np.exp(1j * xif * k) * ph1)
    i = np.arange(m // 2)
    c = math.sqrt(2) * np.real(np.exp(2j * xif * i) * ph2)
    d = math.sqrt(2) * np.real(np.exp(2j * xif * i) * ps2)
    x = W.analysis_1d(s, 0)
    assert np.max(np.abs(x[0::2] - c)) < 1e-14
    assert np.max(np.abs(x[1::2] - d)) < 1e-14
    assert np.max(np.abs(d)) > 1e-6     # the wavelet channel is not trivially zero


def test_magic_filter_gives_point_values_of_smooth_function():
    Fm = OF.filters_mp(8)
    m, kk = 32, 1
    with mp.workdps(30):
        xi = 2 * mp.pi * kk / m
        ph = complex(_phi_hat(Fm["h"], Fm["lo"], xi))
    k = np.arange(m)
    s = np.real(np.exp(1j * float(xi) * k) * ph)
    pv = W.conv(s, OF.filters(8)["omega"], OF.filters(8)["omega_lo"], 0)
    assert np.max(np.abs(pv - np.cos(float(xi) * k))) < 1e-10
    # the transposed filter is not the point-value map (the filter is not symmetric)
    pvt = W.conv_t(s, OF.filters(8)["omega"], OF.filters(8)["omega_lo"], 0)
    assert np.max(np.abs(pvt - np.cos(float(xi) * k))) > 1e-3


@pytest.mark.parametrize("hg", [1.0, 0.5])
def test_kinetic_energy_of_cosine(hg):
    """<s, T s> = (1/2) int_0^L |f'|^2 = xi_phys^2 L / 4 for f = cos(xi_phys x)
    on a period L = m h, with s_j = sqrt(h) Re(e^{i xi j} Phi(xi)),
    xi = xi_phys h."""
    Fm = OF.filters_mp(8)
    m, kk = 32, 1
    with mp.workdps(30):
        xi = 2 * mp.pi * kk / m
        ph = complex(_phi_hat(Fm["h"], Fm["lo"], xi))
    j = np.arange(m)
    s = math.sqrt(hg) * np.real(np.exp(1j * float(xi) * j) * ph)
    e = float(np.dot(s, W.kinetic_1d(s, 0, hg)))
    xphys = float(xi) / hg
    L = m * hg
    ref = xphys ** 2 * L / 4
    assert abs(e - ref) < 1e-10 * ref


@pytest.mark.parametrize("m", [8, 16, 30])
def test_kinetic_on_fourier_modes(m, F):
    """Circulant eigenvalues: the 1D kinetic operator multiplies e^{2 pi i k n/m}
    by the DFT of its periodised filter (library FFT), and kills constants."""
    t = -F["r"] / 2.0
    col = np.zeros(m)
    for k, tl in enumerate(t):
        col[(F["r_lo"] + k) % m] += tl
    lam = np.fft.fft(col)
    n = np.arange(m)
    for k in range(m):
        v = np.cos(2 * np.pi * k * n / m)
        out = W.kinetic_1d(v, 0, 1.0)
        assert np.max(np.abs(out - lam[k].real * v)) < 1e-13
    assert np.max(np.abs(W.kinetic_1d(np.full(m, 2.5), 0, 1.0))) < 1e-13
    assert np.max(np.abs(W.kinetic(np.full((m, 6, 4), 2.5)))) < 1e-13


# ---------------------------------------------------------------- adjoint / energies

def test_magic_filter_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((12, 10, 16))
    y = rng.standard_normal((12, 10, 16))
    assert abs(np.sum(W.magic_filter(x) * y) - np.sum(x * W.magic_filter_t(y))) < 1e-12


def test_density_and_energy_identities():
    case = inputs.random_case(7, 3, (6, 5, 4), potential="gauss16")
    C, V, occ = case["C"], case["V"], case["occ"]
    r = W.local_hpsi(C, V, occ)
    psis = [W.point_values(c) for c in C]
    assert abs(r["rho"].sum() - sum(f * np.sum(p * p) for f, p in zip(occ, psis))) < 1e-12
    assert np.max(np.abs(W.local_density(C, occ) - r["rho"])) < 1e-14
    assert abs(r["e_loc"] - float(np.dot(occ, r["e_loc_orb"]))) < 1e-12
    for i in range(len(C)):
        chc = float(np.sum(C[i] * r["hpsi"][i]))
        assert abs(chc - (r["e_loc_orb"][i] + r["e_kin_orb"][i])) < 1e-12
        assert r["e_kin_orb"][i] > 0


def test_central_differences_are_exact_for_quadratic_energy():
    case = inputs.random_case(9, 2, (4, 5, 6), potential="gauss16")
    C, V, occ = case["C"], case["V"], case["occ"]
    rho, dC = W.energy_gradients(C, V, occ)
    dV = inputs.directions(21, V.shape, 1)[0]
    dc = np.stack(inputs.directions(22, C.shape[1:], 2))
    eps = 1e-3
    def E(Cx, Vx):
        a, b = W.energies(Cx, Vx, occ)
        return a + b
    # E is linear in V and quadratic in c: central differences along V alone or
    # along c alone have no truncation error (a joint step would leave the
    # cubic cross term eps^2 <dc, V' dc>)
    fdV = (E(C, V + eps * dV) - E(C, V - eps * dV)) / (2 * eps)
    fdc = (E(C + eps * dc, V) - E(C - eps * dc, V)) / (2 * eps)
    assert abs(fdV - float(np.sum(rho * dV))) < 1e-11
    an = float(np.sum(dC * dc))
    assert abs(fdc - an) < 1e-11 * max(1.0, abs(an))


def test_cholesky_orthonormalisation():
    case = inputs.random_case(4, 6, (4, 4, 4))
    C = case["C"] + 0.3 * case["C"][0]     # strongly non-orthogonal
    Cn, L = W.cholesky_orthonormalize(C)
    X = Cn.reshape(len(C), -1)
    assert np.max(np.abs(X @ X.T - np.eye(len(C)))) < 1e-13
    assert np.allclose(L, np.tril(L)) and np.all(np.diag(L) > 0)
    S = W.overlap(C)
    assert np.max(np.abs(L @ L.T - S)) < 1e-13
    # Gram-Schmidt order: the first new orbital is the first old one, scaled
    x0 = C[0].ravel()
    assert np.max(np.abs(X[0] - x0 / np.linalg.norm(x0))) < 1e-14
