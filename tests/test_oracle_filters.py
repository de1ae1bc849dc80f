"""Pins of the oracle's filters against mathematics, not against themselves.

* closed forms: the order-4 filter (N = 2) of the same derivation;
* invariants of the two-scale relations (Sec. 2.1, Eq. "refinement");
* moments by an independent route: phi tabulated on a dyadic grid by the
  cascade of the refinement relation, then integrated numerically;
* the magic filter (Sec. 2.3) checked on that tabulated phi (point values of
  polynomials) and in the Fourier domain (infinite product for phi-hat);
* the kinetic filter (Sec. 2.2) checked against the Fourier integral
  r_l = -(1/pi) int_0^inf xi^2 |phi-hat(xi)|^2 cos(l xi) dxi, where
  |phi-hat|^2 is the infinite product of cos^2N(xi/2) P(sin^2(xi/2)): a closed
  form that involves neither the spectral factorisation nor the eigenproblem.
"""

import math

import mpmath as mp
import numpy as np
import pytest

from oracle import filters as OF


@pytest.fixture(scope="module")
def F():
    return OF.filters(8)


@pytest.fixture(scope="module")
def Fmp():
    return OF.filters_mp(8)


# ---------------------------------------------------------------- helpers

def cascade_phi(h, lo, J):
    """phi on the dyadic grid x = k / 2^J, by the refinement relation
    phi(x) = sqrt2 sum_j h_j phi(2x - j).  Values at the integers are the
    eigenvector (eigenvalue 1) of A[k, q] = sqrt2 h_{2k - q}, normalised to
    sum 1.  Returns (x, phi(x))."""
    h = np.asarray(h, dtype=np.float64)
    n = len(h)
    a, b = lo, lo + n - 1          # support [a, b]
    ks = np.arange(a, b + 1)
    A = np.zeros((len(ks), len(ks)))
    for i, k in enumerate(ks):
        for t, q in enumerate(ks):
            j = 2 * k - q
            if a <= j <= b:
                A[i, t] = math.sqrt(2.0) * h[j - a]
    w, V = np.linalg.eig(A)
    i1 = np.argmin(np.abs(w - 1.0))
    v = np.real(V[:, i1])
    v = v / v.sum()
    cur = v
    for lev in range(1, J + 1):
        # x = a + i / 2^lev and 2x - (a + jj) = a + (i - jj 2^(lev-1)) / 2^(lev-1)
        npts = (b - a) * 2 ** lev + 1
        step = 2 ** (lev - 1)
        nxt = np.zeros(npts)
        for jj in range(n):
            off = jj * step
            lo_i, hi_i = off, min(npts, off + len(cur))
            nxt[lo_i:hi_i] += h[jj] * cur[: hi_i - lo_i]
        cur = math.sqrt(2.0) * nxt
    x = a + np.arange(len(cur)) / 2.0 ** J
    return x, cur


def phi_hat_plus(h, lo, xi, terms=70):
    """int phi(u) e^{i xi u} du = prod_{j>=1} m0(xi / 2^j),
    m0(t) = (1/sqrt2) sum_j h_j e^{i t j}, in mpmath."""
    p = mp.mpc(1)
    for k in range(1, terms + 1):
        t = xi / mp.mpf(2) ** k
        p *= mp.fsum(hj * mp.expj(t * (lo + i)) for i, hj in enumerate(h)) / mp.sqrt(2)
    return p


# ---------------------------------------------------------------- closed forms

def test_order4_filter_closed_form():
    """N = 2: the factor is (1+s3, 3+s3, 3-s3, 1-s3)/(4 sqrt2), s3 = sqrt3,
    on taps -1..2 in the orientation with first moment below 1/2."""
    with mp.workdps(40):
        h, lo = OF.least_asymmetric(2)
        s3 = mp.sqrt(3)
        ref = [(1 + s3), (3 + s3), (3 - s3), (1 - s3)]
        ref = [v / (4 * mp.sqrt(2)) for v in ref]
        assert lo == -1
        assert max(abs(a - b) for a, b in zip(h, ref)) < mp.mpf(10) ** -35
        # first moment of the order-4 phi, (3 - sqrt3)/2 on taps 0..3, shifted by -1
        M = OF.moments_from_filter(h, lo, 2)
        assert abs(M[1] - ((3 - s3) / 2 - 1)) < mp.mpf(10) ** -35


def test_haar_special_case():
    """N = 1 is the Haar filter (1, 1)/sqrt2 on taps 0..1."""
    with mp.workdps(40):
        fs = OF.spectral_factors(1)
        assert len(fs) == 1
        h, _ = fs[0]
        assert all(abs(v - 1 / mp.sqrt(2)) < mp.mpf(10) ** -35 for v in h)


# ---------------------------------------------------------------- invariants of h, g

def test_h_orthonormal_and_sums(Fmp):
    h = Fmp["h"]
    with mp.workdps(60):
        for k in range(8):
            s = mp.fsum(h[i] * h[i + 2 * k] for i in range(16 - 2 * k))
            assert abs(s - (1 if k == 0 else 0)) < mp.mpf(10) ** -50
        assert abs(mp.fsum(h) - mp.sqrt(2)) < mp.mpf(10) ** -50
        ev = mp.fsum(h[i] for i in range(0, 16, 2))
        od = mp.fsum(h[i] for i in range(1, 16, 2))
        assert abs(ev - 1 / mp.sqrt(2)) < mp.mpf(10) ** -50
        assert abs(od - 1 / mp.sqrt(2)) < mp.mpf(10) ** -50


def test_g_vanishing_moments_and_orthogonality(Fmp):
    h, g, lo = Fmp["h"], Fmp["g"], Fmp["lo"]
    with mp.workdps(60):
        for p in range(8):
            s = mp.fsum(gj * mp.mpf(lo + i) ** p for i, gj in enumerate(g))
            assert abs(s) < mp.mpf(10) ** -40
        # the 8th moment does not vanish (exactly 8 vanishing moments)
        s8 = mp.fsum(gj * mp.mpf(lo + i) ** 8 for i, gj in enumerate(g))
        assert abs(s8) > 1e-3
        for k in range(-7, 8):
            s = mp.fsum(h[i] * g[i + 2 * k] for i in range(16) if 0 <= i + 2 * k < 16)
            assert abs(s) < mp.mpf(10) ** -50


def test_least_asymmetric_selection(Fmp):
    """The chosen factor minimises the phase non-linearity among all 16
    factors (two mirror images tie), and the kept orientation has M1 < 1/2."""
    cands = OF.spectral_factors(8)
    assert len(cands) == 16
    scores = sorted(OF._phase_nonlinearity(zs) for _, zs in cands)
    assert abs(scores[0] - scores[1]) < 1e-9 and scores[2] - scores[0] > 0.05
    assert 0.0 < float(Fmp["M"][1]) < 0.5


# ---------------------------------------------------------------- moments, magic filter

@pytest.fixture(scope="module")
def tab_phi(F):
    return cascade_phi(F["h"], F["lo"], 11)


def test_moments_against_tabulated_phi(F, tab_phi):
    x, ph = tab_phi
    dx = x[1] - x[0]
    assert abs(ph.sum() * dx - 1.0) < 1e-12
    for p in range(1, 6):
        num = float(np.sum(ph * x ** p) * dx)
        assert abs(num - F["M"][p]) < 1e-9 * max(1.0, abs(F["M"][p])), p


def test_M2_equals_M1_squared(Fmp):
    with mp.workdps(60):
        assert abs(Fmp["M"][2] - Fmp["M"][1] ** 2) < mp.mpf(10) ** -50


def test_magic_filter_sums_and_moments(F, Fmp):
    assert abs(F["omega"].sum() - 1.0) < 1e-15
    with mp.workdps(60):
        for k in range(16):
            s = mp.fsum(w * mp.mpf(Fmp["omega_lo"] + i) ** k for i, w in enumerate(Fmp["omega"]))
            assert abs(s - Fmp["M"][k]) < mp.mpf(10) ** -40 * max(1, abs(Fmp["M"][k]))


def test_magic_filter_point_values_of_polynomials(F, tab_phi):
    """s_j = <phi(. - j), x^p> from the tabulated phi; the magic filter must
    return the point values i^p (exact for degree <= 15)."""
    x, ph = tab_phi
    dx = x[1] - x[0]
    om, olo = F["omega"], F["omega_lo"]
    i0 = 5
    for p in range(0, 6):
        def s(j):
            return float(np.sum(ph * (x + j) ** p) * dx)
        val = sum(om[k] * s(i0 - (olo + k)) for k in range(16))
        assert abs(val - i0 ** p) < 1e-8 * max(1, i0 ** p), p


def test_magic_filter_fourier_order(Fmp):
    """omega-hat(xi) phi-hat(xi) = 1 + O(xi^16) (point values exact to
    order 16): halving xi divides the defect by about 2^16."""
    with mp.workdps(50):
        h, lo, om, olo = Fmp["h"], Fmp["lo"], Fmp["omega"], Fmp["omega_lo"]
        def defect(xi):
            oh = mp.fsum(w * mp.expj(-xi * (olo + i)) for i, w in enumerate(om))
            return abs(oh * phi_hat_plus(h, lo, xi) - 1)
        d1, d2 = defect(mp.mpf("0.8")), defect(mp.mpf("0.4"))
        ratio = d1 / d2
        assert 2 ** 15 < ratio < 2 ** 17, float(ratio)
        assert d2 < 1e-8


# ---------------------------------------------------------------- kinetic filter

def test_kinetic_filter_invariants(F, Fmp):
    r = F["r"]
    assert np.allclose(r, r[::-1], atol=0, rtol=0) or np.max(np.abs(r - r[::-1])) < 1e-15
    assert abs(r.sum()) < 1e-14
    ls = np.arange(-14, 15)
    assert abs(np.sum(ls ** 2 * r) - 2.0) < 1e-13
    with mp.workdps(60):
        rr, L = Fmp["r"], 14
        for k in range(2, 8):
            s = mp.fsum(v * mp.mpf(l) ** (2 * k) for v, l in zip(rr, range(-L, L + 1)))
            assert abs(s) < mp.mpf(10) ** -35 * 10 ** (2 * k)
        s16 = mp.fsum(v * mp.mpf(l) ** 16 for v, l in zip(rr, range(-L, L + 1)))
        assert abs(s16) > 1e-6


def test_kinetic_filter_fourier_integral(F):
    """r_l = Phi''(l) = -(1/pi) int_0^inf xi^2 |phi-hat|^2 cos(l xi) dxi with
    |phi-hat(xi)|^2 = prod_j cos^16(xi/2^(j+1)) P(sin^2(xi/2^(j+1)))."""
    N = 8
    Pc = np.array([math.comb(N - 1 + k, k) for k in range(N)], dtype=np.float64)
    xmax, n = 1600.0, 1_600_001
    xi = np.linspace(0.0, xmax, n)
    mod2 = np.ones_like(xi)
    for j in range(1, 60):
        t = xi / 2.0 ** j
        y = np.sin(t / 2.0) ** 2
        P = np.polyval(Pc[::-1], y)
        mod2 *= np.cos(t / 2.0) ** (2 * N) * P
    w = xi ** 2 * mod2
    dxi = xi[1] - xi[0]
    for l in range(0, 6):
        f = w * np.cos(l * xi)
        integ = dxi * (f.sum() - 0.5 * (f[0] + f[-1]))
        rl = -integ / math.pi
        assert abs(rl - F["r"][14 + l]) < 2e-6, (l, rl, F["r"][14 + l])


# ---------------------------------------------------------------- anchor values

# Values of the least-asymmetric order-16 factor (Daubechies, Ten Lectures on
# Wavelets, 1992, ch. 6 and 8), of its first moment and of the magic and
# kinetic filters derived from it, computed separately at 60 digits by another
# route (roots in z, phase fit of m0 on (0, pi)).  They fix the choice of the
# spectral factor and of its orientation, which the invariants above leave open
# between mirror images and other factors with 0 < M1 < 1/2.
ANCHOR_H = {-7: -0.0033824159510050025955, -6: -0.00054213233180001068935,
            -5: 0.031695087811525991431, -4: 0.0076074873249766081919,
            -3: -0.14329423835127266284, -2: -0.061273359067811077843,
            -1: 0.48135965125905339159, 0: 0.77718575169962802862,
            1: 0.36444189483617893676, 2: -0.051945838107881800736,
            3: -0.027219029917103486322, 4: 0.049137179673730286787,
            5: 0.0038087520138944894631, 6: -0.014952258337062199118,
            7: -0.00030292051472413308126, 8: 0.0018899503327676891843}
ANCHOR_M1 = 0.16041800328247180267
ANCHOR_OMEGA = {0: 0.99404156978340039932, -1: -0.0604895289196983516,
                1: 0.06126258958312079822, -7: 2.7273449291197965966e-6,
                8: 8.4334247333529341095e-7}
ANCHOR_R = {0: -3.5536922899131901941, 1: 2.2191465938911163899,
            2: -0.61561414655700694963, 13: 2.7080049362631943827e-13}


def test_anchor_values(F):
    for j, v in ANCHOR_H.items():
        assert abs(F["h"][j - F["lo"]] - v) < 1e-15, j
    assert abs(F["M"][1] - ANCHOR_M1) < 1e-15
    for l, v in ANCHOR_OMEGA.items():
        assert abs(F["omega"][l - F["omega_lo"]] - v) < 1e-15, l
    for l, v in ANCHOR_R.items():
        assert abs(F["r"][l - F["r_lo"]] - v) < 1e-14 * max(1.0, abs(v)), l
        assert abs(F["r"][-l - F["r_lo"]] - v) < 1e-14 * max(1.0, abs(v)), -l
    assert abs(float(np.sum(F["omega"] ** 2)) - 0.9968193186) < 1e-10
