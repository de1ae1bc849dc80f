"""Oracle-side derivation of the filters of the method (TEST INFRASTRUCTURE).

This module belongs to the oracle: only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it.  The GPU library derives its
own filters with separate code and shares nothing with this file.

Everything is computed from the mathematics in mpmath at 60 significant
digits and rounded to float64 at the end:

* ``h``, ``g``  -- the order-16 Daubechies two-scale filters of the refinement
  relations (Sec. 2.1, Eq. "refinement"): phi(x) = sqrt2 sum_j h_j phi(2x-j),
  psi(x) = sqrt2 sum_j g_j phi(2x-j), g_j = (-1)^j h_{1-j}, taps j = -7..8.
  The paper does not say which of the spectral factors of the Daubechies
  polynomial is used; we take the least-asymmetric one (the symlet), in the
  orientation whose first moment int x phi is 0.1604... (not its mirror).
* ``M``         -- moments M_k = int x^k phi(x) dx from the refinement relation.
* ``omega``     -- the magic filter (Sec. 2.3, Eq. "magicfilter"): the 16-tap
  filter on l = -7..8 whose moments reproduce those of phi,
  sum_l omega_l l^k = M_k for k = 0..15, which makes the point values exact for
  polynomials of degree <= 15 (the O(h^16) statement of Sec. 2.3).
* ``r``         -- the kinetic filter (Sec. 2.2, Eqs. "kiner", "fprod"):
  r_l = Phi''(l) with Phi the autocorrelation of phi, l = -14..14.  The 1D
  kinetic operator on a grid of spacing h is t_l = -r_l / (2 h^2).

The derivation is generic in the order N (number of vanishing moments) so that
it can be pinned against the closed forms of the order-4 (N = 2) filter.
"""

import functools

import mpmath as mp
import numpy as np

DPS = 60


def _with_dps(fn):
    @functools.wraps(fn)
    def wrapped(*a, **k):
        with mp.workdps(DPS):
            return fn(*a, **k)
    return wrapped


@_with_dps
def daubechies_y_roots(N):
    """Roots in y of P(y) = sum_{k<N} C(N-1+k, k) y^k (|m0|^2 = cos^2N P(sin^2))."""
    coeffs_desc = [mp.binomial(N - 1 + k, k) for k in range(N - 1, -1, -1)]
    if N == 1:
        return []
    roots = mp.polyroots(coeffs_desc, maxsteps=2000, extraprec=4 * DPS)
    # polish each root with Newton steps at the full working precision
    dcoeffs = [c * (len(coeffs_desc) - 1 - i) for i, c in enumerate(coeffs_desc[:-1])]
    out = []
    for y in roots:
        y = mp.mpc(y)
        for _ in range(20):
            y = y - mp.polyval(coeffs_desc, y) / mp.polyval(dcoeffs, y)
        out.append(y)
    return out


@_with_dps
def spectral_factors(N):
    """All real spectral factors m0 of the Daubechies polynomial of order N.

    Each root y of P gives two reciprocal roots z, 1/z of
    z^2 - (2 - 4y) z + 1 = 0.  Picking one of the two for every real root and
    for every conjugate pair (the conjugate root takes the conjugate choice)
    gives 2^(#real + #pairs) real filters.  Returns a list of coefficient
    lists (mpf), h_p for p = 0..2N-1, with sum h = sqrt2.
    """
    ys = daubechies_y_roots(N)
    groups = []  # each group: list of y roots handled together
    used = [False] * len(ys)
    for i, y in enumerate(ys):
        if used[i]:
            continue
        used[i] = True
        if abs(mp.im(y)) < mp.mpf(10) ** (-40):
            groups.append([mp.re(y)])
        else:
            # find its conjugate
            best = None
            for j in range(len(ys)):
                if not used[j] and abs(ys[j] - mp.conj(y)) < mp.mpf(10) ** (-30):
                    best = j
                    break
            assert best is not None, "unpaired complex root"
            used[best] = True
            yy = y if mp.im(y) > 0 else ys[best]
            groups.append([yy, mp.conj(yy)])
    out = []
    for bits in range(2 ** len(groups)):
        zs = []
        for gi, grp in enumerate(groups):
            pick = (bits >> gi) & 1
            for y in grp:
                b = 2 - 4 * y
                disc = mp.sqrt(b * b - 4)
                z1 = (b + disc) / 2
                z2 = (b - disc) / 2
                # choose the root inside / outside the unit circle consistently
                zin, zout = (z1, z2) if abs(z1) < abs(z2) else (z2, z1)
                if abs(abs(z1) - 1) < mp.mpf(10) ** (-30):
                    # root on the unit circle (does not happen for these P)
                    zin, zout = z1, z2
                zs.append(zin if pick == 0 else zout)
        # m0(z) = ((1+z)/2)^N prod (z - zk)/(1 - zk), a polynomial in z
        poly = [mp.mpc(1)]  # ascending coefficients
        def mul(p, q):
            r = [mp.mpc(0)] * (len(p) + len(q) - 1)
            for i, a in enumerate(p):
                for j, b in enumerate(q):
                    r[i + j] += a * b
            return r
        for _ in range(N):
            poly = mul(poly, [mp.mpf(1) / 2, mp.mpf(1) / 2])
        for zk in zs:
            poly = mul(poly, [-zk / (1 - zk), 1 / (1 - zk)])
        h = [mp.sqrt(2) * mp.re(c) for c in poly]
        out.append((h, zs))
    return out


def _phase_nonlinearity(zs):
    """Max deviation of the unwrapped phase of m0(e^{-i xi}) from its
    least-squares straight-line fit on the open interval (0, pi).

    The factor ((1+z)/2)^N of m0 only adds the linear phase -N xi/2 and
    vanishes to order N at xi = pi, so the phase is taken from the remaining
    factors prod (z - z_k)/(1 - z_k), which have no zero on the unit circle."""
    xi = np.linspace(0.0, np.pi, 2001)[1:-1]
    z = np.exp(-1j * xi)
    ph = np.zeros_like(xi)
    for zk in zs:
        zk = complex(zk)
        ph += np.unwrap(np.angle((z - zk) / (1 - zk)))
    A = np.stack([np.ones_like(xi), xi], axis=1)
    coef, *_ = np.linalg.lstsq(A, ph, rcond=None)
    return float(np.max(np.abs(ph - A @ coef)))


@_with_dps
def moments_from_filter(h, lo, K):
    """M_k = int x^k phi(x) dx, k = 0..K, for phi(x) = sqrt2 sum_j h_j phi(2x - j)
    with h_j indexed j = lo .. lo+len(h)-1.

    Substituting u = 2x - j in the refinement relation gives
    M_k (1 - 2^-k) = 2^-k / sqrt2 * sum_{l<k} C(k,l) mu_{k-l} M_l,
    mu_p = sum_j h_j j^p, with M_0 = 1 (unit integral)."""
    js = [lo + i for i in range(len(h))]
    mu = [mp.fsum(hj * mp.mpf(j) ** p for hj, j in zip(h, js)) for p in range(K + 1)]
    M = [mp.mpf(1)]
    for k in range(1, K + 1):
        s = mp.fsum(mp.binomial(k, l) * mu[k - l] * M[l] for l in range(k))
        M.append((mp.mpf(2) ** (-k) / mp.sqrt(2)) * s / (1 - mp.mpf(2) ** (-k)))
    return M


@_with_dps
def least_asymmetric(N):
    """The least-asymmetric spectral factor of order N, oriented so that its
    first moment (taps indexed from 1-N) lies below 1/2.  Returns (h, lo)."""
    cands = spectral_factors(N)
    scores = [_phase_nonlinearity(zs) for _, zs in cands]
    best = min(scores)
    # the winner and its mirror image tie; keep every candidate within 1e-9
    winners = [h for (h, _), s in zip(cands, scores) if s - best < 1e-9]
    lo = 1 - N
    for h in winners:
        M1 = moments_from_filter(h, lo, 1)[1]
        if M1 < mp.mpf(1) / 2:
            return h, lo
    # only one winner found: mirror it
    h = list(reversed(winners[0]))
    return h, lo


@_with_dps
def wavelet_filter(h, lo):
    """g_j = (-1)^j h_{1-j} on the same index window as h (window symmetric
    about 1/2, so 1-j stays inside it)."""
    n = len(h)
    hi = lo + n - 1
    assert lo + hi == 1
    g = []
    for j in range(lo, hi + 1):
        g.append((-1) ** (j % 2) * h[(1 - j) - lo])
    return g


@_with_dps
def magic_filter(M, lo, n):
    """omega_l, l = lo .. lo+n-1: the solution of sum_l omega_l l^k = M_k for
    k = 0..n-1 (a Vandermonde system, solved at 60 digits since it is badly
    conditioned in double precision)."""
    ls = [lo + i for i in range(n)]
    A = mp.matrix(n, n)
    b = mp.matrix(n, 1)
    for k in range(n):
        for i, l in enumerate(ls):
            A[k, i] = mp.mpf(l) ** k
        b[k] = M[k]
    x = mp.lu_solve(A, b)
    return [x[i] for i in range(n)]


@_with_dps
def kinetic_filter(h, lo):
    """r_l = Phi''(l), l = -L..L with L = len(h) - 2, Phi(x) = int phi(y) phi(y-x) dy.

    Phi obeys Phi(x) = sum_k c_k Phi(2x - k), c_k = sum_i h_i h_{i+k}; two
    derivatives at the integers give r_l = 4 sum_k c_k r_{2l-k}.  The null
    vector of (4C - I) is fixed by sum_l l^2 r_l = 2 (second derivative of x^2)."""
    n = len(h)
    L = n - 2
    def c(k):
        s = mp.mpf(0)
        for i in range(n):
            j = i + k
            if 0 <= j < n:
                s += h[i] * h[j]
        return s
    idx = list(range(-L, L + 1))
    size = len(idx)
    # the (singular, consistent) eigen-equations plus the normalisation row,
    # solved in the least-squares sense (exact, since the system is consistent)
    A = mp.matrix(size + 1, size)
    b = mp.matrix(size + 1, 1)
    for a, l in enumerate(idx):
        for bcol, q in enumerate(idx):
            A[a, bcol] = 4 * c(2 * l - q) - (1 if a == bcol else 0)
    for bcol, q in enumerate(idx):
        A[size, bcol] = mp.mpf(q) ** 2
    b[size] = 2
    x, res = mp.qr_solve(A, b)
    return [x[i] for i in range(size)], -L


@functools.lru_cache(maxsize=None)
def filters_mp(N=8):
    """All filters of order N as mpf lists, with their first indices."""
    with mp.workdps(DPS):
        h, lo = least_asymmetric(N)
        g = wavelet_filter(h, lo)
        M = moments_from_filter(h, lo, 2 * N + 4)
        om = magic_filter(M, lo, 2 * N)
        r, rlo = kinetic_filter(h, lo)
        return dict(h=h, g=g, lo=lo, M=M, omega=om, omega_lo=lo, r=r, r_lo=rlo)


@functools.lru_cache(maxsize=None)
def filters(N=8):
    """float64 copies of :func:`filters_mp` (numpy arrays, read-only)."""
    f = filters_mp(N)
    def arr(v):
        a = np.array([float(x) for x in v], dtype=np.float64)
        a.setflags(write=False)
        return a
    return dict(h=arr(f["h"]), g=arr(f["g"]), lo=f["lo"], M=arr(f["M"]),
                omega=arr(f["omega"]), omega_lo=f["omega_lo"],
                r=arr(f["r"]), r_lo=f["r_lo"])
