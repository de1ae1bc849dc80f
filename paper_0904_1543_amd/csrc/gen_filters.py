#!/usr/bin/env python3
"""Build step: derive the filters of the method and write ``filters_gen.h``.

The library's own derivation (written separately from any test code), in
mpmath at 64 significant digits, emitted as exact hexadecimal float64
literals plus the float32 hi/lo splits used by the compensated form.

  * h, g   order-16 Daubechies two-scale filters (Sec. 2.1, Eq. "refinement"),
           g_j = (-1)^j h_{1-j}, taps j = -7..8.  Spectral factor: the
           least-asymmetric one.  The 14 non-trivial zeros of |m0|^2 are found
           in the z plane as the roots of z^7 P((2 - z - 1/z)/4); one zero of
           every reciprocal pair (conjugates together) is kept, and the choice
           with the flattest phase (smallest deviation from a straight line on
           (0, pi)) wins; of the two mirror images the one with the first
           moment int x phi below 1/2 is kept.
  * omega  magic filter (Sec. 2.3): the quadrature weights on the nodes -7..8
           that integrate polynomials of degree <= 15 against phi, i.e.
           omega_l = int phi(x) L_l(x) dx with L_l the Lagrange basis
           polynomial of node l (exact rational coefficients) and the moments
           of phi from the refinement relation (a triangular linear system).
  * r      kinetic filter (Sec. 2.2): r_l = Phi''(l), Phi the autocorrelation
           of phi; the eigenvector of r = 4 sum_k a_k r_{2l-k}
           (a_k = sum_i h_i h_{i+k}) found by inverse iteration and scaled so
           that sum_l l^2 r_l = 2.

Usage: python gen_filters.py [output_header]
"""

import os
import sys
from fractions import Fraction

import mpmath as mp
import numpy as np

mp.mp.dps = 64
NVM = 8                # vanishing moments; 2*NVM taps
LO = 1 - NVM           # first tap index (-7)


def z_roots():
    """Roots of Q(z) = z^(N-1) P(y), y = (2 - z - 1/z)/4 = -(z-1)^2/(4z),
    P(y) = sum_k C(N-1+k, k) y^k.  Q has degree 2N-2."""
    N = NVM
    deg = 2 * N - 2
    Q = [mp.mpf(0)] * (deg + 1)        # ascending powers of z
    for k in range(N):
        a = mp.binomial(N - 1 + k, k) * (mp.mpf(-1) / 4) ** k
        # (z-1)^(2k) z^(N-1-k)
        for t in range(2 * k + 1):
            coef = mp.binomial(2 * k, t) * (-1) ** (2 * k - t)
            Q[t + N - 1 - k] += a * coef
    desc = list(reversed(Q))
    rts = mp.polyroots(desc, maxsteps=4000, extraprec=300)
    dQ = [c * (deg - i) for i, c in enumerate(desc[:-1])]
    out = []
    for z in rts:
        z = mp.mpc(z)
        for _ in range(30):
            z -= mp.polyval(desc, z) / mp.polyval(dQ, z)
        out.append(z)
    return out


def candidates():
    rts = z_roots()
    inside = [z for z in rts if abs(z) < 1]
    assert len(inside) == NVM - 1
    # group conjugates
    reals = [z for z in inside if abs(mp.im(z)) < mp.mpf(10) ** -40]
    upper = [z for z in inside if mp.im(z) >= mp.mpf(10) ** -40]
    groups = [[mp.re(z)] for z in reals] + [[z, mp.conj(z)] for z in upper]
    res = []
    for mask in range(1 << len(groups)):
        zs = []
        for gi, grp in enumerate(groups):
            for z in grp:
                zs.append(z if not (mask >> gi) & 1 else 1 / z)
        # m0(z) proportional to (1 + z)^N prod (z - zk), normalised m0(1) = 1
        coeffs = [mp.mpc(1)]
        for root in [mp.mpf(-1)] * NVM + zs:
            nxt = [mp.mpc(0)] * (len(coeffs) + 1)
            for i, c in enumerate(coeffs):
                nxt[i + 1] += c
                nxt[i] -= root * c
            coeffs = nxt
        norm = mp.fsum(coeffs)
        h = [mp.sqrt(2) * mp.re(c / norm) for c in coeffs]
        res.append((h, zs))
    return res


def phase_deviation(zs):
    xi = np.linspace(0.0, np.pi, 4097)[1:-1]
    e = np.exp(-1j * xi)
    total = np.zeros_like(xi)
    for zk in zs:
        total += np.unwrap(np.angle(e - complex(zk)))
    fit = np.polyfit(xi, total, 1)
    return float(np.max(np.abs(total - np.polyval(fit, xi))))


def moments(h, K):
    """Moments of phi: M_k = 2^(-k) / sqrt2 * sum_l C(k,l) mu_{k-l} M_l with
    mu_p = sum_j h_j j^p, assembled as one lower-triangular system."""
    mu = [mp.fsum(hj * mp.mpf(LO + i) ** p for i, hj in enumerate(h)) for p in range(K + 1)]
    A = mp.matrix(K + 1, K + 1)
    b = mp.matrix(K + 1, 1)
    A[0, 0] = 1
    b[0] = 1
    for k in range(1, K + 1):
        fac = mp.mpf(2) ** (-k) / mp.sqrt(2)
        for l in range(k + 1):
            A[k, l] -= fac * mp.binomial(k, l) * mu[k - l]
        A[k, k] += 1
    m = mp.lu_solve(A, b)
    return [m[i] for i in range(K + 1)]


def select():
    cands = candidates()
    devs = [phase_deviation(zs) for _, zs in cands]
    best = min(devs)
    for (h, _), d in zip(cands, devs):
        if d - best < 1e-9 and moments(h, 1)[1] < mp.mpf("0.5"):
            return h
    raise RuntimeError("no least-asymmetric factor with first moment below 1/2")


def lagrange_weights(M, nodes):
    """omega_l = sum_k [x^k] L_l(x) * M_k, L_l the Lagrange basis polynomial."""
    out = []
    for l in nodes:
        poly = [Fraction(1)]
        den = Fraction(1)
        for q in nodes:
            if q == l:
                continue
            nxt = [Fraction(0)] * (len(poly) + 1)
            for i, c in enumerate(poly):
                nxt[i + 1] += c
                nxt[i] -= q * c
            poly = nxt
            den *= (l - q)
        w = mp.fsum(mp.mpf(c.numerator) / mp.mpf(c.denominator) * M[k] for k, c in enumerate(poly))
        out.append(w / den)
    return out


def kinetic(h):
    n = len(h)
    L = n - 2
    a = {}
    for k in range(-(n - 1), n):
        a[k] = mp.fsum(h[i] * h[i + k] for i in range(n) if 0 <= i + k < n)
    idx = range(-L, L + 1)
    size = 2 * L + 1
    B = mp.matrix(size, size)
    for i, l in enumerate(idx):
        for j, q in enumerate(idx):
            B[i, j] = 4 * a.get(2 * l - q, mp.mpf(0))
    shift = 1 + mp.mpf(10) ** -30
    Bs = B - shift * mp.eye(size)
    v = mp.matrix([[1] for _ in range(size)])
    for _ in range(4):
        v = mp.lu_solve(Bs, v)
        v = v / mp.norm(v)
    s2 = mp.fsum(v[i] * (i - L) ** 2 for i in range(size))
    return [v[i] * 2 / s2 for i in range(size)]


# ---------------------------------------------------------------------------
# Polyphase form of the 1D operators: y[k] = sum_o F_{k mod 2}(o) x[k - o].
# Returned as (lo, [row_p0, row_p1]) with rows indexed by o - lo.
# ---------------------------------------------------------------------------
def poly(table_fn, lo, hi):
    return lo, [[table_fn(p, o) for o in range(lo, hi + 1)] for p in (0, 1)]


def base_polyphase(h, g, om, r):
    zero = mp.mpf(0)
    def tap(arr, j):
        return arr[j - LO] if LO <= j < LO + 2 * NVM else zero
    L = len(r) // 2
    mf = poly(lambda p, o: tap(om, o), -7, 8)
    mft = poly(lambda p, o: tap(om, -o), -8, 7)
    syn = poly(lambda p, o: tap(h, o) if (o - p) % 2 == 0 else tap(g, o + 1), -8, 8)
    ana = poly(lambda p, o: tap(h, -o) if p == 0 else tap(g, 1 - o), -8, 8)
    kin = poly(lambda p, o: r[o + L], -L, L)
    return dict(mf=mf, mft=mft, syn=syn, ana=ana, kin=kin)


def compose(B, A):
    """Polyphase table of the operator B(A(x)):
    C_p(o) = sum_{o2 + o1 = o} B_p(o2) A_{(p - o2) mod 2}(o1)."""
    blo, brow = B
    alo, arow = A
    bhi, ahi = blo + len(brow[0]) - 1, alo + len(arow[0]) - 1
    lo, hi = blo + alo, bhi + ahi
    out = [[mp.mpf(0)] * (hi - lo + 1) for _ in (0, 1)]
    for p in (0, 1):
        for o2 in range(blo, bhi + 1):
            b = brow[p][o2 - blo]
            if b == 0:
                continue
            pa = (p - o2) % 2
            for o1 in range(alo, ahi + 1):
                out[p][o2 + o1 - lo] += b * arow[pa][o1 - alo]
    # trim zero columns at both ends
    while all(out[p][0] == 0 for p in (0, 1)):
        out = [row[1:] for row in out]
        lo += 1
    while all(out[p][-1] == 0 for p in (0, 1)):
        out = [row[:-1] for row in out]
    return lo, out


def split32(x):
    hi = np.float32(float(x))
    lo = np.float32(float(x - mp.mpf(float(hi))))
    return hi, lo


def emit(path):
    h = select()
    g = [(-1) ** ((LO + i) % 2) * h[(1 - (LO + i)) - LO] for i in range(2 * NVM)]
    M = moments(h, 2 * NVM)
    om = lagrange_weights(M, list(range(LO, LO + 2 * NVM)))
    r = kinetic(h)

    def dbl(name, vals):
        body = ",\n    ".join(float(v).hex() for v in vals)
        return f"static constexpr double {name}[{len(vals)}] = {{\n    {body}}};\n"

    def flt(name, vals):
        his, los = zip(*(split32(v) for v in vals))
        def lit(x):
            return float(x).hex() + "f" if float(x) != 0.0 else "0.0f"
        out = f"static constexpr float {name}_HI[{len(vals)}] = {{\n    " + \
            ",\n    ".join(lit(x) for x in his) + "};\n"
        out += f"static constexpr float {name}_LO[{len(vals)}] = {{\n    " + \
            ",\n    ".join(lit(x) for x in los) + "};\n"
        return out

    text = ["// Generated by gen_filters.py (filters of the method, derived from",
            "// the mathematics in 64-digit arithmetic).  Do not edit.",
            "#pragma once", "",
            f"#define WVL_NTAP {2 * NVM}",
            f"#define WVL_TAP_LO ({LO})",
            f"#define WVL_KIN_HALF {2 * NVM - 2}", ""]
    text.append("// h_j, j = -7..8 (scaling two-scale filter)")
    text.append(dbl("WVL_H", h))
    text.append("// g_j = (-1)^j h_{1-j}, j = -7..8 (wavelet two-scale filter)")
    text.append(dbl("WVL_G", g))
    text.append("// omega_l, l = -7..8 (magic filter)")
    text.append(dbl("WVL_OMEGA", om))
    text.append("// r_l = Phi''(l), l = -14..14 (kinetic filter before -1/(2 h^2))")
    text.append(dbl("WVL_KIN", r))
    P = base_polyphase(h, g, om, r)
    combos = {
        # synthesis then magic filter: coarse coefficients -> point values
        "WVL_CW": compose(P["mf"], P["syn"]),
        # transposed magic filter then analysis: point values -> coarse coefficients
        "WVL_CWT": compose(P["ana"], P["mft"]),
        # analysis o kinetic o synthesis: the kinetic filter on coarse coefficients
        "WVL_CK": compose(P["ana"], compose(P["kin"], P["syn"])),
    }
    for name, (lo, rows) in combos.items():
        n = len(rows[0])
        text.append(f"// combined polyphase filter: y[k] = sum_o F[k mod 2][o - lo] x[k - o], o = {lo}..{lo + n - 1}")
        text.append(f"#define {name}_LO ({lo})")
        text.append(f"#define {name}_N {n}")
        text.append(dbl(name + "0", rows[0]))
        text.append(dbl(name + "1", rows[1]))
        text.append(flt(name + "0_32", rows[0]))
        text.append(flt(name + "1_32", rows[1]))
    text.append(flt("WVL_H32", h))
    text.append(flt("WVL_G32", g))
    text.append(flt("WVL_OMEGA32", om))
    text.append(flt("WVL_KIN32", r))
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(text))
    os.replace(tmp, path)


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    emit(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "filters_gen.h"))
