"""Float64 oracle of the preconditioner (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; it shares no code with the GPU library.

The preconditioned gradient g~ of an orbital of energy eps solves the
Helmholtz equation (Sec. 2, Eq. "precon")

    (-1/2 nabla^2 - eps) g~ = g,

by a preconditioned conjugate-gradient method.  In the orthonormal wavelet
basis the operator is  H_eps = A Kin S - eps I  (synthesis S, kinetic operator
Kin on the fine scaling coefficients, analysis A = S^T): the kinetic recursion
of Sec. 3.4 with K_0 = -eps s, followed by the analysis, since A S = I.

Readings (the paper gives the equation and the method's name, nothing more):
  * eps < 0 (a bound orbital), so H_eps is symmetric positive definite;
  * the CG preconditioner is the diagonal of H_eps in the wavelet basis
    (Jacobi); the kinetic part of the diagonal depends only on whether a
    coefficient is a scaling or a wavelet coefficient along each axis;
  * with isolated or surface boundary conditions the same, with the
    operators of those conditions;
  * the iteration starts from g~ = 0 and runs a fixed number of steps; a step
    whose curvature p.H p or previous r.z is not positive leaves the iterate
    unchanged (alpha = 0, beta = 0), which only happens for g = 0.
"""

import numpy as np

from . import boundary as BC
from . import wavelet as W


def helmholtz(c, eps, hgrid=(1.0, 1.0, 1.0), bc="periodic"):
    """H_eps c = A (Kin (S c) + K_0) with K_0 = -eps S c (Sec. 3.4), with the
    boundary condition `bc` ("periodic", "free", "surface")."""
    if bc == "periodic":
        s = W.synthesis(c)
        return W.analysis(W.kinetic(s, hgrid, k0=-eps * s))
    s = BC.synthesis(c, bc)
    return BC.analysis(BC.kinetic(s, bc, hgrid, k0=-eps * s), bc)


def kinetic_diagonal_1d(m, hgrid, free=False):
    """Diagonal of the 1D operator A Kin S on a line of m coefficients
    (periodic, or isolated), one column at a time (unit vectors through the
    1D synthesis, kinetic filter and analysis)."""
    d = np.empty(m)
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        if free:
            col = BC.analysis_1d_free(BC.kinetic_1d_free(BC.synthesis_1d_free(e, -1), -1, hgrid), -1)
        else:
            col = W.analysis_1d(W.kinetic_1d(W.synthesis_1d(e, -1), -1, hgrid), -1)
        d[j] = col[j]
    return d


def helmholtz_diagonal(shape, eps, hgrid=(1.0, 1.0, 1.0), bc="periodic"):
    """Diagonal of H_eps on a (m3, m2, m1) grid: A Kin S is the sum over axes
    of the 1D operator along that axis (A_a S_a = I on the others), so its
    diagonal is d_1[i1] + d_2[i2] + d_3[i3]; then minus eps."""
    m3, m2, m1 = shape
    free = BC.BCS[bc]
    d1 = kinetic_diagonal_1d(m1, hgrid[0], free[0] == "f")
    d2 = kinetic_diagonal_1d(m2, hgrid[1], free[1] == "f")
    d3 = kinetic_diagonal_1d(m3, hgrid[2], free[2] == "f")
    return d3[:, None, None] + d2[None, :, None] + d1[None, None, :] - eps


def pcg(g, eps, iters, hgrid=(1.0, 1.0, 1.0), history=False, bc="periodic"):
    """`iters` steps of preconditioned conjugate gradients on H_eps x = g from
    x = 0 with the diagonal preconditioner M = diag(H_eps):

        r = g, z = M^-1 r, p = z
        repeat: q = H_eps p; alpha = (r.z) / (p.q); x += alpha p;
                r -= alpha q; z' = M^-1 r; beta = (r.z') / (r.z)_old;
                p = z' + beta p

    Returns (x, ||r||) after the last step, and the iterates if `history`."""
    g = np.asarray(g, dtype=np.float64)
    diag = helmholtz_diagonal(g.shape, eps, hgrid, bc)
    x = np.zeros_like(g)
    r = g.copy()
    z = r / diag
    p = z.copy()
    rz = float(np.sum(r * z))
    xs = [x.copy()]
    for _ in range(iters):
        q = helmholtz(p, eps, hgrid, bc)
        pq = float(np.sum(p * q))
        alpha = rz / pq if (pq > 0.0 and rz > 0.0) else 0.0
        x = x + alpha * p
        r = r - alpha * q
        z = r / diag
        rz_new = float(np.sum(r * z))
        beta = rz_new / rz if rz > 0.0 else 0.0
        p = z + beta * p
        rz = rz_new
        if history:
            xs.append(x.copy())
    res = float(np.sqrt(np.sum(r * r)))
    return (x, res, xs) if history else (x, res)
