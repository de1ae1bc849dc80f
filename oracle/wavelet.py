"""Plain float64 CPU oracle of the local Hamiltonian path (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It is slow on purpose: every operator is written straight
from its definition with periodic (modular) indexing, one filter tap at a time
(``np.roll`` shifts a whole line by one tap), with no blocking, no fusion, no
transposes and no reordering beyond what the definitions state.  It shares no
code, table or constant generator with the GPU library.

Array convention: one orbital on a periodic fine grid is a float64 array of
shape ``(m3, m2, m1)`` (C order, axis 1 fastest), m_a = 2 n_a.  A batch is
``(B, m3, m2, m1)``.  Coarse coefficients (Sec. 2.1, Eq. "wavef0") use the same
shape with the two-level components interleaved along every axis: along axis
a, position 2i holds the scaling part and 2i+1 the wavelet part of coarse
point i, so component mu = b1 + 2 b2 + 4 b3 (b_a = 1 for "wavelet along a")
of coarse point (i1, i2, i3) sits at (2 i3 + b3, 2 i2 + b2, 2 i1 + b1).

Operators (index convention of Sec. 3.1, Eqs. "3dconv" and "1dconvtrans": a
filter w on taps l = lo..hi acts on a periodic line x of length m):

  conv      y[I] = sum_l w_l x[(I - l) mod m]
  conv_t    y[i] = sum_l w_l x[(i + l) mod m]          (adjoint of conv)
  synthesis s[(2i + j) mod m] += h_j c_i + g_j d_i      (fast wavelet transform,
                                                         Sec. 2.1, Eq. "refinement")
  analysis  c_i = sum_j h_j s[(2i+j) mod m], d_i = sum_j g_j s[(2i+j) mod m]
  magic filter  conv with omega (Sec. 2.3, Eq. "magicfilter"); its transpose conv_t
  kinetic   conv with t_l = -r_l / (2 h_a^2) along each axis, summed
            (Sec. 2.2, Eqs. "kiner", "fprod"; sign: the operator is -1/2 nabla^2)

3D operators apply the 1D operator along axes 1, 2, 3 (Sec. 3.1: three 1D
passes; in exact arithmetic the order does not matter).
"""

import numpy as np

from . import filters as _filters

AXES = {1: -1, 2: -2, 3: -3}   # paper axis -> numpy axis of (..., m3, m2, m1)


def _F():
    return _filters.filters(8)


# --------------------------------------------------------------------------
# 1D periodic operators along one numpy axis
# --------------------------------------------------------------------------

def conv(x, w, lo, axis):
    """y[I] = sum_{l=lo}^{lo+len(w)-1} w_l x[(I-l) mod m] along ``axis``.
    ``np.roll(x, l)[I] = x[(I-l) mod m]``; the shift wraps as often as needed,
    so lines shorter than the filter are periodised correctly."""
    y = np.zeros_like(x, dtype=np.float64)
    for k, wl in enumerate(w):
        y += wl * np.roll(x, lo + k, axis=axis)
    return y


def conv_t(x, w, lo, axis):
    """y[i] = sum_l w_l x[(i+l) mod m]: the adjoint of :func:`conv`."""
    y = np.zeros_like(x, dtype=np.float64)
    for k, wl in enumerate(w):
        y += wl * np.roll(x, -(lo + k), axis=axis)
    return y


def synthesis_1d(x, axis):
    """Fine scaling coefficients from an interleaved (c, d) line (Sec. 2.1):
    s[(2i + j) mod m] += h_j c_i + g_j d_i.  Placing c_i (resp. d_i) at
    position 2i of an otherwise zero line u (resp. v) gives
    s = sum_j h_j roll(u, j) + g_j roll(v, j)."""
    F = _F()
    x = np.asarray(x, dtype=np.float64)
    ax = axis % x.ndim
    m = x.shape[ax]
    assert m % 2 == 0
    even = [slice(None)] * x.ndim
    odd = [slice(None)] * x.ndim
    even[ax] = slice(0, m, 2)
    odd[ax] = slice(1, m, 2)
    u = np.zeros_like(x)
    v = np.zeros_like(x)
    u[tuple(even)] = x[tuple(even)]
    v[tuple(even)] = x[tuple(odd)]
    return conv(u, F["h"], F["lo"], ax) + conv(v, F["g"], F["lo"], ax)


def analysis_1d(s, axis):
    """Interleaved (c, d) line from fine scaling coefficients:
    c_i = sum_j h_j s[(2i+j) mod m], d_i = sum_j g_j s[(2i+j) mod m]
    (the adjoint of synthesis, and its inverse since the basis is orthogonal)."""
    F = _F()
    s = np.asarray(s, dtype=np.float64)
    ax = axis % s.ndim
    m = s.shape[ax]
    assert m % 2 == 0
    ch = conv_t(s, F["h"], F["lo"], ax)     # ch[k] = sum_j h_j s[k + j]
    dg = conv_t(s, F["g"], F["lo"], ax)
    even = [slice(None)] * s.ndim
    odd = [slice(None)] * s.ndim
    even[ax] = slice(0, m, 2)
    odd[ax] = slice(1, m, 2)
    out = np.empty_like(s)
    out[tuple(even)] = ch[tuple(even)]
    out[tuple(odd)] = dg[tuple(even)]
    return out


def kinetic_1d(s, axis, hgrid):
    """One axis of the kinetic operator -1/2 d^2/dx^2 on a fine grid of
    spacing ``hgrid``: y[I] = sum_l t_l s[(I-l) mod m], t_l = -r_l/(2 hgrid^2)."""
    F = _F()
    t = -F["r"] / (2.0 * hgrid * hgrid)
    return conv(s, t, F["r_lo"], axis)


# --------------------------------------------------------------------------
# 3D separable operators (Sec. 3.1 and Sec. 3.3): the 1D operator along
# every axis of each orbital
# --------------------------------------------------------------------------

def _each_axis(x, op1d):
    y = np.asarray(x, dtype=np.float64)
    for a in (1, 2, 3):
        y = op1d(y, AXES[a])
    return y


def synthesis(c):
    """Fast wavelet transform, coarse (scaling + 7 wavelets) -> fine scaling
    coefficients (Sec. 2.4 step 2)."""
    return _each_axis(c, synthesis_1d)


def analysis(s):
    """Inverse wavelet transform, fine scaling -> coarse coefficients
    (Sec. 2.4 step 6)."""
    return _each_axis(s, analysis_1d)


def magic_filter(s):
    """Point values on the fine grid (Sec. 2.3, Eq. "magicfilter")."""
    F = _F()
    return _each_axis(s, lambda y, ax: conv(y, F["omega"], F["omega_lo"], ax))


def magic_filter_t(y):
    """Transposed magic filter (Sec. 2.3, last sentence; Sec. 2.4 step 3c)."""
    F = _F()
    return _each_axis(y, lambda v, ax: conv_t(v, F["omega"], F["omega_lo"], ax))


def kinetic(s, hgrid=(1.0, 1.0, 1.0), k0=None):
    """Kinetic operator on fine scaling coefficients (Sec. 2.2, Eqs. "kiner",
    "fprod"): K = T x delta x delta + delta x T x delta + delta x delta x T,
    i.e. the sum of the three 1D operators.  With ``k0`` the result is
    Kin(s) + k0 (the K_0 initialisation of Sec. 3.4, Eq. "kinetic1d")."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s) if k0 is None else np.array(k0, dtype=np.float64)
    for a in (1, 2, 3):
        out = out + kinetic_1d(s, AXES[a], hgrid[a - 1])
    return out


# --------------------------------------------------------------------------
# Pipelines of Sec. 2.4 (local Hamiltonian) and Sec. 2.5 (local density)
# --------------------------------------------------------------------------

def point_values(c):
    """psi_r = magic filter of the synthesis of c (Sec. 2.5: steps 2 and 3a)."""
    return magic_filter(synthesis(c))


def local_density(C, occ):
    """rho_r = sum_i f_i psi_i(r)^2 (Sec. 2, Eq. "density"; Sec. 2.5)."""
    C = np.asarray(C, dtype=np.float64)
    rho = np.zeros(C.shape[1:], dtype=np.float64)
    for i in range(C.shape[0]):
        psi = point_values(C[i])
        rho += occ[i] * psi * psi
    return rho


def local_hpsi_orbital(c, V, hgrid=(1.0, 1.0, 1.0)):
    """Local Hamiltonian on one orbital, steps 2 to 6 of Sec. 2.4:
    s = S c; psi = Omega s; y = V psi; x' = Omega^T y;
    k = Kin(s) + x' (steps 4 and 5 together, Sec. 3.4 with K_0 = x');
    Hc = A k.  Returns (Hc, psi, s)."""
    s = synthesis(c)
    psi = magic_filter(s)
    y = V * psi
    xp = magic_filter_t(y)
    k = kinetic(s, hgrid, k0=xp)
    return analysis(k), psi, s


def local_hpsi(C, V, occ, hgrid=(1.0, 1.0, 1.0), shared_v=True):
    """Local Hamiltonian on a batch of orbitals plus the float64 reductions.

    ``C``: (B, m3, m2, m1) coarse coefficients; ``V``: (m3, m2, m1) shared
    potential, or a list of per-orbital potentials when ``shared_v`` is False.
    Returns a dict with
      hpsi      (B, ...) H c_i
      rho       sum_i f_i psi_i^2 (only with a shared potential)
      e_loc     sum_r V_r rho_r  (shared V) -- the potential energy
      e_loc_orb per orbital sum_r V_r psi_i(r)^2 (no occupation)
      e_kin_orb per orbital <c_i, A Kin S c_i> = <s_i, Kin s_i>
      e_kin     sum_i f_i e_kin_orb[i]
    """
    B = len(C)
    hps, eloc_o, ekin_o = [], np.zeros(B), np.zeros(B)
    rho = None
    for i in range(B):
        Vi = V if shared_v else V[i]
        h, psi, s = local_hpsi_orbital(C[i], Vi, hgrid)
        hps.append(h)
        eloc_o[i] = float(np.sum(Vi * psi * psi))
        ekin_o[i] = float(np.sum(s * kinetic(s, hgrid)))
        if shared_v:
            rho = occ[i] * psi * psi if rho is None else rho + occ[i] * psi * psi
    out = dict(hpsi=np.stack(hps) if shared_v else hps,
               e_loc_orb=eloc_o, e_kin_orb=ekin_o,
               e_kin=float(np.sum(np.asarray(occ) * ekin_o)))
    if shared_v:
        out["rho"] = rho
        out["e_loc"] = float(np.sum(V * rho))
    return out


# --------------------------------------------------------------------------
# Energies and their gradients (the differentiation form)
# --------------------------------------------------------------------------

def energies(C, V, occ, hgrid=(1.0, 1.0, 1.0)):
    """E_loc = sum_r V_r rho_r and E_kin = sum_i f_i <psi_i|T|psi_i>."""
    r = local_hpsi(C, V, occ, hgrid)
    return r["e_loc"], r["e_kin"]


def energy_gradients(C, V, occ, hgrid=(1.0, 1.0, 1.0)):
    """Both energies are quadratic in c_i (E = sum_i f_i <c_i, H_part c_i> with
    a symmetric H_part) and E_loc is linear in V, so
    dE_loc/dV = rho, d(E_loc + E_kin)/dc_i = 2 f_i H c_i."""
    r = local_hpsi(C, V, occ, hgrid)
    occ = np.asarray(occ, dtype=np.float64)
    dC = 2.0 * occ[:, None, None, None] * r["hpsi"]
    return r["rho"], dC


# --------------------------------------------------------------------------
# Overlap matrix and Cholesky orthonormalisation (Sec. 2.6 and Sec. 5,
# step VIII): scalar products are taken directly on the coefficients since
# the basis is orthonormal.
# --------------------------------------------------------------------------

def overlap(C):
    """S_ij = <c_i, c_j> over all coefficients of the orbitals."""
    X = np.asarray(C, dtype=np.float64).reshape(len(C), -1)
    return X @ X.T


def cholesky_orthonormalize(C):
    """S = L L^T (lower, positive diagonal); the new orbitals are the rows of
    L^{-1} X, i.e. C' = C L^{-T} with orbitals as columns of C.
    Returns (C', L)."""
    X = np.asarray(C, dtype=np.float64).reshape(len(C), -1)
    S = X @ X.T
    L = np.linalg.cholesky(S)
    Xn = np.linalg.solve(L, X)
    return Xn.reshape(np.shape(C)), L
