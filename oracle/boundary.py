"""Float64 oracle of the local Hamiltonian with isolated and surface boundary
conditions (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; it shares no code with the GPU library.

Sec. 3.1: the boundary conditions decide the values of the arrays in the
convolutions when an index falls outside the box.  Periodic: the data wrap
(the rest of the oracle).  Isolated (free) along an axis: there is nothing
outside, the basis functions of the box are those of the infinite line, and
every 1D operator maps an array onto the whole range its result can occupy:

  coefficients  c, d at coarse points i = 0..n-1, interleaved: length m = 2n,
                global fine positions 0..m-1;
  synthesis     s[2i + j] += h_j c_i + g_j d_i        -> positions -7..m+6
                (length m + 14);
  magic filter  psi[I] = sum_l w_l s[I - l]           -> positions -14..m+14
                (length m + 29): the real-space grid of V and rho;
  transpose     x[i] = sum_l w_l y[i + l]             on positions -7..m+6;
  kinetic       K[I] = sum_l t_l s[I - l]             on positions -7..m+6
                (the Galerkin matrix of -1/2 d^2/dx^2 among the fine scaling
                functions present);
  analysis      c_i = sum_j h_j x[2i + j], d_i = sum_j g_j x[2i + j].

Surface (slab) boundary conditions: periodic along axes 1 and 3, isolated
along axis 2.  A 3D operator applies the 1D operator of each axis with that
axis's condition.  Readings: the free range conventions above are the
smallest ones that hold every nonzero value (BigDFT's isolated grids have the
same extents); no h^3 volume element, as everywhere in the oracle.
"""

import numpy as np

from . import filters as _filters
from . import wavelet as W

S_LO = -7       # first global position of the fine scaling coefficients
R_LO = -14      # first global position of the real-space grid
S_EXTRA = 14    # m + 14 fine scaling coefficients
R_EXTRA = 29    # m + 29 real-space points

BCS = {"periodic": ("p", "p", "p"), "free": ("f", "f", "f"), "surface": ("p", "f", "p")}


def _F():
    return _filters.filters(8)


def _shift_add(out, x, w, lo, axis, out_lo, in_lo):
    """out[K] += sum_k w_k x[K - (lo + k)] along `axis`, with K the global
    position of out's entries (first: out_lo) and x's entries at global
    positions in_lo.., zero outside.  Plain index arithmetic, one tap at a
    time."""
    ax = axis % x.ndim
    nin, nout = x.shape[ax], out.shape[ax]
    for k, wl in enumerate(w):
        sh = lo + k                     # out[K] uses x[K - sh]
        # local indices: K = out_lo + a, input global K - sh = in_lo + b
        # -> b = a + out_lo - sh - in_lo
        d = out_lo - sh - in_lo
        a0 = max(0, -d)
        a1 = min(nout, nin - d)
        if a1 <= a0:
            continue
        dst = [slice(None)] * x.ndim
        src = [slice(None)] * x.ndim
        dst[ax] = slice(a0, a1)
        src[ax] = slice(a0 + d, a1 + d)
        out[tuple(dst)] += wl * x[tuple(src)]
    return out


def _resized(x, axis, n):
    shp = list(x.shape)
    shp[axis % x.ndim] = n
    return np.zeros(shp)


def synthesis_1d_free(x, axis):
    """c, d on positions 0..m-1 (interleaved) -> s on -7..m+6."""
    F = _F()
    x = np.asarray(x, dtype=np.float64)
    ax = axis % x.ndim
    m = x.shape[ax]
    even = [slice(None)] * x.ndim
    odd = [slice(None)] * x.ndim
    even[ax] = slice(0, m, 2)
    odd[ax] = slice(1, m, 2)
    u = np.zeros_like(x)
    v = np.zeros_like(x)
    u[tuple(even)] = x[tuple(even)]     # c_i at position 2i
    v[tuple(even)] = x[tuple(odd)]      # d_i at position 2i
    out = _resized(x, ax, m + S_EXTRA)
    _shift_add(out, u, F["h"], F["lo"], ax, S_LO, 0)
    _shift_add(out, v, F["g"], F["lo"], ax, S_LO, 0)
    return out


def analysis_1d_free(s, axis):
    """s on -7..m+6 -> interleaved c, d on 0..m-1: c_i = sum_j h_j s[2i+j]."""
    F = _F()
    s = np.asarray(s, dtype=np.float64)
    ax = axis % s.ndim
    m = s.shape[ax] - S_EXTRA
    # ch[k] = sum_j h_j s[k + j]: a filter with taps -j, evaluated at k = 0..m-1
    ch = _resized(s, ax, m)
    dg = _resized(s, ax, m)
    _shift_add(ch, s, F["h"][::-1], -(F["lo"] + len(F["h"]) - 1), ax, 0, S_LO)
    _shift_add(dg, s, F["g"][::-1], -(F["lo"] + len(F["g"]) - 1), ax, 0, S_LO)
    out = np.empty(ch.shape)
    even = [slice(None)] * s.ndim
    odd = [slice(None)] * s.ndim
    even[ax] = slice(0, m, 2)
    odd[ax] = slice(1, m, 2)
    out[tuple(even)] = ch[tuple(even)]
    out[tuple(odd)] = dg[tuple(even)]
    return out


def magic_filter_1d_free(s, axis):
    """s on -7..m+6 -> psi on -14..m+14."""
    F = _F()
    s = np.asarray(s, dtype=np.float64)
    ax = axis % s.ndim
    m = s.shape[ax] - S_EXTRA
    out = _resized(s, ax, m + R_EXTRA)
    return _shift_add(out, s, F["omega"], F["omega_lo"], ax, R_LO, S_LO)


def magic_filter_t_1d_free(y, axis):
    """y on -14..m+14 -> x on -7..m+6: x[i] = sum_l w_l y[i + l]."""
    F = _F()
    y = np.asarray(y, dtype=np.float64)
    ax = axis % y.ndim
    m = y.shape[ax] - R_EXTRA
    out = _resized(y, ax, m + S_EXTRA)
    w = F["omega"][::-1]
    return _shift_add(out, y, w, -(F["omega_lo"] + len(F["omega"]) - 1), ax, S_LO, R_LO)


def kinetic_1d_free(s, axis, hgrid):
    """K[I] = sum_l t_l s[I - l] on -7..m+6, t_l = -r_l / (2 h^2), zero outside."""
    F = _F()
    s = np.asarray(s, dtype=np.float64)
    ax = axis % s.ndim
    out = np.zeros_like(s)
    return _shift_add(out, s, -F["r"] / (2.0 * hgrid * hgrid), F["r_lo"], ax, S_LO, S_LO)


# -------------------------------------------------------------------------
# 3D operators with one boundary condition per axis
# -------------------------------------------------------------------------

def _per_axis(x, bc, free_op, per_op):
    y = np.asarray(x, dtype=np.float64)
    for a in (1, 2, 3):
        ax = W.AXES[a]
        y = free_op(y, ax) if BCS[bc][a - 1] == "f" else per_op(y, ax)
    return y


def synthesis(c, bc):
    return _per_axis(c, bc, synthesis_1d_free, W.synthesis_1d)


def analysis(s, bc):
    return _per_axis(s, bc, analysis_1d_free, W.analysis_1d)


def magic_filter(s, bc):
    F = _F()
    return _per_axis(s, bc, magic_filter_1d_free,
                     lambda y, ax: W.conv(y, F["omega"], F["omega_lo"], ax))


def magic_filter_t(y, bc):
    F = _F()
    return _per_axis(y, bc, magic_filter_t_1d_free,
                     lambda v, ax: W.conv_t(v, F["omega"], F["omega_lo"], ax))


def kinetic(s, bc, hgrid=(1.0, 1.0, 1.0), k0=None):
    """Sum over axes of the 1D kinetic operator, each with its axis's
    condition, on fine scaling coefficients s; plus k0 if given."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s) if k0 is None else np.array(k0, dtype=np.float64)
    for a in (1, 2, 3):
        ax = W.AXES[a]
        if BCS[bc][a - 1] == "f":
            out = out + kinetic_1d_free(s, ax, hgrid[a - 1])
        else:
            out = out + W.kinetic_1d(s, ax, hgrid[a - 1])
    return out


def real_space_shape(dims, bc):
    """(M3, M2, M1) of V and rho: m_a + 29 along isolated axes."""
    n1, n2, n3 = dims
    m = [2 * n1, 2 * n2, 2 * n3]
    M = [mm + (R_EXTRA if BCS[bc][a] == "f" else 0) for a, mm in enumerate(m)]
    return (M[2], M[1], M[0])


def local_hpsi_orbital(c, V, bc, hgrid=(1.0, 1.0, 1.0)):
    """Steps 2-6 of Sec. 2.4 with the boundary condition `bc` ("periodic",
    "free", "surface"): s = S c, psi = Omega s, y = V psi, H c =
    A (Omega^T y + Kin s).  V lives on real_space_shape.  Returns (Hc, psi, s)."""
    s = synthesis(c, bc)
    psi = magic_filter(s, bc)
    k = kinetic(s, bc, hgrid, k0=magic_filter_t(V * psi, bc))
    return analysis(k, bc), psi, s


def local_hpsi(C, V, occ, bc, hgrid=(1.0, 1.0, 1.0)):
    """Batch with a shared potential: H c_i, rho, E_loc, per-orbital energies."""
    hps, epot, ekin = [], [], []
    rho = None
    for i, c in enumerate(C):
        h, psi, s = local_hpsi_orbital(c, V, bc, hgrid)
        hps.append(h)
        epot.append(float(np.sum(V * psi * psi)))
        ekin.append(float(np.sum(s * kinetic(s, bc, hgrid))))
        rho = occ[i] * psi * psi if rho is None else rho + occ[i] * psi * psi
    return dict(hpsi=hps, rho=rho, e_loc=float(np.sum(V * rho)),
                e_loc_orb=np.array(epot), e_kin_orb=np.array(ekin),
                e_kin=float(np.dot(occ, ekin)))
