"""Float64 oracle of the compressed wavefunction storage (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; it shares no code with the GPU library.

Sec. 2.1: a wavefunction keeps its scaling coefficient c^0 only at the coarse
grid points of the low-resolution region and its seven wavelet coefficients
c^1..c^7 only at the points of the high-resolution region; everything else is
zero and not stored.  Steps 1 and 7 of the local Hamiltonian (Sec. 2.4) unpack
this compressed form onto the whole grid and pack the result back.

Conventions (readings; the paper gives no storage layout):
  * a region is a list of segments [start, end) of consecutive points along
    axis 1 in the linear coarse index  i1 + n1 (i2 + n2 i3);
  * the compressed vector of one orbital holds the coarse-region scaling
    coefficients in segment order, then for every fine-region point in
    segment order its seven wavelet coefficients, mu = 1..7;
  * component mu = b1 + 2 b2 + 4 b3 of coarse point (i1, i2, i3) sits at
    (2 i3 + b3, 2 i2 + b2, 2 i1 + b1) of the interleaved (m3, m2, m1) array
    (the full-grid layout of the rest of the oracle).
"""

import numpy as np

from . import wavelet as W


def region_points(segs):
    """Linear coarse indices of a region, in segment order."""
    pts = []
    for a, b in np.asarray(segs, dtype=np.int64).reshape(-1, 2):
        pts.extend(range(int(a), int(b)))
    return np.asarray(pts, dtype=np.int64)


def _coords(p, dims):
    n1, n2, _ = dims
    return p % n1, (p // n1) % n2, p // (n1 * n2)


def compressed_length(seg_c, seg_f):
    return len(region_points(seg_c)) + 7 * len(region_points(seg_f))


def decompress(v, seg_c, seg_f, dims):
    """Full interleaved coefficient array of one orbital (zeros outside the
    regions) from its compressed vector (step 1 of Sec. 2.4)."""
    n1, n2, n3 = dims
    out = np.zeros((2 * n3, 2 * n2, 2 * n1))
    pc = region_points(seg_c)
    pf = region_points(seg_f)
    for k, p in enumerate(pc):
        i1, i2, i3 = _coords(p, dims)
        out[2 * i3, 2 * i2, 2 * i1] = v[k]
    base = len(pc)
    for k, p in enumerate(pf):
        i1, i2, i3 = _coords(p, dims)
        for mu in range(1, 8):
            b1, b2, b3 = mu & 1, (mu >> 1) & 1, (mu >> 2) & 1
            out[2 * i3 + b3, 2 * i2 + b2, 2 * i1 + b1] = v[base + 7 * k + mu - 1]
    return out


def compress(x, seg_c, seg_f, dims):
    """Compressed vector of one orbital: the region coefficients of the full
    array x, nothing else (step 7 of Sec. 2.4)."""
    pc = region_points(seg_c)
    pf = region_points(seg_f)
    v = np.empty(len(pc) + 7 * len(pf))
    for k, p in enumerate(pc):
        i1, i2, i3 = _coords(p, dims)
        v[k] = x[2 * i3, 2 * i2, 2 * i1]
    base = len(pc)
    for k, p in enumerate(pf):
        i1, i2, i3 = _coords(p, dims)
        for mu in range(1, 8):
            b1, b2, b3 = mu & 1, (mu >> 1) & 1, (mu >> 2) & 1
            v[base + 7 * k + mu - 1] = x[2 * i3 + b3, 2 * i2 + b2, 2 * i1 + b1]
    return v


def local_hpsi_compressed(v, V, seg_c, seg_f, dims, hgrid=(1.0, 1.0, 1.0)):
    """Steps 1 to 7 of Sec. 2.4 on one orbital: decompress, local H on the
    whole grid (steps 2-6), compress.  Returns (H v, psi) with psi the point
    values of the decompressed orbital."""
    c = decompress(v, seg_c, seg_f, dims)
    h, psi, _ = W.local_hpsi_orbital(c, V, hgrid)
    return compress(h, seg_c, seg_f, dims), psi
