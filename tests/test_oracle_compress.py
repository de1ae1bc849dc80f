"""Pins of the compressed-storage oracle (Sec. 2.1, steps 1 and 7 of Sec. 2.4).

* packing: compress o decompress is the identity on compressed vectors;
  decompress o compress keeps exactly the region coefficients (a mask built
  point by point from the region's definition) and zeroes the rest;
  decompress is the adjoint of compress;
* the compressed local Hamiltonian is the Galerkin restriction P H P^T of the
  full one: equal to the dense matrix product on a tiny grid, symmetric;
  with regions covering the whole box it is the full H with the
  coefficients reordered;
* the synthetic sphere regions hold exactly the points within their radius
  (brute force over every coarse point).
"""

import numpy as np
import pytest

from oracle import compress as CP
from oracle import wavelet as W
from paper_0904_1543_amd import inputs


def _mask(seg_c, seg_f, dims):
    """Full-array mask of the stored coefficients, from the regions' points."""
    n1, n2, n3 = dims
    m = np.zeros((2 * n3, 2 * n2, 2 * n1), dtype=bool)
    for p in CP.region_points(seg_c):
        i1, i2, i3 = p % n1, (p // n1) % n2, p // (n1 * n2)
        m[2 * i3, 2 * i2, 2 * i1] = True
    for p in CP.region_points(seg_f):
        i1, i2, i3 = p % n1, (p // n1) % n2, p // (n1 * n2)
        for b3 in (0, 1):
            for b2 in (0, 1):
                for b1 in (0, 1):
                    if b1 or b2 or b3:
                        m[2 * i3 + b3, 2 * i2 + b2, 2 * i1 + b1] = True
    return m


DIMS = [(6, 5, 7), (8, 8, 8)]


@pytest.mark.parametrize("dims", DIMS)
def test_pack_unpack(dims):
    seg_c, seg_f = inputs.sphere_regions(3, dims, natoms=3, rc=0.4, rf=0.2)
    L = CP.compressed_length(seg_c, seg_f)
    rng = inputs.rng_for(4)
    v = rng.standard_normal(L)
    x = rng.standard_normal(inputs.fine_shape(dims))
    assert np.array_equal(CP.compress(CP.decompress(v, seg_c, seg_f, dims), seg_c, seg_f, dims), v)
    m = _mask(seg_c, seg_f, dims)
    assert m.sum() == L
    back = CP.decompress(CP.compress(x, seg_c, seg_f, dims), seg_c, seg_f, dims)
    assert np.array_equal(back, np.where(m, x, 0.0))
    lhs = np.sum(CP.decompress(v, seg_c, seg_f, dims) * x)
    rhs = np.dot(v, CP.compress(x, seg_c, seg_f, dims))
    assert abs(lhs - rhs) < 1e-12


def test_compressed_hamiltonian_is_the_galerkin_restriction():
    from oracle import filters as OF
    from test_oracle_ops import dense_ops
    dims = (4, 4, 4)                       # fine 8^3
    F = OF.filters(8)
    seg_c, seg_f = inputs.sphere_regions(5, dims, natoms=2, rc=0.45, rf=0.25)
    L = CP.compressed_length(seg_c, seg_f)
    V = inputs.potential_gauss(inputs.rng_for(6), inputs.fine_shape(dims))
    S3, A3, O3, K3 = dense_ops(inputs.fine_shape(dims), F)
    H = A3 @ (O3.T @ np.diag(V.ravel()) @ O3 + K3) @ S3
    P = np.zeros((L, H.shape[0]))           # P: full -> compressed, row by row
    for j in range(L):
        e = np.zeros(L)
        e[j] = 1.0
        P[j] = CP.decompress(e, seg_c, seg_f, dims).ravel()
    Hc = np.empty((L, L))
    for j in range(L):
        e = np.zeros(L)
        e[j] = 1.0
        Hc[:, j] = CP.local_hpsi_compressed(e, V, seg_c, seg_f, dims)[0]
    assert np.max(np.abs(Hc - P @ H @ P.T)) < 1e-12
    assert np.max(np.abs(Hc - Hc.T)) < 1e-12


def test_whole_box_regions_reorder_the_full_hamiltonian():
    dims = (5, 4, 6)
    n1, n2, n3 = dims
    full = np.array([[0, n1 * n2 * n3]], dtype=np.int32)
    rng = inputs.rng_for(8)
    c = rng.standard_normal(inputs.fine_shape(dims))
    V = inputs.potential_gauss(rng, inputs.fine_shape(dims))
    v = CP.compress(c, full, full, dims)
    hv, _ = CP.local_hpsi_compressed(v, V, full, full, dims)
    href = W.local_hpsi_orbital(c, V)[0]
    assert np.max(np.abs(hv - CP.compress(href, full, full, dims))) < 1e-13
    assert np.max(np.abs(CP.decompress(hv, full, full, dims) - href)) < 1e-13


def test_sphere_regions_hold_the_points_within_the_radius():
    dims = (9, 7, 8)
    n1, n2, n3 = dims
    seg_c, seg_f = inputs.sphere_regions(9, dims, natoms=2, rc=0.35, rf=0.2)
    rng = inputs.rng_for(9)
    centres = rng.uniform(0.0, 1.0, size=(2, 3)) * np.array([n1, n2, n3])
    for segs, rad in ((seg_c, 0.35 * 7), (seg_f, 0.2 * 7)):
        got = set(int(p) for p in CP.region_points(segs))
        want = set()
        for i3 in range(n3):
            for i2 in range(n2):
                for i1 in range(n1):
                    for c in centres:
                        d = [min(abs(i - cc), n - abs(i - cc)) for i, cc, n in
                             ((i1, c[0], n1), (i2, c[1], n2), (i3, c[2], n3))]
                        if d[0] ** 2 + d[1] ** 2 + d[2] ** 2 <= rad ** 2:
                            want.add(i1 + n1 * (i2 + n2 * i3))
        assert got == want
        starts = segs[:, 0]
        assert np.all(np.diff(starts) > 0) and np.all(segs[:, 1] > segs[:, 0])
