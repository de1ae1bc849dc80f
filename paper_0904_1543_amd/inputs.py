"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method: it only draws random
coefficients and potentials (numpy ``Generator(PCG64(seed))``) in a fixed
order, so that the GPU library, the oracle and the benchmark all see the same
inputs.  It imports nothing from the rest of the package.

The paper's test systems are ZnO wurtzite supercells (Sec. 6) whose structures,
pseudopotentials and grids are not available; these workloads stand in for
them.  Draw order for every workload:
  1. per-orbital coarse grid dimensions (uneven batch only),
  2. coefficients, orbital by orbital, in C order of the interleaved
     (m3, m2, m1) array, N(0, 1), each orbital scaled to unit L2 norm,
  3. the potential: uniform draws, or for each potential 16 Gaussians as
     centres (3 per Gaussian), widths, depths -- in that order.

Grid conventions: coarse dims (n1, n2, n3) with axis 1 fastest; the fine grid
and the interleaved coefficient array are (m3, m2, m1) = (2 n3, 2 n2, 2 n1).
Fine spacing 1 on every axis; occupation 2 for every orbital.
"""

import numpy as np

WORKLOADS = {
    1: dict(name="fp64 single orbital, coarse 16^3 (fine 32^3)",
            norb=1, dims=(16, 16, 16), potential="uniform"),
    2: dict(name="fp64 batch of 64 orbitals, coarse 32^3 (fine 64^3)",
            norb=64, dims=(32, 32, 32), potential="gauss16"),
    3: dict(name="precision form, 256 orbitals, coarse 48^3 (fine 96^3)",
            norb=256, dims=(48, 48, 48), potential="gauss16"),
    4: dict(name="differentiation form, 128 orbitals, coarse 32^3 (fine 64^3)",
            norb=128, dims=(32, 32, 32), potential="gauss16"),
    5: dict(name="uneven batch, 512 orbitals, coarse dims uniform in 16..64 per axis",
            norb=512, dims=None, potential="gauss16-per-orbital"),
}

OCCUPATION = 2.0
NGAUSS = 16


def fine_shape(dims):
    n1, n2, n3 = dims
    return (2 * n3, 2 * n2, 2 * n1)


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uneven_dims(rng, norb, lo=16, hi=64):
    """Coarse dims (n1, n2, n3) drawn independently and uniformly in lo..hi."""
    d = rng.integers(lo, hi + 1, size=(norb, 3))
    return [tuple(int(v) for v in row) for row in d]


def coefficients(rng, dims_list, out=None):
    """Unit-norm N(0,1) coefficient arrays; returns a list of (m3, m2, m1)
    float64 arrays, or fills ``out`` (B, m3, m2, m1) for a uniform batch."""
    res = []
    for b, dims in enumerate(dims_list):
        shp = fine_shape(dims)
        x = rng.standard_normal(int(np.prod(shp)))
        x /= np.sqrt(np.dot(x, x))
        if out is not None:
            out[b] = x.reshape(shp)
        else:
            res.append(x.reshape(shp))
    return out if out is not None else res


def potential_uniform(rng, shp, lo=-1.0, hi=0.0):
    return rng.uniform(lo, hi, size=shp)


def gaussian_parameters(rng, shp, ngauss=NGAUSS):
    """Centres uniform over the continuous periodic box, widths uniform in
    [1, 4] fine spacings, depths uniform in [-2, 0]."""
    m3, m2, m1 = shp
    centres = rng.uniform(0.0, 1.0, size=(ngauss, 3)) * np.array([m1, m2, m3])
    sigma = rng.uniform(1.0, 4.0, size=ngauss)
    depth = rng.uniform(-2.0, 0.0, size=ngauss)
    return centres, sigma, depth


def potential_gauss(rng, shp, ngauss=NGAUSS):
    """V(r) = sum_g d_g exp(-|r - r_g|^2 / (2 sigma_g^2)) on the periodic fine
    grid (integer points), with the minimum-image distance per axis."""
    m3, m2, m1 = shp
    centres, sigma, depth = gaussian_parameters(rng, shp, ngauss)
    V = np.zeros(shp, dtype=np.float64)
    for g in range(ngauss):
        parts = []
        for m, c in zip((m1, m2, m3), centres[g]):
            d = np.arange(m, dtype=np.float64) - c
            d = (d + m / 2.0) % m - m / 2.0
            parts.append(np.exp(-d * d / (2.0 * sigma[g] ** 2)))
        e1, e2, e3 = parts
        V += depth[g] * (e3[:, None, None] * e2[None, :, None] * e1[None, None, :])
    return V


def workload(k, norb=None):
    """Inputs of workload ``k`` (1..5), seed = k.  ``norb`` truncates the
    batch (the first orbitals are the same as in the full batch, because the
    potential is drawn after all coefficients only for the shared-potential
    workloads; pass None for the full workload).

    Returns dict(dims=[(n1,n2,n3)...], C=(B,m3,m2,m1) array or list,
    V=array or list, occ=(B,) array, hgrid=(1,1,1), shared_v=bool)."""
    w = WORKLOADS[k]
    rng = rng_for(k)
    B = w["norb"]
    if w["dims"] is None:
        dims = uneven_dims(rng, B)
    else:
        dims = [w["dims"]] * B
    Bc = B if norb is None else min(norb, B)
    if w["dims"] is not None:
        shp = fine_shape(w["dims"])
        C = np.empty((Bc,) + shp, dtype=np.float64)
        coefficients(rng, dims[:Bc], out=C)
        if Bc < B:  # keep the draw stream of the full workload
            for dd in dims[Bc:]:
                rng.standard_normal(int(np.prod(fine_shape(dd))))
        if w["potential"] == "uniform":
            V = potential_uniform(rng, shp)
        else:
            V = potential_gauss(rng, shp)
        shared = True
    else:
        C = coefficients(rng, dims)[:Bc]
        V = [potential_gauss(rng, fine_shape(d)) for d in dims][:Bc]
        shared = False
    return dict(dims=dims[:Bc], C=C, V=V, occ=np.full(Bc, OCCUPATION),
                hgrid=(1.0, 1.0, 1.0), shared_v=shared, name=w["name"])


def random_case(seed, norb, dims, potential="uniform"):
    """A small seeded case of the same recipe (uniform batch)."""
    rng = rng_for(seed)
    shp = fine_shape(dims)
    C = np.empty((norb,) + shp, dtype=np.float64)
    coefficients(rng, [dims] * norb, out=C)
    V = potential_uniform(rng, shp) if potential == "uniform" else potential_gauss(rng, shp)
    return dict(dims=[dims] * norb, C=C, V=V, occ=np.full(norb, OCCUPATION),
                hgrid=(1.0, 1.0, 1.0), shared_v=True)


def random_uneven_case(seed, norb, lo=4, hi=12):
    """A small seeded uneven batch with per-orbital potentials."""
    rng = rng_for(seed)
    dims = uneven_dims(rng, norb, lo, hi)
    C = coefficients(rng, dims)
    V = [potential_gauss(rng, fine_shape(d)) for d in dims]
    return dict(dims=dims, C=C, V=V, occ=np.full(norb, OCCUPATION),
                hgrid=(1.0, 1.0, 1.0), shared_v=False)


def sphere_regions(seed, dims, natoms=4, rc=0.3, rf=0.15):
    """Synthetic coarse and fine regions of a periodic box of coarse dims
    (n1, n2, n3), shaped like those of an atomic system: `natoms` centres
    uniform in the box; the coarse region is every coarse point within
    rc * min(dims) of a centre, the fine region within rf * min(dims)
    (periodic minimum-image distances, in coarse spacings).  Returned as
    segment lists [start, end) of consecutive points along axis 1 in the
    linear coarse index i1 + n1 (i2 + n2 i3), int32 arrays of shape (k, 2)."""
    n1, n2, n3 = dims
    rng = rng_for(seed)
    centres = rng.uniform(0.0, 1.0, size=(natoms, 3)) * np.array([n1, n2, n3])
    i3, i2, i1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    d2 = np.full((n3, n2, n1), np.inf)
    for c1, c2, c3 in centres:
        e = [(np.asarray(i, dtype=np.float64) - c + n / 2.0) % n - n / 2.0
             for i, c, n in ((i1, c1, n1), (i2, c2, n2), (i3, c3, n3))]
        d2 = np.minimum(d2, e[0] ** 2 + e[1] ** 2 + e[2] ** 2)
    lim = float(min(dims))
    return (segments_of_mask(d2 <= (rc * lim) ** 2), segments_of_mask(d2 <= (rf * lim) ** 2))


def segments_of_mask(mask):
    """[start, end) runs of True along the last axis of a (n3, n2, n1) mask,
    in linear index order."""
    flat = np.asarray(mask, dtype=bool)
    n1 = flat.shape[-1]
    rows = flat.reshape(-1, n1)
    segs = []
    for r, row in enumerate(rows):
        d = np.diff(np.concatenate([[0], row.astype(np.int8), [0]]))
        for a, b in zip(np.flatnonzero(d == 1), np.flatnonzero(d == -1)):
            segs.append((r * n1 + a, r * n1 + b))
    return np.asarray(segs, dtype=np.int32).reshape(-1, 2)


def directions(seed, shape, count):
    """``count`` unit-norm N(0,1) directions of the given shape."""
    rng = rng_for(seed)
    out = []
    for _ in range(count):
        d = rng.standard_normal(int(np.prod(shape)))
        d /= np.sqrt(np.dot(d, d))
        out.append(d.reshape(shape))
    return out


def split_hilo(x):
    """float64 -> (hi, lo) float32 pair with hi = fl32(x), lo = fl32(x - hi):
    the storage format of the compensated single-precision form."""
    x = np.asarray(x, dtype=np.float64)
    hi = x.astype(np.float32)
    lo = (x - hi.astype(np.float64)).astype(np.float32)
    return hi, lo
