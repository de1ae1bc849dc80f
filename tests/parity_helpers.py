"""Error measures of the parity tests (GPU result against the float64 oracle).

Every array result is held to two bounds with the same tolerance:
  * normwise   ||got - ref||_2 / ||ref||_2  over the whole result, and
  * elementwise max|got - ref| / max|ref|, so that an error confined to a few
    points (a ragged tile edge, one plane) cannot hide under the norm.
Scalars use |got - ref| / |ref|.  Tolerances: float64 1e-12, plain float32
2e-6, compensated float32 (hi + lo) 1e-10.
"""

import numpy as np

TOL = {"f64": 1e-12, "f32": 2e-6, "f32c": 1e-10}


def _arrays(x):
    if isinstance(x, (list, tuple)):
        return [np.asarray(a, dtype=np.float64).ravel() for a in x]
    return [np.asarray(x, dtype=np.float64).ravel()]


def normwise(got, ref):
    g, r = _arrays(got), _arrays(ref)
    assert len(g) == len(r)
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(g, r))
    den = sum(float(np.sum(b ** 2)) for b in r)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def elementwise(got, ref):
    g, r = _arrays(got), _arrays(ref)
    num = max(float(np.max(np.abs(a - b))) if a.size else 0.0 for a, b in zip(g, r))
    den = max(float(np.max(np.abs(b))) if b.size else 0.0 for b in r)
    return num / den if den > 0 else num


def assert_close(got, ref, tol, what="result"):
    n = normwise(got, ref)
    e = elementwise(got, ref)
    assert n < tol, f"{what}: normwise relative error {n:.3e} >= {tol:.1e}"
    assert e < tol, f"{what}: max elementwise error / max|ref| {e:.3e} >= {tol:.1e}"


def assert_scalar(got, ref, tol, what="scalar"):
    err = abs(float(got) - float(ref))
    assert err <= tol * abs(float(ref)), f"{what}: {got!r} vs {ref!r} (rel {err / abs(ref):.3e})"
