"""Host-side contracts: the seeded input recipe and the bench's one-GPU rule."""

import os
import subprocess
import sys

import numpy as np

from paper_0904_1543_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_workload_recipe_is_seeded_and_shaped():
    a = inputs.workload(1)
    b = inputs.workload(1)
    assert np.array_equal(a["C"], b["C"]) and np.array_equal(a["V"], b["V"])
    assert a["C"].shape == (1, 32, 32, 32)
    assert np.allclose(np.sqrt(np.sum(a["C"] ** 2, axis=(1, 2, 3))), 1.0)
    assert a["V"].min() >= -1.0 and a["V"].max() <= 0.0
    assert np.all(a["occ"] == 2.0)


def test_truncated_batch_keeps_the_first_orbitals():
    full = inputs.workload(2)
    part = inputs.workload(2, norb=3)
    assert np.array_equal(part["C"], full["C"][:3])
    assert np.array_equal(part["V"], full["V"])


def test_gaussian_potential_range_and_periodicity():
    rng = inputs.rng_for(7)
    V = inputs.potential_gauss(rng, (12, 10, 8))
    assert V.shape == (12, 10, 8)
    assert V.max() <= 0.0 and V.min() >= -2.0 * inputs.NGAUSS
    rng = inputs.rng_for(7)
    c, s, d = inputs.gaussian_parameters(rng, (12, 10, 8))
    assert np.all((c >= 0) & (c < np.array([8, 10, 12])))
    assert np.all((s >= 1) & (s <= 4)) and np.all((d >= -2) & (d <= 0))


def test_uneven_dims_are_in_range():
    dims = inputs.uneven_dims(inputs.rng_for(5), 512)
    arr = np.array(dims)
    assert arr.shape == (512, 3) and arr.min() >= 16 and arr.max() <= 64


def test_split_hilo_recovers_float64():
    x = inputs.rng_for(3).standard_normal(1000)
    hi, lo = inputs.split_hilo(x)
    assert hi.dtype == np.float32 and lo.dtype == np.float32
    assert np.max(np.abs((hi.astype(np.float64) + lo) - x) / np.abs(x)) < 1e-13


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
