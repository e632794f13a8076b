"""Seeded synthetic workloads: shapes, determinism and exact positions."""
import numpy as np

from paper_2607_02954_amd import workloads as wl


def test_scaling_lengths_sum_exactly():
    ls = wl.scaling_lengths(0, 1_048_576)
    assert sum(ls) == 1_048_576 and min(ls) >= 16 and max(ls) <= 256


def test_worlds_are_deterministic_and_split_exactly():
    a = wl.uniform_population(3, n_fil=20, length=16, nx=64, ny=64)
    b = wl.uniform_population(3, n_fil=20, length=16, nx=64, ny=64)
    for k in ("cell", "frac", "rest_angle", "act_period", "act_phase"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert a.frac.dtype == np.float32 and a.cell.dtype == np.int32
    assert np.all(a.frac >= 0) and np.all(a.frac < 1)
    x = a.positions64()
    bond = np.linalg.norm(np.diff(x[:, :16], axis=1), axis=0)
    assert np.max(np.abs(bond - 1.0)) < 1e-6


def test_folding_targets_and_served_jobs():
    w = wl.folding_population(0, n_fil=4, length=12, nx=64, ny=64)
    assert w.target.shape == (2, 48)
    d = np.linalg.norm(np.diff(w.target[:, :12], axis=1), axis=0)
    assert np.max(np.abs(d - 1.0)) < 1e-12
    jobs = wl.served_jobs(0, n_jobs=16, make_world=False)
    arr = [j.arrival for j in jobs]
    assert all(b > a for a, b in zip(arr, arr[1:]))
    assert all(200 <= j.steps <= 2000 for j in jobs)
