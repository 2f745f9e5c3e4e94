"""Seeded input generators: reproducibility and the stated distributions."""
import numpy as np

import workloads as W


def test_rhs_reproducible_and_uniform():
    a = W.rhs(100000, 2)
    b = W.rhs(100000, 2)
    assert np.array_equal(a, b)
    assert a.min() >= -1 and a.max() <= 1
    assert abs(a.mean()) < 0.01 and abs(a.var() - 1 / 3) < 0.01


def test_gaussian_field_unit_variance_and_correlation():
    g = W.gaussian_field(63, 2, seed=5, corr_len=1.0 / 16.0)
    assert g.shape == (65, 65)
    assert abs(g.var() - 1.0) < 0.35
    # lag of one correlation length (4 nodes at h = 1/64): exp(-1/2)
    c = np.mean((g[:, 4:] - g.mean()) * (g[:, :-4] - g.mean())) / g.var()
    assert abs(c - np.exp(-0.5)) < 0.15
    assert np.array_equal(g, W.gaussian_field(63, 2, seed=5, corr_len=1.0 / 16.0))


def test_batched_table():
    t = W.batched_instances()
    assert len(t) == 512
    assert all(31 <= i.n <= 255 for i in t)
    assert W.batched_levels(31) == 3 and W.batched_levels(255) == 6 and W.batched_levels(100) == 4
    tot = sum(i.ndof for i in t)
    assert 10_000_000 < tot < 15_000_000


def test_level_sizes():
    assert W.level_sizes(127, 6) == [127, 63, 31, 15, 7, 3]
    assert W.level_sizes(31, 4) == [31, 15, 7, 3]
