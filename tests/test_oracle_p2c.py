"""Pins of the oracle's particle-to-cell sums (section "Particle-to-Cell").

* Unit quantities give the particle count of every cell (numpy's bincount).
* Integer-valued quantities sum exactly, so they equal numpy's weighted
  bincount bit for bit.
* Each cell's sum is within n eps sum|q| of the correctly rounded sum
  (math.fsum) of its particles, found by brute force.
* Summed over the cells, the result is the sum over all particles.
* Ids outside the grid are skipped and counted.
* Per-cell temperatures of a Maxwellian of temperature T from the sums of
  1, v and |v|^2 agree with T within the sampling error.
"""
import math

import numpy as np

import oracle


def test_unit_quantities_count_particles():
    rng = np.random.default_rng(0)
    cell = rng.integers(0, 37, 5000).astype(np.int32)
    s, bad = oracle.p2c(np.ones((1, cell.size)), cell, 37)
    assert bad == 0
    assert np.array_equal(s[:, 0], np.bincount(cell, minlength=37).astype(np.float64))


def test_integer_quantities_exact():
    rng = np.random.default_rng(1)
    n, M = 20_000, 301
    cell = rng.integers(0, M, n).astype(np.int32)
    q = rng.integers(-1000, 1000, (4, n)).astype(np.float64)
    s, _ = oracle.p2c(q, cell, M)
    for k in range(4):
        assert np.array_equal(s[:, k], np.bincount(cell, weights=q[k], minlength=M))


def test_brute_force_fsum():
    rng = np.random.default_rng(2)
    n, M = 3000, 17
    cell = rng.integers(0, M, n).astype(np.int32)
    q = rng.normal(size=(3, n)) * rng.lognormal(0, 3, size=(3, n))
    s, _ = oracle.p2c(q, cell, M)
    eps = 2.0 ** -53
    for j in range(M):
        sel = cell == j
        for k in range(3):
            exact = math.fsum(q[k, sel].tolist())
            bound = sel.sum() * eps * np.abs(q[k, sel]).sum()
            assert abs(s[j, k] - exact) <= bound


def test_total_over_cells():
    rng = np.random.default_rng(3)
    n, M = 10_000, 64
    cell = rng.integers(0, M, n).astype(np.int32)
    q = rng.normal(size=(2, n))
    s, _ = oracle.p2c(q, cell, M)
    for k in range(2):
        assert abs(math.fsum(s[:, k].tolist()) - math.fsum(q[k].tolist())) <= 2 * n * 2.0 ** -53 * np.abs(q[k]).sum()


def test_out_of_range_skipped():
    cell = np.array([0, 1, -1, 2, 3, 7], np.int32)
    q = np.arange(6, dtype=np.float64)[None, :]
    s, bad = oracle.p2c(q, cell, 3)
    assert bad == 3
    assert np.array_equal(s[:, 0], [0.0, 1.0, 3.0])


def test_maxwellian_temperature():
    rng = np.random.default_rng(4)
    M, per, T = 50, 4000, 2.5
    cell = np.repeat(np.arange(M, dtype=np.int32), per)
    perm = rng.permutation(cell.size)
    cell = cell[perm]
    v = rng.normal(0.0, math.sqrt(T), (3, cell.size)) + np.array([[0.3], [0.0], [-1.0]])
    q = np.vstack([np.ones(cell.size), v, (v * v).sum(axis=0)])
    s, _ = oracle.p2c(q, cell, M)
    N = s[:, 0]
    u = s[:, 1:4] / N[:, None]
    Tc = (s[:, 4] / N - (u * u).sum(axis=1)) / 3
    assert np.array_equal(N, np.full(M, float(per)))
    # var of the sample temperature ~ 2 T^2 / (3 per)
    assert np.all(np.abs(Tc - T) < 5 * T * math.sqrt(2 / (3 * per)))
    assert np.all(np.abs(u - [0.3, 0.0, -1.0]) < 5 * math.sqrt(T / per))
