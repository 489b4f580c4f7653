"""Pins of the oracle's Takizuka-Abe step with the triplet for odd cells.

* Cells of even size: identical, bit for bit, to the plain step (the pinned
  Takizuka-Abe oracle).
* Odd cells: every member but the last three moves as in the plain step;
  each cell keeps its momentum and kinetic energy.
* Physics: in cells of three members the plain step leaves one member idle,
  so a bi-Maxwellian isotropises at about 2/3 of the rate ODE; with the
  triplet (three collisions at dt/2) it follows the rate ODE.
"""
import numpy as np

import oracle
from oracle import physics
from paper_2508_06771_amd import workloads


def population(seed, counts, aniso=True):
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts)
    n = int(counts.sum())
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    cell = np.repeat(np.arange(counts.size, dtype=np.int32), counts)
    v = workloads.bi_maxwellian(rng, n) if aniso else rng.normal(size=(3, n))
    pid = rng.permutation(n).astype(np.uint32)
    return np.ascontiguousarray(v, dtype=np.float64), cell, pid, cs


def test_even_cells_equal_plain_step():
    rng = np.random.default_rng(0)
    counts = 2 * rng.integers(0, 600, 50)
    v, cell, pid, cs = population(1, counts)
    a, b = v.copy(), v.copy()
    oracle.step_triplet(a, cs, pid, 0.05, 10.0, 3, 7)
    oracle.step(b, cell.copy(), pid.copy(), counts.size, dt=0.05, lnL=10.0, seed=3, step=7)
    assert np.array_equal(a, b)


def test_odd_cells_conserve_and_match_outside_triplet():
    counts = np.array([1, 3, 5, 7, 101, 999, 2, 0, 3])
    v, cell, pid, cs = population(2, counts)
    a, b = v.copy(), v.copy()
    oracle.step_triplet(a, cs, pid, 0.05, 10.0, 5, 1)
    oracle.step(b, cell.copy(), pid.copy(), counts.size, dt=0.05, lnL=10.0, seed=5, step=1)
    srt, _ = oracle.pairs(cs, pid, 5, 1)
    for j, N in enumerate(counts):
        sl = slice(cs[j], cs[j + 1])
        p0, e0 = v[:, sl].sum(1), (v[:, sl] ** 2).sum()
        assert np.allclose(a[:, sl].sum(1), p0, rtol=0, atol=1e-12 * (1 + np.abs(v[:, sl]).sum()))
        assert abs((a[:, sl] ** 2).sum() - e0) <= 1e-12 * e0 + 1e-300
        if N % 2 == 1 and N >= 3:
            rest = srt[cs[j]:cs[j + 1] - 3]
            assert np.array_equal(a[:, rest], b[:, rest])
            tri = srt[cs[j + 1] - 3:cs[j + 1]]
            assert np.all(np.any(a[:, tri] != v[:, tri], axis=0))
        elif N == 1:
            assert np.array_equal(a[:, sl], v[:, sl])


def temps(v):
    c = v - v.mean(axis=1, keepdims=True)
    return float(np.mean(c[2] ** 2)), float(0.5 * np.mean(c[0] ** 2 + c[1] ** 2))


def test_three_member_cells_relax_at_the_rate():
    dt = 0.1 * workloads.DT
    counts = np.full(150_000, 3)
    v, cell, pid, cs = population(4, counts)
    t0 = temps(v)
    a, b = v.copy(), v.copy()
    for k in range(40):
        oracle.step_triplet(a, cs, pid, dt, 10.0, 0, k)
        oracle.step(b, cell.copy(), pid.copy(), counts.size, dt=dt, lnL=10.0, seed=0, step=k)
    opa, ope = physics.isotropisation_rk4(t0[0], t0[1], dt, 40)
    o = (opa[-1] - ope[-1]) - (opa[0] - ope[0])
    ta, tb = temps(a), temps(b)
    ma = ((ta[0] - ta[1]) - (t0[0] - t0[1])) / o
    mb = ((tb[0] - tb[1]) - (t0[0] - t0[1])) / o
    assert abs(ma - 1) < 0.05, ma
    assert abs(mb - 2 / 3) < 0.05, mb
