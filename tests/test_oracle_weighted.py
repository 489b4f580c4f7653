"""Pins of the oracle's step for variable-weight particles (reading W1: the
uniform step's pairs and half changes; the member of smaller weight always
takes its half change, the one of larger weight with probability w_l / w_h).

* Equal weights (any common value): identical, bit for bit, to the plain step.
* Unequal weights: every member ends either where the plain step puts it or,
  for the heavier member of a pair only, where it started; the lighter member
  always moves as in the plain step.
* The heavier member's acceptance frequency is w_l / w_h (binomial bounds).
* Momentum sum w v and energy sum w |v|^2 are conserved on average: their
  change over many pairs is zero within its statistical error, while a rule
  with the roles of the weights swapped fails the same test.
"""
import numpy as np

import oracle
from paper_2508_06771_amd import workloads

DT, LNL = 0.05, 10.0


def population(seed, counts):
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts)
    n = int(counts.sum())
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    cell = np.repeat(np.arange(counts.size, dtype=np.int32), counts)
    v = workloads.bi_maxwellian(rng, n)
    pid = rng.permutation(n).astype(np.uint32)
    return np.ascontiguousarray(v, dtype=np.float64), cell, pid, cs, rng


def plain(v, cell, pid, cs, seed, step, **kw):
    b = v.copy()
    oracle.step(b, cell.copy(), pid.copy(), cs.size - 1, dt=DT, lnL=LNL, seed=seed, step=step, **kw)
    return b


def test_equal_weights_equal_plain_step():
    counts = np.array([0, 1, 2, 3, 64, 257, 1000, 5])
    v, cell, pid, cs, _ = population(1, counts)
    ref = plain(v, cell, pid, cs, 3, 9, mcc=True, sigma0=0.7, n_neutral=1.0)
    for wv in (1.0, 2.5, 1e-3):
        a = v.copy()
        oracle.step_weighted(a, np.full(v.shape[1], wv), cs, pid, DT, LNL, 3, 9, mcc=True,
                             sigma0=0.7, n_neutral=1.0)
        assert np.array_equal(a, ref)


def test_lighter_member_moves_as_plain_heavier_moves_or_stays():
    counts = np.array([2, 3, 500, 1001, 64])
    v, cell, pid, cs, rng = population(2, counts)
    w = rng.choice([0.5, 1.0, 2.0, 3.0], v.shape[1])
    ref = plain(v, cell, pid, cs, 5, 1)
    a = v.copy()
    oracle.step_weighted(a, w, cs, pid, DT, LNL, 5, 1)
    srt, par = oracle.pairs(cs, pid, 5, 1)
    moved = np.all(a == ref, axis=0)
    stayed = np.all(a == v, axis=0)
    assert np.all(moved | stayed)
    paired = par >= 0
    other = np.where(paired, par, 0)
    lighter = paired & (w <= w[other])
    assert np.all(moved[lighter])                   # lighter (or equal) members always move
    assert np.all(stayed[~paired] | moved[~paired])  # idle members: unchanged by Coulomb
    assert np.array_equal(a[:, ~paired], v[:, ~paired])
    heavier = paired & (w > w[other])
    assert stayed[heavier].any() and moved[heavier].any()


def test_acceptance_frequency():
    """Pairs of weights (1, r): the heavier member takes its change with
    probability 1/r, within 5 binomial standard deviations."""
    for r in (1.5, 4.0, 20.0):
        counts = np.full(4000, 2)
        v, cell, pid, cs, rng = population(int(10 * r), counts)
        w = np.empty(v.shape[1])
        w[0::2], w[1::2] = 1.0, r
        flip = rng.random(counts.size) < 0.5            # heavier member first or second
        w[0::2][flip], w[1::2][flip] = r, 1.0
        a = v.copy()
        oracle.step_weighted(a, w, cs, pid, DT, LNL, 7, 3)
        heavy = w == r
        took = np.any(a[:, heavy] != v[:, heavy], axis=0)
        k, m, p = took.sum(), heavy.sum(), 1.0 / r
        assert abs(k - m * p) < 5 * np.sqrt(m * p * (1 - p)) + 1, (r, k, m * p)


def _changes(v, a, w, cs):
    """Per-cell changes of the weighted momentum (3) and energy sums."""
    dv = [np.add.reduceat((w * (a[c] - v[c])), cs[:-1]) for c in range(3)]
    de = np.add.reduceat(w * ((a ** 2).sum(0) - (v ** 2).sum(0)), cs[:-1])
    return np.stack(dv + [de])


def test_weighted_sums_conserved_on_average():
    """Cells of two members, a heavier one (weight r uniform in [1.5, 5])
    moving at about (0, 0, 1.5) and a lighter one (weight 1) at about
    (0, 0, -0.5): the heavier one's expected change points towards the
    lighter one.  The mean change of sum w v and sum w |v|^2 per cell is zero
    within 5 standard errors; the rule with the weights' roles swapped (the
    heavier member always moves, the lighter with probability w_l / w_h)
    changes the z momentum and the energy by more than 10 standard errors."""
    counts = np.full(40000, 2)
    v, cell, pid, cs, rng = population(4, counts)
    n = v.shape[1]
    v = 0.1 * rng.standard_normal((3, n))
    v[2, 0::2] += 1.5
    v[2, 1::2] -= 0.5
    w = np.ones(n)
    w[0::2] = rng.uniform(1.5, 5.0, counts.size)
    dtc = 0.02                     # deflections of order one at |u| = 2
    a = v.copy()
    oracle.step_weighted(a, w, cs, pid, dtc, LNL, 11, 2)
    ch = _changes(v, a, w, cs)
    z = ch.mean(1) / (ch.std(1) / np.sqrt(ch.shape[1]))
    assert np.all(np.abs(z) < 5), z
    assert np.any(a != v)
    b = v.copy()
    oracle.step_weighted(b, 1.0 / w, cs, pid, dtc, LNL, 11, 2)   # swapped roles
    chs = _changes(v, b, w, cs)
    zs = chs.mean(1) / (chs.std(1) / np.sqrt(chs.shape[1]))
    assert abs(zs[2]) > 10 and abs(zs[3]) > 10, zs
    # equal weights: conserved in every cell to rounding
    e = v.copy()
    oracle.step_weighted(e, np.ones(n), cs, pid, dtc, LNL, 11, 2)
    che = _changes(v, e, np.ones(n), cs)
    assert np.max(np.abs(che)) < 1e-12 * (1 + np.abs(v).max() ** 2)
