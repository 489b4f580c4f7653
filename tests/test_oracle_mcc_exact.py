"""Pins of the oracle's exact-count null-collision selection.

The paper draws P_null N of the N particles at random (paragraph "Null
Collision Method"); the oracle selects exactly K = round(P_null n) of them,
the K smallest candidate words.  Pinned here against what fixes it from
outside its own code:

* the count is the rounded closed form, and k = 0 and k = n select nothing
  and everything;
* the selected set is the brute-force K smallest (word, pid, slot) triples of
  the Philox words (the generator itself is pinned against the published
  Random123 answers elsewhere);
* the per-particle test (the word below floor(P_null 2^32)) picks a subset or
  a superset of it;
* over seeds every particle is picked with probability K/n, and pairs with
  probability K(K-1)/(n(n-1)) (a uniformly random K-subset);
* ties at the threshold (equal pids give equal words) still select exactly K;
* selected particles move exactly as the per-particle step moves them when it
  selects everyone, the others not at all, and speeds are kept with infinitely
  heavy neutrals.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2508_06771_amd import workloads

SIGMA0 = workloads.SIGMA0


def p_null(dt, sigma0=SIGMA0, n_neutral=1.0):
    return 1.0 - math.exp(-n_neutral * sigma0 * math.sqrt(2.0) * dt)


def dt_for(k, n, sigma0=SIGMA0, n_neutral=1.0):
    """dt at which round(P_null n) = k (k < n)."""
    return -math.log1p(-k / n) / (n_neutral * sigma0 * math.sqrt(2.0))


def case(seed, n):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, n))
    pid = rng.permutation(np.arange(n, dtype=np.uint32) * 7 + 3).astype(np.uint32)
    return v, pid


def brute_force(pid, k, seed, step):
    w1 = oracle.philox_fill(seed, step, 0, pid)[:, 1]
    order = np.lexsort((np.arange(pid.size), pid, w1))   # last key is primary
    sel = np.zeros(pid.size, np.uint8)
    sel[order[:k]] = 1
    return sel


def test_count_is_rounded_closed_form():
    for n in (1, 2, 999, 10_000):
        for dt in (1e-6, 0.01, 0.3, 5.0):
            k = oracle.mcc_exact_count(n, dt, SIGMA0, 1.0)
            assert k == round(p_null(dt) * n)
    assert oracle.mcc_exact_count(10, 1e-300, 1.0, 1.0) == 0
    assert oracle.mcc_exact_count(10, 1e300, 1.0, 1.0) == 10
    assert oracle.mcc_exact_count(10, 1.0, 0.0, 1.0) == 0


@pytest.mark.parametrize("n,k", [(1000, 1), (1000, 137), (1000, 999), (4097, 2048)])
def test_selected_set_is_k_smallest_words(n, k):
    v, pid = case(n + k, n)
    dt = dt_for(k, n)
    assert oracle.mcc_exact_count(n, dt, SIGMA0, 1.0) == k
    sel = oracle.mcc_exact(v.copy(), pid, dt, SIGMA0, 1.0, 0.0, 5, 9)
    assert int(sel.sum()) == k
    assert np.array_equal(sel, brute_force(pid, k, 5, 9))


def test_k_zero_and_all():
    v, pid = case(1, 500)
    v0 = v.copy()
    assert oracle.mcc_exact(v, pid, 1e-300, SIGMA0, 1.0, 0.0, 1, 1).sum() == 0
    assert np.array_equal(v, v0)
    sel = oracle.mcc_exact(v, pid, 1e300, SIGMA0, 1.0, 0.0, 1, 1)
    assert sel.sum() == 500 and np.all(v != v0)


@pytest.mark.parametrize("dt", [0.01, 0.2])
def test_nested_with_per_particle_test(dt):
    n = 20_000
    v, pid = case(7, n)
    ex = oracle.mcc_exact(v.copy(), pid, dt, SIGMA0, 1.0, 0.0, 3, 4).astype(bool)
    cand = oracle.mcc(v.copy(), pid, dt, SIGMA0, 1.0, 0.0, 3, 4, return_flags=True).astype(bool)
    assert np.all(ex <= cand) or np.all(cand <= ex)
    # both cut the same words: the larger set adds only the next-smallest ones
    w1 = oracle.philox_fill(3, 4, 0, pid)[:, 1].astype(np.int64)
    big, small = (ex, cand) if ex.sum() >= cand.sum() else (cand, ex)
    if small.any() and (big & ~small).any():
        assert w1[small].max() <= w1[big & ~small].min()


def test_uniform_random_subset_over_seeds():
    n, k, trials = 40, 10, 3000
    v, pid = case(3, n)
    dt = dt_for(k, n)
    hits = np.zeros(n)
    pair = 0
    for s in range(trials):
        sel = oracle.mcc_exact(v.copy(), pid, dt, SIGMA0, 1.0, 0.0, 1000 + s, 2)
        assert sel.sum() == k
        hits += sel
        pair += int(sel[0] & sel[1])
    p = k / n
    sd = math.sqrt(p * (1 - p) / trials)
    assert np.max(np.abs(hits / trials - p)) < 5 * sd
    # chi-square of the per-particle counts (each Binomial(trials, k/n),
    # negatively correlated by the fixed total: scale (n-1)/n)
    chi2 = np.sum((hits - trials * p) ** 2 / (trials * p * (1 - p))) * n / (n - 1)
    assert chi2 < (n - 1) + 5 * math.sqrt(2 * (n - 1))
    q = k * (k - 1) / (n * (n - 1))
    assert abs(pair / trials - q) < 5 * math.sqrt(q * (1 - q) / trials)


def test_ties_at_threshold():
    n = 1000
    rng = np.random.default_rng(11)
    v = rng.normal(size=(3, n))
    pid = (rng.permutation(n) // 4).astype(np.uint32)    # every pid four times
    w1 = oracle.philox_fill(2, 6, 0, pid)[:, 1]
    for k in (1, 2, 3, 5, 502, 999):
        dt = dt_for(k, n)
        sel = oracle.mcc_exact(v.copy(), pid, dt, SIGMA0, 1.0, 0.0, 2, 6)
        assert sel.sum() == k
        assert np.array_equal(sel, brute_force(pid, k, 2, 6))
        # the threshold word is shared: below it all taken, above it none
        t = w1[sel.astype(bool)].max()
        assert np.all(sel[w1 < t] == 1) and np.all(sel[w1 > t] == 0)


@pytest.mark.parametrize("mr", [0.0, 0.01])
def test_scatter_equals_per_particle_step(mr):
    n = 3000
    v, pid = case(4, n)
    dt = dt_for(450, n)
    ve = v.copy()
    sel = oracle.mcc_exact(ve, pid, dt, SIGMA0, 1.0, mr, 8, 1).astype(bool)
    va = v.copy()
    oracle.mcc(va, pid, 1e300, SIGMA0, 1.0, mr, 8, 1)        # everyone scatters
    assert np.array_equal(ve[:, sel], va[:, sel])
    assert np.array_equal(ve[:, ~sel], v[:, ~sel])
    if mr == 0.0:
        assert np.allclose(np.linalg.norm(ve, axis=0), np.linalg.norm(v, axis=0),
                           rtol=1e-15, atol=0)
