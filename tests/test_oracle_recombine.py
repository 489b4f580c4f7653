"""Pins of the oracle's recombination C5 (section "Kernel for Recombination
Collision C5"): primaries matched one to one with catalytes of their cell.

* Counts: each cell has min(P_j, C_j) events (numpy counts of the flags and
  weights), only primaries lose their weight, and they are the first ones
  in storage order.
* One to one: the catalytes that change are distinct, non-primary, alive,
  in the primary's cell, a wrapped run of consecutive catalyte ranks.
* Energy: the kinetic energy of the live particles grows by eps per event
  (each catalyte takes its primary's energy plus eps).
* The run's start is uniform over the catalytes (chi-square over seeds);
  new directions are isotropic.
* Dead particles take no part; a cell without catalytes has no event.
"""
import math

import numpy as np

import oracle


def population(seed, M=40, per=200, p_prim=0.05, p_dead=0.05):
    rng = np.random.default_rng(seed)
    n = M * per
    cs = np.arange(0, n + 1, per, dtype=np.int32)
    v = rng.normal(size=(3, n))
    w = np.where(rng.random(n) < p_dead, 0.0, 1.0)
    prim = (rng.random(n) < p_prim).astype(np.uint8)
    pid = rng.permutation(n).astype(np.uint32)
    return v, w, pid, prim, cs


def energy(v, w):
    return 0.5 * float(np.sum((v * v).sum(axis=0)[w > 0]))


def test_counts_and_destroyed_primaries():
    v, w, pid, prim, cs = population(1)
    v1, w1 = v.copy(), w.copy()
    ev = oracle.recombine(v1, w1, pid, prim, cs, 0.7, 3, 5)
    for j in range(cs.size - 1):
        sl = slice(cs[j], cs[j + 1])
        alive = w[sl] > 0
        P = int(np.sum(alive & (prim[sl] == 1)))
        C = int(np.sum(alive & (prim[sl] == 0)))
        assert ev[j] == min(P, C)
        killed = np.nonzero((w[sl] > 0) & (w1[sl] == 0))[0]
        assert np.all(prim[sl][killed] == 1)
        prims = np.nonzero(alive & (prim[sl] == 1))[0]
        assert np.array_equal(killed, prims[:ev[j]])
    assert np.all(w1[w == 0] == 0)


def test_one_to_one_and_wrapped_run():
    v, w, pid, prim, cs = population(2)
    v1, w1 = v.copy(), w.copy()
    ev = oracle.recombine(v1, w1, pid, prim, cs, 0.7, 4, 1)
    changed = np.any(v1 != v, axis=0)
    for j in range(cs.size - 1):
        sl = slice(cs[j], cs[j + 1])
        cats = np.nonzero((w[sl] > 0) & (prim[sl] == 0))[0]
        hit = np.nonzero(changed[sl])[0]
        assert hit.size == ev[j]
        assert np.all(np.isin(hit, cats))           # only live catalytes move
        if ev[j]:
            ranks = np.searchsorted(cats, hit)
            C = cats.size
            # consecutive ranks modulo C
            start = [r for r in ranks if (r - 1) % C not in set(ranks)] if ev[j] < C else [ranks[0]]
            assert len(start) == 1
    assert np.array_equal(changed & (prim == 1), np.zeros_like(changed))


def test_energy_bookkeeping():
    v, w, pid, prim, cs = population(3)
    e0 = energy(v, w)
    v1, w1 = v.copy(), w.copy()
    eps = 1.0
    ev = oracle.recombine(v1, w1, pid, prim, cs, eps, 7, 2)
    assert math.isclose(energy(v1, w1), e0 + eps * ev.sum(), rel_tol=1e-12)
    assert ev.sum() > 0


def test_start_uniform_and_isotropic():
    C, trials = 12, 2400
    n = C + 1
    cs = np.array([0, n], np.int32)
    rng = np.random.default_rng(4)
    v = rng.normal(size=(3, n))
    w = np.ones(n)
    prim = np.zeros(n, np.uint8)
    prim[5] = 1
    pid = np.arange(n, dtype=np.uint32) + 100
    counts = np.zeros(n)
    dirs = []
    for s in range(trials):
        v1, w1 = v.copy(), w.copy()
        ev = oracle.recombine(v1, w1, pid, prim, cs, 0.5, s, 0)
        assert ev[0] == 1 and w1[5] == 0
        c = np.nonzero(np.any(v1 != v, axis=0))[0]
        assert c.size == 1 and c[0] != 5
        counts[c[0]] += 1
        dirs.append(v1[:, c[0]] / np.linalg.norm(v1[:, c[0]]))
    counts = np.delete(counts, 5)
    expect = trials / C
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < (C - 1) + 5 * math.sqrt(2 * (C - 1))
    d = np.array(dirs)
    assert np.all(np.abs(d.mean(axis=0)) < 5 / math.sqrt(3 * trials))


def test_no_catalytes_and_more_primaries_than_catalytes():
    n = 10
    cs = np.array([0, 4, 10], np.int32)
    v = np.random.default_rng(5).normal(size=(3, n))
    w = np.ones(n)
    prim = np.array([1, 1, 1, 1, 1, 1, 1, 0, 1, 0], np.uint8)
    pid = np.arange(n, dtype=np.uint32)
    v1, w1 = v.copy(), w.copy()
    ev = oracle.recombine(v1, w1, pid, prim, cs, 1.0, 0, 0)
    assert list(ev) == [0, 2]
    assert np.array_equal(w1, [1, 1, 1, 1, 0, 0, 1, 1, 1, 1])
    assert np.array_equal(v1[:, :4], v[:, :4])
