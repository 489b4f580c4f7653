"""Pins of the oracle's per-cell pairing.

The Coulombic collision steps pair consecutive entries of the per-cell list
and only collide particles of the same cell; the reading used here orders
each cell by (Philox key, pid) and re-draws the order every step.
Checks: a naive O(N^2) selection sort, the pid tie-break on colliding keys,
structural validity (no particle twice, no pair across cells, odd cells leave
exactly one idle member) and chi-square uniformity over all matchings of
small cells.
"""
import itertools

import numpy as np
import pytest
from scipy import stats


def naive_sorted(keys, pids):
    idx = list(range(len(keys)))
    out = []
    while idx:
        best = idx[0]
        for i in idx[1:]:
            if (keys[i], pids[i]) < (keys[best], pids[best]):
                best = i
        out.append(best)
        idx.remove(best)
    return out


@pytest.mark.parametrize("sizes", [[0, 1, 2, 3, 7, 16, 33], [64] * 5, [1] * 9, [250, 1, 0, 5]])
def test_pairing_matches_selection_sort(orc, sizes):
    rng = np.random.default_rng(len(sizes))
    cs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(cs[-1])
    pid = rng.permutation(10 * n + 10)[:n].astype(np.uint32)
    for step in (0, 1, 77):
        srt, par = orc.pairs(cs, pid, seed=5, step=step)
        keys = orc.philox_fill(5, step, 0, pid)[:, 0]
        for j in range(len(sizes)):
            lo, hi = cs[j], cs[j + 1]
            ref = [lo + r for r in naive_sorted(list(keys[lo:hi]), list(pid[lo:hi]))]
            assert list(srt[lo:hi]) == ref
            for i in range(0, hi - lo - 1, 2):
                a, b = ref[i], ref[i + 1]
                assert par[a] == b and par[b] == a
            if (hi - lo) % 2 == 1:
                assert par[ref[-1]] == -1


def test_pid_tie_break(orc):
    """Find two pids whose pairing keys collide and check they are ordered by pid."""
    pids = np.arange(300000, dtype=np.uint32)
    keys = orc.philox_fill(0, 0, 0, pids)[:, 0]
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    dup = np.flatnonzero(ks[1:] == ks[:-1])
    assert dup.size > 0, "no colliding keys in range (increase it)"
    a, b = sorted([int(order[dup[0]]), int(order[dup[0] + 1])])
    # cell of 4: the colliding pair stored in reverse pid order plus two others
    cell_pid = np.array([b, 5, a, 6], np.uint32)
    cs = np.array([0, 4], np.int32)
    srt, _ = orc.pairs(cs, cell_pid, seed=0, step=0)
    pos = {int(cell_pid[s]): r for r, s in enumerate(srt)}
    assert pos[a] + 1 == pos[b]


def test_pairing_structure_random_sizes(orc):
    rng = np.random.default_rng(9)
    sizes = rng.integers(0, 40, 300)
    cs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(cs[-1])
    pid = np.arange(n, dtype=np.uint32)
    srt, par = orc.pairs(cs, pid, seed=1, step=3)
    cell = np.repeat(np.arange(sizes.size), sizes)
    assert np.array_equal(np.sort(srt), np.arange(n))   # a permutation
    paired = par >= 0
    assert np.all(par[par[paired]] == np.flatnonzero(paired))   # involution
    assert np.all(cell[par[paired]] == cell[paired])             # same cell only
    idle = np.bincount(cell[~paired], minlength=sizes.size)
    assert np.array_equal(idle, sizes % 2)


def canonical_matching(members_sorted):
    pairs = [tuple(sorted(members_sorted[2 * i:2 * i + 2])) for i in range(len(members_sorted) // 2)]
    idle = members_sorted[-1] if len(members_sorted) % 2 else None
    return (tuple(sorted(pairs)), idle)


@pytest.mark.parametrize("size,n_match", [(4, 3), (5, 15), (6, 15)])
def test_matchings_uniform_chi2(orc, size, n_match):
    """Every perfect matching (with the idle member for odd sizes) is equally likely."""
    n_cells = 20000
    cs = (np.arange(n_cells + 1) * size).astype(np.int32)
    pid = np.arange(n_cells * size, dtype=np.uint32)
    counts = {}
    for step in range(3):
        srt, _ = orc.pairs(cs, pid, seed=11, step=step)
        loc = (srt - np.repeat(cs[:-1], size)).reshape(n_cells, size)
        for row in loc:
            key = canonical_matching(list(row))
            counts[key] = counts.get(key, 0) + 1
    assert len(counts) == n_match
    obs = np.array(list(counts.values()))
    p = stats.chisquare(obs).pvalue
    assert p > 1e-4, (obs, p)


def test_pairing_changes_every_step(orc):
    cs = np.array([0, 1000], np.int32)
    pid = np.arange(1000, dtype=np.uint32)
    _, p0 = orc.pairs(cs, pid, seed=0, step=0)
    _, p1 = orc.pairs(cs, pid, seed=0, step=1)
    _, p0b = orc.pairs(cs, pid, seed=0, step=0)
    assert np.array_equal(p0, p0b)
    assert np.mean(p0 == p1) < 0.05
