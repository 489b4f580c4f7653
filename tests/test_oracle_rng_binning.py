"""Pins of the oracle's random numbers and binning against independent sources.

* Philox4x32-10: cross-checked block by block against rocRAND's own engine
  (compiled here from the installed header, run on the host).
* Uniform mapping: range and exact representability in binary32.
* Binning (counting sort by cell, CCS1-CCS3 of the Coulombic collision
  steps): brute-force counting and numpy's lexsort.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2508_06771_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    if shutil.which("hipcc") is None or not os.path.exists(
            "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND header / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "probe")
    subprocess.run(["hipcc", "-O1", "--offload-arch=gfx950",
                    os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(123)
    blocks = rng.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64).astype(np.uint32)
    blocks[0] = 0
    blocks[1] = 0xFFFFFFFF
    blocks[2] = [7, 0, 0, 0, 0, 0]
    text = "\n".join(" ".join(f"{x:08x}" for x in row) for row in blocks) + "\n"
    res = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True,
                         check=True)
    ref = np.array([[int(t, 16) for t in line.split()] for line in res.stdout.splitlines()],
                   dtype=np.uint32)
    ours = np.array([orc.philox(b[:4], b[4:]) for b in blocks])
    assert ref.shape == ours.shape
    assert np.array_equal(ref, ours)


def test_philox_fill_counter_layout(orc):
    """philox_fill(seed, step, domain, c0, c3) is the block with counter
    (c0, lo32(step), domain, c3) and key (lo32(seed), hi32(seed))."""
    seed, step, dom, c3 = 0x0123456789ABCDEF, (5 << 32) | 17, 2, 9
    c0 = np.array([0, 1, 99, 0xFFFFFFFF], np.uint32)
    out = orc.philox_fill(seed, step, dom, c0, c3)
    for i, c in enumerate(c0):
        ref = orc.philox([c, 17, dom, c3], [0x89ABCDEF, 0x01234567])
        assert np.array_equal(out[i], ref)


def test_uniform_mapping(orc):
    x = np.array([0, 1, 511, 512, 0x80000000, 0xFFFFFFFF], np.uint32)
    u = orc.u01(x)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 2.0 ** -24
    assert u[3] == 3 * 2.0 ** -24
    assert u[-1] == 1.0 - 2.0 ** -24
    assert all(orc.lib().orc_u01(int(a)) == b for a, b in zip(x, u))
    rng = np.random.default_rng(0)
    y = rng.integers(0, 2 ** 32, 100000, dtype=np.uint64).astype(np.uint32)
    uy = orc.u01(y)
    assert np.all(uy.astype(np.float32).astype(np.float64) == uy)   # exact in binary32
    assert np.all((uy > 0) & (uy < 1))


def test_philox_uniformity(orc):
    """Words of consecutive counters are uniform: bin counts within 5 sigma."""
    out = orc.philox_fill(0, 0, 0, np.arange(200000, dtype=np.uint32))
    for w in range(4):
        hist = np.bincount(out[:, w] >> 28, minlength=16)
        exp = out.shape[0] / 16
        assert np.all(np.abs(hist - exp) < 5 * np.sqrt(exp))


def brute_bin(cell_of, M):
    counts = np.array([(cell_of == j).sum() for j in range(M)], np.int64)
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    order = np.lexsort((np.arange(cell_of.size), cell_of)).astype(np.int32)
    return cs, order


@pytest.mark.parametrize("n,M", [(0, 1), (1, 1), (5, 3), (100, 7), (1000, 1), (3000, 97),
                                 (2000, 4000)])
def test_bin_bruteforce(orc, n, M):
    rng = np.random.default_rng(n * 31 + M)
    cell_of = rng.integers(0, M, n).astype(np.int32)
    cs, order = orc.bin_cells(cell_of, M)
    cs2, order2 = brute_bin(cell_of, M)
    assert np.array_equal(cs, cs2)
    assert np.array_equal(order, order2)


def test_bin_workloads(orc):
    for w in (workloads.c1(0), workloads.c2(0, n_cells=64, per_cell=500)):
        cs, order = orc.bin_cells(w.cell_of, w.n_cells)
        cs2, order2 = brute_bin(w.cell_of, w.n_cells)
        assert np.array_equal(cs, cs2) and np.array_equal(order, order2)


def test_bin_rejects_out_of_range(orc):
    with pytest.raises(ValueError):
        orc.bin_cells(np.array([0, 3], np.int32), 3)
    with pytest.raises(ValueError):
        orc.bin_cells(np.array([-1], np.int32), 3)
