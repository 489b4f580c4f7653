"""GPU parity of Nanbu's Coulomb operator (through the C ABI) against the
FP64 oracle: velocities within 1e-5 relative per step in FP32 and 1e-12 in
FP64 from identical inputs (binary64 arithmetic on both sides; the
difference is the last bits of the math library and, in FP32, the storage
rounding).  Cases: odd, single-member and empty cells, a cell beyond the
LDS classes (pairing on the multi-block path), per-cell densities, a pair
with identical velocities, five consecutive steps, and the 41M-electron
plain workload in its cell-sorted storage.
"""
import numpy as np
import pytest

import oracle
from paper_2508_06771_amd import workloads
from tests.gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu
TOL = {"f32": 1e-5, "f64": 1e-12}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2508_06771_amd import piccoll
    assert torch.cuda.is_available()
    c = piccoll.Context(0)
    yield c
    c.sync()
    c.close()


def one_step(ctx, v, pid, cs, dtype, dt, lnL=10.0, seed=3, step=0, density=None):
    import torch
    tv = dev(v, torch.float32 if dtype == "f32" else torch.float64)
    td = None if density is None else dev(density)
    ctx.nanbu(tv, dev(pid), dev(cs), dt=dt, lnL=lnL, seed=seed, step=step, density=td)
    ctx.sync()
    v64 = v.astype(np.float32).astype(np.float64) if dtype == "f32" else v.copy()
    oracle.nanbu(v64, cs, pid, dt, lnL, seed, step, density)
    g = host(tv).astype(np.float64)
    assert rel_err(g, v64) < TOL[dtype]
    return g


def population(seed, counts):
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts)
    n = int(counts.sum())
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    v = rng.normal(size=(3, n)) * np.array([[1.0], [1.0], [1.4]])
    pid = rng.permutation(n).astype(np.uint32)
    return v, pid, cs


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_nanbu_parity_steps(ctx, dtype):
    rng = np.random.default_rng(1)
    counts = rng.integers(0, 3000, 200)
    counts[[0, 7, 8]] = [0, 1, 3]
    v, pid, cs = population(2, counts)
    for step in range(5):
        v = one_step(ctx, v, pid, cs, dtype, workloads.DT, step=step)
        if dtype == "f32":
            v = v.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_nanbu_large_cell_density_and_identical_pair(ctx, dtype):
    v, pid, cs = population(3, [25_000, 5, 4000, 2])
    v[:, cs[3]:cs[4]] = 0.7                      # the last cell's two members coincide
    dens = np.array([0.5, 2.0, 1.0, 3.0])
    one_step(ctx, v, pid, cs, dtype, 0.05, seed=9, step=2, density=dens)


def test_full_size_plain_workload(ctx):
    w = workloads.c2(0)
    order = np.argsort(w.cell_of, kind="stable")
    v = np.ascontiguousarray(w.v[:, order])
    pid = w.pid[order]
    cs = np.searchsorted(w.cell_of[order], np.arange(w.n_cells + 1)).astype(np.int32)
    one_step(ctx, v, pid, cs, "f32", w.dt, seed=4, step=11)
