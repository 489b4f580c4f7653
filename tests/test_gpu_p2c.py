"""GPU parity of the particle-to-cell sums (through the C ABI) against the
FP64 oracle.

Both sides sum the same binary64 values (binary32 inputs convert exactly) in
different orders, so each cell's sum differs by rounding only: the bar is
4 N_j eps sum_{l in j} |q_l| per cell (N_j its particle count, eps 2^-53).
Cases: both the LDS form (n_cells * nq <= 16384) and the global-atomic form,
cell-sorted and random particle order, nq 1..4, binary32 and binary64, one
crowded cell, n = 0, n = 1, a ragged tail, an id outside the grid (reported
by pic_sync, the rest still summed), and the 41M-electron plain workload in
its cell-sorted storage.
"""
import numpy as np
import pytest

import oracle
from paper_2508_06771_amd import workloads
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2508_06771_amd import piccoll
    assert torch.cuda.is_available()
    c = piccoll.Context(0)
    yield c
    c.sync()
    c.close()


def check(ctx, q, cell, M, dtype="f64"):
    import torch
    tq = dev(q, torch.float32 if dtype == "f32" else torch.float64)
    out = ctx.p2c_sums(tq, dev(cell), M)
    ctx.sync()
    qh = host(tq).astype(np.float64)
    ref, bad = oracle.p2c(qh, cell, M)
    absq, _ = oracle.p2c(np.abs(qh), cell, M)
    cnt, _ = oracle.p2c(np.ones((1, cell.size)), cell, M)
    tol = 4 * cnt[:, :1] * EPS * absq + 1e-300
    g = host(out)
    assert np.all(np.abs(g - ref) <= tol), np.max(np.abs(g - ref) / tol)
    return g


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("nq", [1, 2, 3, 4])
@pytest.mark.parametrize("M,order", [(64, "random"), (4096, "sorted"), (4096, "random"),
                                     (5000, "random"), (65536, "sorted"), (65536, "random")])
def test_p2c_parity(ctx, dtype, nq, M, order):
    rng = np.random.default_rng(M + nq)
    n = 1_000_003
    cell = rng.integers(0, M, n).astype(np.int32)
    if order == "sorted":
        cell = np.sort(cell)
    q = rng.normal(size=(nq, n)) * rng.lognormal(0, 1, size=(nq, n))
    check(ctx, q, cell, M, dtype)


def test_crowded_cell_and_small_sizes(ctx):
    rng = np.random.default_rng(9)
    n = 300_001
    cell = np.where(rng.random(n) < 0.9, 7, rng.integers(0, 100_000, n)).astype(np.int32)
    check(ctx, rng.normal(size=(4, n)), cell, 100_000)      # global form, one crowded cell
    check(ctx, rng.normal(size=(4, n)), cell % 1000, 1000)  # LDS form
    for n in (1, 2, 63, 65, 1025):
        c = rng.integers(0, 10, n).astype(np.int32)
        check(ctx, rng.normal(size=(3, n)), c, 10)


def test_empty_input(ctx):
    import torch
    out = ctx.p2c_sums(torch.empty((4, 0), dtype=torch.float32, device="cuda"),
                       torch.empty(0, dtype=torch.int32, device="cuda"), 33)
    ctx.sync()
    assert np.array_equal(host(out), np.zeros((33, 4)))


def test_out_of_range_id_reported():
    import torch
    from paper_2508_06771_amd import piccoll
    c = piccoll.Context(0)
    try:
        rng = np.random.default_rng(3)
        n = 50_000
        cell = rng.integers(0, 200, n).astype(np.int32)
        cell[[5, 777, 40_000]] = [200, -1, 1 << 20]
        q = rng.normal(size=(2, n))
        out = c.p2c_sums(dev(q, torch.float64), dev(cell), 200)
        with pytest.raises(piccoll.PicError) as e:
            c.sync()
        assert e.value.status == 2
        ref, bad = oracle.p2c(q, cell, 200)
        assert bad == 3
        assert np.allclose(host(out), ref, rtol=1e-12, atol=1e-12)
    finally:
        c.close()


def test_full_size_plain_workload(ctx):
    """41M electrons, 4096 cells, cell-sorted storage: count, momentum."""
    w = workloads.c2(0)
    order = np.argsort(w.cell_of, kind="stable")
    cell = w.cell_of[order]
    v = w.v[:, order]
    q = np.vstack([np.ones((1, w.n), np.float32), v]).astype(np.float32)
    g = check(ctx, q, cell, w.n_cells, "f32")
    assert np.array_equal(g[:, 0], np.full(w.n_cells, 10_000.0))
