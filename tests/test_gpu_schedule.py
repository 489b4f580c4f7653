"""The plain step as one persistent launch (pic_set_schedule 1: largest cells
first on whole workgroups, the smallest class one wave per cell; 2: every
cell on whole workgroups) against the default launch per size class and the
FP64 oracle: identical pairs, rotations and null collisions, so velocities
agree bit for bit with the class launches and within 1e-5 (FP32) / 1e-12
(FP64) with the oracle; graph replays equal eager steps bit for bit.  Cells of
every class size, empty and single cells, cells beyond the LDS classes
(segments inside the same launch), densities, null collisions."""
import numpy as np
import pytest

import oracle
from paper_2508_06771_amd import workloads
from tests.gpu_util import dev, host, host_u32, rel_err

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


def ragged(seed, sizes, dtype):
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    v = workloads.maxwellian_beam(rng, sizes, dtype=dtype)
    return workloads._finish(rng, "ragged", v, sizes, dtype, mcc=True)


SIZES = [0, 1, 2, 3, 17, 64, 255, 256, 257, 511, 512, 513, 2047, 2049, 4095, 4097, 6143,
         6145, 10239, 10241, 25000, 0, 1, 300, 40, 700]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_one_launch_equals_class_launches_and_oracle(ctx, dtype):
    import torch
    from paper_2508_06771_amd import piccoll
    tdt = torch.float32 if dtype == "f32" else torch.float64
    w = ragged(3, SIZES, np.float32 if dtype == "f32" else np.float64)
    dens = np.linspace(0.5, 2.0, w.n_cells)
    ctx.set_mcc(w.sigma0, w.n_neutral, w.mass_ratio)
    out = {}
    for sched in (0, 1, 2):
        ctx.set_schedule(tdt, sched)
        tv, tc, tp = dev(w.v, tdt), dev(w.cell_of), dev(w.pid)
        for step in range(2):
            ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=5, step=step,
                                density=dev(dens), flags=piccoll.FUSE_MCC)
        ctx.sync()
        out[sched] = (tv, tc, tp)
    ctx.set_schedule(tdt, 0)
    for sched in (1, 2):
        assert torch.equal(out[sched][1], out[0][1]) and torch.equal(out[sched][2], out[0][2])
        assert torch.equal(out[sched][0], out[0][0]), sched
    v = w.v.astype(np.float64).copy()
    c, p = w.cell_of.copy(), w.pid.copy()
    for step in range(2):
        oracle.step(v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, seed=5, step=step, density=dens,
                    mcc=True, sigma0=w.sigma0, n_neutral=w.n_neutral, mass_ratio=w.mass_ratio)
    assert np.array_equal(host(out[1][1]), c) and np.array_equal(host_u32(out[1][2]), p)
    assert rel_err(host(out[1][0]).astype(np.float64), v) < 2 * TOL[dtype]


def test_one_launch_graph_equals_eager(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    rng = np.random.default_rng(9)
    sizes = workloads.c3_counts(rng, 400, median=2000, hi=30000)
    w = ragged(9, sizes, np.float32)
    ctx.set_mcc(w.sigma0, w.n_neutral, 0.0)
    ctx.set_schedule(torch.float32, 1)
    A = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
    ctx.run_steps(*A, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step0=0, nsteps=6,
                  flags=piccoll.FUSE_MCC)
    B = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
    for k in range(6):
        ctx.coulomb_collide(*B, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step=k,
                            flags=piccoll.FUSE_MCC)
    ctx.sync()
    ctx.set_schedule(torch.float32, 0)
    assert torch.equal(A[0], B[0]) and torch.equal(A[2], B[2])


def test_set_schedule_rejects(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    with pytest.raises(piccoll.PicError) as e:
        ctx.set_schedule(torch.float32, 3)
    assert e.value.status == piccoll.PIC_ERR_ARG
