"""GPU parity of the variable-weight Takizuka-Abe step (through the C ABI)
against the FP64 oracle: which members take their half change is decided in
binary64 from the weights and one Philox word on both sides, so it matches
exactly; velocities within 1e-5 relative per step in FP32 and 1e-12 in FP64
from identical inputs.  Equal weights give exactly coulomb_collide's
velocities.  Cases: empty, single, odd and even cells of every class size, a
cell beyond the LDS classes (one-workgroup path), zero weights, per-cell
densities, null collisions, three consecutive steps."""
import numpy as np
import pytest

import oracle
from paper_2508_06771_amd import workloads
from tests.gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu
TOL = {"f32": 1e-5, "f64": 1e-12}
SIGMA0, NN = 0.7, 1.0


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2508_06771_amd import piccoll
    assert torch.cuda.is_available()
    c = piccoll.Context(0)
    c.set_mcc(SIGMA0, NN, 0.0)
    yield c
    c.sync()
    c.close()


def population(seed, counts):
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts)
    n = int(counts.sum())
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    cell = np.repeat(np.arange(counts.size, dtype=np.int32), counts)
    v = np.ascontiguousarray(workloads.bi_maxwellian(rng, n), dtype=np.float64)
    pid = rng.permutation(n).astype(np.uint32)
    w = rng.choice([0.5, 1.0, 1.0, 2.0, 3.5], n)
    return v, w, cell, pid, cs, rng


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mcc", [False, True])
def test_weighted_parity_steps(ctx, dtype, mcc):
    import torch
    from paper_2508_06771_amd import piccoll
    rng = np.random.default_rng(5)
    counts = rng.integers(0, 3000, 60)
    counts[:12] = [0, 1, 2, 3, 511, 512, 513, 2049, 4097, 6145, 10240, 14001]
    v, w, cell, pid, cs, rng = population(2, counts)
    w[:50] = 0.0                                        # dead particles
    dens = np.linspace(0.5, 2.0, counts.size)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    tv, tw = dev(v, tdt), dev(w, tdt)
    ref = v.astype(np.float32).astype(np.float64) if dtype == "f32" else v.copy()
    wr = w.astype(np.float32).astype(np.float64) if dtype == "f32" else w
    fl = piccoll.FUSE_MCC if mcc else 0
    for step in range(3):
        ctx.weighted(tv, tw, dev(pid), dev(cs), dt=0.01, lnL=10.0, seed=4, step=step,
                     density=dev(dens), flags=fl)
        ctx.sync()
        oracle.step_weighted(ref, wr, cs, pid, 0.01, 10.0, 4, step, density=dens, mcc=mcc,
                             sigma0=SIGMA0, n_neutral=NN)
        g = host(tv).astype(np.float64)
        assert rel_err(g, ref) < TOL[dtype], (step, rel_err(g, ref))
        if dtype == "f32":
            ref = g.copy()          # next step from the same binary32 state on both sides
    assert np.array_equal(host(tw).astype(np.float64), wr)     # weights untouched


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_equal_weights_equal_plain_step(ctx, dtype):
    import torch
    from paper_2508_06771_amd import piccoll
    counts = np.array([0, 1, 2, 3, 100, 513, 2048, 4097, 9000, 12001, 7])
    v, w, cell, pid, cs, rng = population(3, counts)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    tv = dev(v, tdt)
    ctx.weighted(tv, dev(np.full(v.shape[1], 1.5), tdt), dev(pid), dev(cs), dt=0.01, lnL=10.0,
                 seed=8, step=2, flags=piccoll.FUSE_MCC)
    pv, pc, pp = dev(v, tdt), dev(cell), dev(pid)
    ctx.coulomb_collide(pv, pc, pp, counts.size, dt=0.01, lnL=10.0, seed=8, step=2,
                        flags=piccoll.FUSE_MCC | piccoll.ASSUME_SORTED)
    ctx.sync()
    assert torch.equal(tv, pv)


def test_weighted_rejections(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    v, w, cell, pid, cs, rng = population(4, [10, 20])
    with pytest.raises(piccoll.PicError) as e:
        ctx.weighted(dev(v, torch.float32), dev(w, torch.float32), dev(pid), dev(cs), dt=0.01,
                     lnL=10.0, seed=1, step=0, flags=piccoll.CONSERVE_FIX)
    assert e.value.status == piccoll.PIC_ERR_ARG
