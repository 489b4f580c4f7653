"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bars: bit-exact on Philox words, cell_start, orders, storage permutations,
pairings and null-collision candidate flags; velocities within 1e-12
relative in FP64 over 100 steps and within 1e-5 relative per step in FP32
(metric max_l ||dv||_inf / max(||v||_2, 1e-3 v_th)) from identical inputs.
"""
import numpy as np
import pytest

import oracle
from paper_2508_06771_amd import workloads
from tests.gpu_util import dev, host, host_u32, rel_err

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP64_TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2508_06771_amd import piccoll
    assert torch.cuda.is_available()
    c = piccoll.Context(0)
    yield c
    c.sync()
    c.close()


# ------------------------------------------------------------------ Philox
def test_philox_bitexact(ctx):
    rng = np.random.default_rng(0)
    c0 = rng.integers(0, 2 ** 32, 1_000_000, dtype=np.uint64).astype(np.uint32)
    for seed, step, dom, c3 in ((0, 0, 0, 0), (0xDEADBEEF12345678, 77, 1, 0), (5, 2 ** 32 + 3, 3, 7)):
        g = host_u32(ctx.philox(seed, step, dom, dev(c0), c3))
        ref = oracle.philox_fill(seed, step, dom, c0[:200_000], c3)
        assert np.array_equal(g[:200_000], ref)
    ctx.sync()


# ------------------------------------------------------------------ binning
def bin_case(ctx, cell_of, M):
    cs, order = ctx.bin_cells(dev(cell_of), M)
    ctx.sync()
    rcs, rorder = oracle.bin_cells(cell_of, M)
    assert np.array_equal(host(cs), rcs)
    assert np.array_equal(host(order), rorder)


@pytest.mark.parametrize("n,M", [(0, 1), (1, 1), (7, 1), (1000, 1), (5, 3), (1000, 7),
                                 (4097, 64), (100_000, 4096), (300_000, 70_000), (50_000, 2)])
def test_bin_random(ctx, n, M):
    rng = np.random.default_rng(n + M)
    bin_case(ctx, rng.integers(0, M, n).astype(np.int32), M)


def test_bin_sorted_and_empty_cells(ctx):
    cell = np.repeat(np.arange(0, 100, 3, dtype=np.int32), 17)   # every third cell used
    bin_case(ctx, cell, 101)
    bin_case(ctx, cell[::-1].copy(), 101)
    bin_case(ctx, np.full(5000, 99, np.int32), 100)


def test_bin_workloads(ctx):
    for w in (workloads.c1(0), workloads.c2(0, n_cells=128, per_cell=2000)):
        bin_case(ctx, w.cell_of, w.n_cells)


def test_bin_out_of_range_reported(ctx):
    from paper_2508_06771_amd.piccoll import PicError
    ctx.bin_cells(dev(np.array([0, 5, 1], np.int32)), 3)
    with pytest.raises(PicError) as e:
        ctx.sync()
    assert e.value.status == 2
    ctx.sync()   # latched error was cleared


# ------------------------------------------------------------------ pairing
@pytest.mark.parametrize("sizes", [
    [0, 1, 2, 3, 5, 64, 65, 255, 256, 257, 511, 512, 513],
    [2048, 2049, 4096, 4097, 6000, 10240],
    [10241, 20000, 3, 1, 0],
])
def test_pairs_bitexact(ctx, sizes):
    rng = np.random.default_rng(len(sizes))
    sizes = np.array(sizes)
    cs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(cs[-1])
    pid = rng.permutation(4 * n + 8)[:n].astype(np.uint32)
    for step in (0, 9):
        srt, par = ctx.pairs(dev(cs), dev(pid), seed=3, step=step)
        ctx.sync()
        rs, rp = oracle.pairs(cs, pid, seed=3, step=step)
        assert np.array_equal(host(srt), rs)
        assert np.array_equal(host(par), rp)


def test_pairs_tie_break(ctx):
    pids = np.arange(300000, dtype=np.uint32)
    keys = oracle.philox_fill(0, 0, 0, pids)[:, 0]
    o = np.argsort(keys, kind="stable")
    d = np.flatnonzero(keys[o][1:] == keys[o][:-1])
    a, b = sorted([int(o[d[0]]), int(o[d[0] + 1])])
    pid = np.array([b, 11, a, 12, 13], np.uint32)
    cs = np.array([0, 5], np.int32)
    srt, par = ctx.pairs(dev(cs), dev(pid), seed=0, step=0)
    rs, rp = oracle.pairs(cs, pid, 0, 0)
    assert np.array_equal(host(srt), rs) and np.array_equal(host(par), rp)


# ------------------------------------------------------------------ full step
def run_gpu_step(ctx, w, v, dtype, step, flags=0, seed=0, density=None, mcc=False):
    import torch
    from paper_2508_06771_amd import piccoll
    tv = dev(v, torch.float32 if dtype == "f32" else torch.float64)
    tc, tp = dev(w.cell_of), dev(w.pid)
    if mcc:
        ctx.set_mcc(w.sigma0, w.n_neutral, w.mass_ratio)
        flags |= piccoll.FUSE_MCC
    dens = None if density is None else dev(density)
    ctx.conserve_reset()
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=seed, step=step,
                        density=dens, flags=flags)
    ctx.sync()
    return host(tv).astype(np.float64), host(tc), host_u32(tp)


def run_oracle_step(w, v64, step, seed=0, density=None, mcc=False, conserve=False, cell=None,
                    pid=None):
    v = np.ascontiguousarray(v64, dtype=np.float64).copy()
    c = (w.cell_of if cell is None else cell).copy()
    p = (w.pid if pid is None else pid).copy()
    oracle.step(v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, seed=seed, step=step, density=density,
                mcc=mcc, sigma0=w.sigma0, n_neutral=w.n_neutral, mass_ratio=w.mass_ratio,
                conserve=conserve)
    return v, c, p


def test_fp64_c1_100_steps(ctx):
    """c1 (64 x 256, FP64): 100 steps on the GPU match 100 oracle steps."""
    import torch
    w = workloads.c1(0)
    tv = dev(w.v, torch.float64)
    tc, tp = dev(w.cell_of), dev(w.pid)
    v, c, p = w.v.copy(), w.cell_of.copy(), w.pid.copy()
    for k in range(100):
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=k)
        oracle.step(v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=k)
    ctx.sync()
    assert np.array_equal(host(tc), c) and np.array_equal(host_u32(tp), p)
    err = rel_err(host(tv), v)
    assert err < FP64_TOL, err


@pytest.mark.parametrize("mcc,dens", [(False, False), (True, False), (True, True)])
def test_fp64_step_many_large_cells(ctx, mcc, dens):
    """Binary64, 600 cells of 4,097..10,240 members (more cells than the GPU has
    compute units, ragged sizes, odd and even: the binary64 lean pass) plus
    the class boundaries 4,096 / 4,097 / 6,144 / 6,145 / 10,240 / 10,241, a
    25,000-member cell (segmented path) and tiny ones; optionally per-cell
    densities: one step from identical input equals the oracle's, every
    cell."""
    rng = np.random.default_rng(41)
    sizes = np.concatenate([rng.integers(4097, 10241, 600),
                            [0, 1, 3, 4096, 4097, 6144, 6145, 10240, 10241, 25000]])
    rng.shuffle(sizes)
    v = workloads.maxwellian_beam(rng, sizes.astype(np.int64), dtype=np.float64)
    w = workloads._finish(rng, "f64_large", v, sizes.astype(np.int64), np.float64, mcc=True)
    density = rng.uniform(0.5, 2.0, sizes.size) if dens else None
    vg, cg, pg = run_gpu_step(ctx, w, w.v, "f64", 5, mcc=mcc, density=density)
    vr, cr, pr = run_oracle_step(w, w.v, 5, mcc=mcc, density=density)
    assert np.array_equal(cg, cr) and np.array_equal(pg, pr)
    assert rel_err(vg, vr) < FP64_TOL, rel_err(vg, vr)


@pytest.mark.parametrize("mcc", [False, True])
def test_fp32_step_c2_small(ctx, mcc):
    """c2 shape at 96 cells x 10,000 (a tile-multiple plus ragged tails via the
    random storage order), one FP32 step from identical input."""
    w = workloads.c2(0, n_cells=96, per_cell=10000)
    for step in (0, 1):
        vg, cg, pg = run_gpu_step(ctx, w, w.v, "f32", step, mcc=mcc)
        vr, cr, pr = run_oracle_step(w, w.v.astype(np.float64), step, mcc=mcc)
        assert np.array_equal(cg, cr) and np.array_equal(pg, pr)
        assert rel_err(vg, vr) < FP32_TOL, rel_err(vg, vr)


def ragged_workload(seed, sizes, dtype=np.float32):
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    v = workloads.maxwellian_beam(rng, sizes, dtype=dtype)
    return workloads._finish(rng, "ragged", v, sizes, dtype, mcc=True)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_crowded_bucket_and_equal_keys(ctx, dtype):
    """Cells of 10,000, 3,000 and 600 members (binary32: the lean passes of
    three size classes; binary64: the lean pass at ten and at four members
    per thread, and the class kernel) whose pids are chosen so that 20
    members share one sort bucket (past the rank's four unrolled slots and
    past the 15 its size field holds) and two members have the same 32-bit
    key (the pid tie-break): one step with null collisions equals the
    oracle's, every member."""
    import dataclasses
    pool = np.arange(400000, dtype=np.uint32)
    keys = oracle.philox_fill(0, 0, 0, pool)[:, 0]
    o = np.argsort(keys, kind="stable")
    dup = np.flatnonzero(keys[o][1:] == keys[o][:-1])
    assert dup.size >= 3
    rng = np.random.default_rng(17)
    used, cells = set(), []
    for c, n in enumerate((10000, 3000, 600)):
        bits = int(np.ceil(np.log2(n)))
        a, b = int(o[dup[c]]), int(o[dup[c] + 1])
        top = keys >> np.uint32(32 - bits)
        vals, counts = np.unique(top, return_counts=True)
        crowd = [int(p) for p in np.flatnonzero(top == vals[np.argmax(counts)])
                 if int(p) not in used and int(p) not in (a, b)][:20]
        assert len(crowd) == 20
        members = [a, b] + crowd
        used.update(members)
        fill = [int(p) for p in rng.permutation(pool)[:2 * n] if int(p) not in used][:n - len(members)]
        used.update(fill)
        cell = np.array(members + fill, dtype=np.uint32)
        cells.append(cell[rng.permutation(n)])
    sizes = np.array([c.size for c in cells], dtype=np.int64)
    v = workloads.maxwellian_beam(rng, sizes, dtype=np.float32 if dtype == "f32" else np.float64)
    w = workloads._finish(rng, "crowded", v, sizes, np.float32 if dtype == "f32" else np.float64,
                          shuffle=False, mcc=True)
    w = dataclasses.replace(w, pid=np.concatenate(cells))
    vg, cg, pg = run_gpu_step(ctx, w, w.v, dtype, 0, mcc=True)
    vr, cr, pr = run_oracle_step(w, w.v.astype(np.float64), 0, mcc=True)
    assert np.array_equal(cg, cr) and np.array_equal(pg, pr)
    tol = FP32_TOL if dtype == "f32" else FP64_TOL
    assert rel_err(vg, vr) < tol, rel_err(vg, vr)


def test_fp32_two_round_cells_dense_mcc(ctx):
    """Binary32 cells just above what one exchange round of the largest class
    holds (10,177..10,240 members: two rounds, an odd cell's unpaired member
    in the second), beside cells of the smaller classes, with a
    null-collision probability of about 0.33, so that most threads scatter
    several members, in both rounds, with a mass ratio: one step equals the
    oracle's, every member."""
    import dataclasses
    sizes = [10177, 10239, 10240, 10200, 10178, 9999, 600, 2047, 3001, 4096, 1, 2, 3, 0]
    w = ragged_workload(13, sizes, np.float32)
    w = dataclasses.replace(w, n_neutral=w.n_neutral * 40, mass_ratio=1e-3)
    p_null = oracle.mcc_threshold(w.dt, w.sigma0, w.n_neutral) / 2.0 ** 32
    assert 0.2 < p_null < 0.5, p_null
    vg, cg, pg = run_gpu_step(ctx, w, w.v, "f32", 4, mcc=True)
    vr, cr, pr = run_oracle_step(w, w.v.astype(np.float64), 4, mcc=True)
    assert np.array_equal(cg, cr) and np.array_equal(pg, pr)
    assert rel_err(vg, vr) < FP32_TOL, rel_err(vg, vr)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ragged_cells_all_classes(ctx, dtype):
    """Cell sizes spanning every size class, empty and single-member cells and
    cells beyond the largest LDS class, with density and MCC."""
    sizes = [0, 1, 2, 3, 17, 64, 511, 512, 513, 2047, 2049, 4095, 4097, 6143, 6145, 10239,
             10241, 25000, 0, 1]
    w = ragged_workload(7, sizes, np.float32 if dtype == "f32" else np.float64)
    dens = np.linspace(0.5, 2.0, w.n_cells)
    vg, cg, pg = run_gpu_step(ctx, w, w.v, dtype, 3, density=dens, mcc=True)
    vr, cr, pr = run_oracle_step(w, w.v.astype(np.float64), 3, density=dens, mcc=True)
    assert np.array_equal(cg, cr) and np.array_equal(pg, pr)
    tol = FP32_TOL if dtype == "f32" else FP64_TOL
    assert rel_err(vg, vr) < tol, rel_err(vg, vr)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_large_cells_segmented(ctx, dtype):
    """Cells beyond the largest LDS class are split into key segments sorted
    by separate workgroups, with the pairs across segment edges done after;
    the step equals the oracle's (sizes give several segments, odd and even
    counts, and a cell beside them of each small kind)."""
    sizes = [10241, 12800, 40000, 100003, 2, 0, 30001, 6145]
    w = ragged_workload(11, sizes, np.float32 if dtype == "f32" else np.float64)
    dens = np.linspace(0.7, 1.6, w.n_cells)
    for step in (5, 6):
        vg, cg, pg = run_gpu_step(ctx, w, w.v, dtype, step, density=dens, mcc=True)
        vr, cr, pr = run_oracle_step(w, w.v.astype(np.float64), step, density=dens, mcc=True)
        assert np.array_equal(cg, cr) and np.array_equal(pg, pr)
        tol = FP32_TOL if dtype == "f32" else FP64_TOL
        assert rel_err(vg, vr) < tol, (step, rel_err(vg, vr))


def test_segmented_equals_one_workgroup_path(ctx):
    """The same step through the segmented path and through the one-workgroup
    path of the largest cells (taken when the pass also writes moment sums)
    gives bitwise equal velocities: both apply the same rotation to the same
    pairs and the same null collisions."""
    import torch
    from paper_2508_06771_amd import piccoll
    w = ragged_workload(12, [10241, 25000, 77777, 4], np.float32)
    ctx.set_mcc(w.sigma0, w.n_neutral, w.mass_ratio)
    out = []
    mom = torch.zeros(w.n_cells * 14, dtype=torch.float64, device="cuda")
    for extra in (0, piccoll.MOMENTS):
        tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
        if extra:
            ctx.set_moments_out(mom)
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=4, step=2,
                            flags=piccoll.FUSE_MCC | extra)
        ctx.sync()
        out.append(tv)
    ctx.set_moments_out(None)
    assert torch.equal(out[0], out[1])


def test_conservation_correction_fp32(ctx):
    from paper_2508_06771_amd import piccoll
    w = workloads.c2(1, n_cells=32, per_cell=10000)
    vg, cg, _ = run_gpu_step(ctx, w, w.v, "f32", 0, flags=piccoll.CONSERVE_FIX)
    vr, cr, _ = run_oracle_step(w, w.v.astype(np.float64), 0, conserve=True)
    assert rel_err(vg, vr) < FP32_TOL
    # FP64 sums of the FP32 output equal the sums of the (sorted) input
    cs, order = oracle.bin_cells(w.cell_of, w.n_cells)
    m0 = oracle.cell_moments(np.ascontiguousarray(w.v.astype(np.float64)[:, order]), cs)
    m1 = oracle.cell_moments(vg, cs)
    e0 = m0[:, 4] + m0[:, 5] + m0[:, 6]
    e1 = m1[:, 4] + m1[:, 5] + m1[:, 6]
    assert np.max(np.abs(e1 - e0) / e0) < 2e-7
    assert np.max(np.abs(m1[:, 1:4] - m0[:, 1:4])) < 2e-7 * np.sqrt(e0.max())


def test_assume_sorted_and_determinism(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    w = workloads.c2(2, n_cells=64, per_cell=3000)
    outs = []
    for _ in range(2):
        tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0)
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=1,
                            flags=piccoll.ASSUME_SORTED)
        ctx.sync()
        outs.append(host(tv).tobytes())
    assert outs[0] == outs[1]
    # asserting sorted storage that is not sorted is reported
    tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0,
                        flags=piccoll.ASSUME_SORTED)
    with pytest.raises(piccoll.PicError) as e:
        ctx.sync()
    assert e.value.status == 6
    assert np.array_equal(host(tv), w.v)    # nothing was modified


def test_out_of_range_cell_reported(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    w = workloads.c1(0, n_cells=4, per_cell=16)
    bad = w.cell_of.copy()
    bad[5] = 4
    tv, tc, tp = dev(w.v, torch.float64), dev(bad), dev(w.pid)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0)
    with pytest.raises(piccoll.PicError) as e:
        ctx.sync()
    assert e.value.status == 2
    with pytest.raises(piccoll.PicError):
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=-1.0, lnL=w.lnL, seed=0, step=0)


# ------------------------------------------------------------------ MCC alone
@pytest.mark.parametrize("dtype,mr", [("f32", 0.0), ("f64", 0.0), ("f32", 1.373e-5), ("f64", 0.01)])
def test_mcc_standalone(ctx, dtype, mr):
    import torch
    w = workloads.c2(3, n_cells=16, per_cell=5000)
    tv = dev(w.v, torch.float32 if dtype == "f32" else torch.float64)
    cand = ctx.mcc_null_collide(tv, dev(w.pid), dt=w.dt, sigma0=w.sigma0, n_neutral=1.0,
                                mass_ratio=mr, seed=4, step=11, candidates=True)
    ctx.sync()
    v = w.v.astype(np.float64).copy()
    rc = oracle.mcc(v, w.pid, w.dt, w.sigma0, 1.0, mr, 4, 11, return_flags=True)
    assert np.array_equal(host(cand), rc)
    tol = FP32_TOL if dtype == "f32" else 1e-14
    assert rel_err(host(tv).astype(np.float64), v) < tol


def test_fused_mcc_equals_standalone(ctx):
    """Coulomb with fused MCC == Coulomb then stand-alone MCC (same kernels'
    arithmetic for the scattering)."""
    import torch
    from paper_2508_06771_amd import piccoll
    w = workloads.c2(4, n_cells=16, per_cell=4000)
    tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    ctx.set_mcc(w.sigma0, 1.0, 0.0)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=5,
                        flags=piccoll.FUSE_MCC)
    tv2, tc2, tp2 = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    ctx.coulomb_collide(tv2, tc2, tp2, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=5)
    ctx.mcc_null_collide(tv2, tp2, dt=w.dt, sigma0=w.sigma0, n_neutral=1.0, mass_ratio=0.0,
                         seed=0, step=5)
    ctx.sync()
    assert np.array_equal(host(tv), host(tv2))


# ------------------------------------------------------------------ moments / unsort
def test_moments(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    w = ragged_workload(9, [0, 1, 5, 600, 3000, 12000], np.float64)
    cs, order = oracle.bin_cells(w.cell_of, w.n_cells)
    vs = np.ascontiguousarray(w.v[:, order])
    m = host(ctx.cell_moments(dev(vs, torch.float64), dev(cs)))
    ctx.sync()
    ref = oracle.cell_moments(vs, cs)
    assert np.allclose(m, ref, rtol=1e-12, atol=1e-12)
    # fused into the step: moments of the post-step state
    out = torch.zeros((w.n_cells, 14), dtype=torch.float64, device="cuda")
    ctx.set_moments_out(out)
    vg, cg, pg = run_gpu_step(ctx, w, w.v, "f64", 2, flags=piccoll.MOMENTS)
    ctx.set_moments_out(None)
    assert np.allclose(host(out), oracle.cell_moments(vg, cs), rtol=1e-12, atol=1e-11)


def test_unsort_restores_pid_order(ctx):
    import torch
    w = workloads.c2(5, n_cells=8, per_cell=1000)
    tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0)
    ctx.unsort(tv, tp, tc)
    ctx.sync()
    assert np.array_equal(host_u32(tp), np.arange(w.n, dtype=np.uint32))
    assert np.array_equal(host(tc), w.cell_of)
    vr, cr, pr = run_oracle_step(w, w.v.astype(np.float64), 0)
    back = np.empty_like(vr)
    back[:, pr] = vr
    assert rel_err(host(tv).astype(np.float64), back) < FP32_TOL


# ------------------------------------------------------------------ full size, sampled
def test_c2_full_size_sampled_cells(ctx):
    """The full c2 workload (4096 x 10,000, FP32, Coulomb + MCC) in one GPU step;
    16 sampled cells re-run by the oracle (cells are independent)."""
    w = workloads.c2(0)
    vg, cg, pg = run_gpu_step(ctx, w, w.v, "f32", 0, mcc=True)
    rng = np.random.default_rng(1)
    cells = np.sort(rng.choice(w.n_cells, 16, replace=False))
    sel = np.isin(w.cell_of, cells)
    remap = np.full(w.n_cells, -1, np.int32)
    remap[cells] = np.arange(cells.size, dtype=np.int32)
    sub = workloads.Workload("sub", np.ascontiguousarray(w.v[:, sel]), remap[w.cell_of[sel]],
                             w.pid[sel].copy(), cells.size, mcc=True)
    vr, cr, pr = run_oracle_step(sub, sub.v.astype(np.float64), 0, mcc=True)
    gsel = np.isin(cg, cells)
    assert np.array_equal(pg[gsel], pr)
    assert rel_err(vg[:, gsel], vr) < FP32_TOL


# ------------------------------------------------------------------ graph replays
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_run_steps_graph_matches_eager(ctx, dtype):
    """pic_run_steps (first step eager, then replays of a captured graph whose
    kernels read the step number from device memory) equals step-by-step
    coulomb_collide bitwise, across two calls that reuse the graph with eager
    work in between."""
    import torch
    from paper_2508_06771_amd import piccoll
    td = torch.float32 if dtype == "f32" else torch.float64
    w = ragged_workload(11, [3000] * 40 + [0, 1, 700, 12000], np.float32 if dtype == "f32" else np.float64)
    ctx.set_mcc(w.sigma0, 1.0, 0.0)
    fl = piccoll.FUSE_MCC | piccoll.CONSERVE_FIX
    # the per-cell conservation shortfall is context state: one context per
    # particle population
    eager = piccoll.Context(0)
    eager.set_mcc(w.sigma0, 1.0, 0.0)
    ctx.conserve_reset()
    A = [dev(w.v, td), dev(w.cell_of), dev(w.pid)]
    B = [dev(w.v, td), dev(w.cell_of), dev(w.pid)]
    ctx.run_steps(*A, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step0=0, nsteps=6, flags=fl)
    ctx.sync()
    for k in range(6):
        eager.coulomb_collide(*B, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step=k, flags=fl)
    eager.sync()
    assert torch.equal(A[0], B[0]) and torch.equal(A[1], B[1]) and torch.equal(A[2], B[2])
    ctx.run_steps(*A, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step0=6, nsteps=4, flags=fl)
    ctx.sync()
    for k in range(6, 10):
        eager.coulomb_collide(*B, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step=k, flags=fl)
    eager.sync()
    eager.close()
    assert torch.equal(A[0], B[0])
    # and against the oracle for the first of these steps from the same state
    vr, cr, pr = run_oracle_step(w, w.v.astype(np.float64), 0, seed=2, mcc=True, conserve=True)
    v1 = [dev(w.v, td), dev(w.cell_of), dev(w.pid)]
    ctx.conserve_reset()
    ctx.run_steps(*v1, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step0=0, nsteps=1, flags=fl)
    ctx.sync()
    tol = FP32_TOL if dtype == "f32" else FP64_TOL
    assert rel_err(host(v1[0]).astype(np.float64), vr) < tol


# ------------------------------------------------------------------ batching / autotuning
def test_autotune_keeps_results_and_caches(ctx, tmp_path, monkeypatch):
    """The tuned routing and grid sizes change where cells run, not the
    result: a step after pic_autotune equals the default-routed step bitwise
    (pairs, rotations and null collisions are per pair and per particle).
    With the conservation correction the FP64 cell sums are added in the
    order of the class's thread layout, so there the two agree to rounding.
    The choice is written to and read back from the JSON-lines cache."""
    import torch
    from paper_2508_06771_amd import piccoll
    rng = np.random.default_rng(12)
    sizes = workloads.c3_counts(rng, 300, median=2000, hi=30000)
    w = ragged_workload(12, sizes, np.float32)
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("PICCOLL_TUNE_CACHE", str(cache))
    for fl in (piccoll.FUSE_MCC, piccoll.FUSE_MCC | piccoll.CONSERVE_FIX):
        ctx = piccoll.Context(0)    # default routing until the autotune below
        ctx.set_mcc(w.sigma0, 1.0, 0.0)
        ref = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
        ctx.conserve_reset()
        ctx.coulomb_collide(*ref, w.n_cells, dt=w.dt, lnL=w.lnL, seed=4, step=0, flags=fl)
        src = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
        choice = ctx.autotune(*src, w.n_cells, dt=w.dt, lnL=w.lnL, flags=fl)
        assert torch.equal(src[0], dev(w.v, torch.float32))        # caller's state untouched
        ctx.conserve_reset()
        ctx.coulomb_collide(*src, w.n_cells, dt=w.dt, lnL=w.lnL, seed=4, step=0, flags=fl)
        ctx.sync()
        assert torch.equal(src[2], ref[2])
        if fl & piccoll.CONSERVE_FIX:
            d = (src[0].double() - ref[0].double()).abs().max().item()
            assert d <= 1e-6 * ref[0].abs().max().item(), d
        else:
            assert torch.equal(src[0], ref[0])
        again = ctx.autotune(*[dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)], w.n_cells,
                             dt=w.dt, lnL=w.lnL, flags=fl)
        assert again == choice
        ctx.close()
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and all('"choice": ' in ln for ln in lines)
