"""The allocation-free collision step (coulomb_collide_noalloc) through the C
ABI: on storage in cell order it gives coulomb_collide's velocities bit for bit
(the same kernels, scratch from the library's fixed per-GPU array), on two
calls in a row with the second one smaller, and it rejects what its fixed
scratch cannot hold."""
import numpy as np
import pytest

from tests.gpu_util import dev, host, host_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_06771_amd import piccoll
    c = piccoll.Context(0)
    yield c
    c.close()


def sorted_workload(seed, sizes, dtype):
    """Maxwellian + beam cells of the given sizes, storage already in cell order."""
    from paper_2508_06771_amd import workloads
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    v = workloads.maxwellian_beam(rng, sizes, dtype=dtype)
    w = workloads._finish(rng, "sorted", v, sizes, dtype, mcc=True)
    order = np.argsort(w.cell_of, kind="stable")
    w.v = np.ascontiguousarray(w.v[:, order])
    w.cell_of = np.ascontiguousarray(w.cell_of[order])
    w.pid = np.ascontiguousarray(w.pid[order])
    return w


def run_both(ctx, w, tdt, seed, step, flags, density=None):
    import torch
    from paper_2508_06771_amd import piccoll
    dens = None if density is None else torch.from_numpy(density).cuda()
    ref = [dev(w.v, tdt), dev(w.cell_of), dev(w.pid)]
    ctx.coulomb_collide(*ref, w.n_cells, dt=w.dt, lnL=w.lnL, seed=seed, step=step, density=dens,
                        flags=flags | piccoll.ASSUME_SORTED)
    ctx.sync()
    out = [dev(w.v, tdt), dev(w.cell_of), dev(w.pid)]
    ctx.coulomb_collide_noalloc(*out, w.n_cells, dt=w.dt, lnL=w.lnL, seed=seed, step=step,
                                density=dens, flags=flags)
    ctx.sync()
    return ref, out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_equals_coulomb_collide_two_calls(ctx, dtype):
    import torch
    from paper_2508_06771_amd import piccoll
    tdt = torch.float32 if dtype == "f32" else torch.float64
    ndt = np.float32 if dtype == "f32" else np.float64
    cap = piccoll.NOALLOC_MAX_CELL_F32 if dtype == "f32" else piccoll.NOALLOC_MAX_CELL_F64
    ctx.set_mcc(0.5, 1.0, 0.0)
    big = [0, 1, 2, 3, 64, 511, 512, 513, 2048, 2049, 4096, 4097, cap - 1, cap, 7, 0] * 3
    small = [5, 0, 300, 1, 2000, 17]
    for call, (sizes, seed) in enumerate(((big, 11), (small, 12))):
        w = sorted_workload(seed, sizes, ndt)
        dens = np.linspace(0.5, 2.0, w.n_cells)
        ref, out = run_both(ctx, w, tdt, seed=3, step=7 + call, flags=piccoll.FUSE_MCC,
                            density=dens)
        assert torch.equal(out[1], ref[1]) and torch.equal(out[2], ref[2])
        assert torch.equal(out[0], ref[0]), (call, (out[0] - ref[0]).abs().max().item())
        assert not torch.equal(out[0], dev(w.v, tdt))   # the step changed the velocities


def test_noalloc_moments_and_grid_sizes(ctx):
    """Moment sums written by both entry points agree; a grid of the largest
    size the scratch holds runs; one cell more is rejected."""
    import torch
    from paper_2508_06771_amd import piccoll
    ctx.set_mcc(0.5, 1.0, 0.0)
    w = sorted_workload(21, [40] * piccoll.NOALLOC_MAX_CELLS, np.float32)
    m_ref = torch.zeros(w.n_cells * 14, dtype=torch.float64, device="cuda")
    m_out = torch.zeros_like(m_ref)
    ref = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
    ctx.set_moments_out(m_ref)
    ctx.coulomb_collide(*ref, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=2,
                        flags=piccoll.FUSE_MCC | piccoll.MOMENTS | piccoll.ASSUME_SORTED)
    out = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
    ctx.set_moments_out(m_out)
    ctx.coulomb_collide_noalloc(*out, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=2,
                                flags=piccoll.FUSE_MCC | piccoll.MOMENTS)
    ctx.sync()
    ctx.set_moments_out(None)
    assert torch.equal(out[0], ref[0])
    assert torch.equal(m_out, m_ref)
    with pytest.raises(piccoll.PicError) as e:
        ctx.coulomb_collide_noalloc(*out, piccoll.NOALLOC_MAX_CELLS + 1, dt=w.dt, lnL=w.lnL,
                                    seed=1, step=2)
    assert e.value.status == piccoll.PIC_ERR_RANGE


def test_noalloc_rejections(ctx):
    """Flags it cannot serve, a cell beyond the largest class (left unchanged,
    PIC_ERR_STATE at pic_sync) and storage out of cell order (nothing changed,
    PIC_ERR_STATE)."""
    import torch
    from paper_2508_06771_amd import piccoll
    ctx.set_mcc(0.5, 1.0, 0.0)
    cap = piccoll.NOALLOC_MAX_CELL_F32
    w = sorted_workload(31, [100, cap + 1, 50], np.float32)
    t = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
    for bad in (piccoll.CONSERVE_FIX, piccoll.GATE):
        with pytest.raises(piccoll.PicError) as e:
            ctx.coulomb_collide_noalloc(*t, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0,
                                        flags=bad)
        assert e.value.status == piccoll.PIC_ERR_ARG
    ctx.coulomb_collide_noalloc(*t, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0,
                                flags=piccoll.FUSE_MCC)
    with pytest.raises(piccoll.PicError) as e:
        ctx.sync()
    assert e.value.status == piccoll.PIC_ERR_STATE
    big = slice(100, 100 + cap + 1)
    assert np.array_equal(host(t[0])[:, big], w.v[:, big])           # the large cell is unchanged
    assert not np.array_equal(host(t[0])[:, :100], w.v[:, :100])     # the others collided
    # storage out of cell order
    perm = np.random.default_rng(0).permutation(w.n)
    u = [dev(np.ascontiguousarray(w.v[:, perm]), torch.float32), dev(w.cell_of[perm]),
         dev(w.pid[perm])]
    ctx.coulomb_collide_noalloc(*u, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0)
    with pytest.raises(piccoll.PicError) as e:
        ctx.sync()
    assert e.value.status == piccoll.PIC_ERR_STATE
    assert np.array_equal(host(u[0]), w.v[:, perm])
    assert np.array_equal(host_u32(u[2]), w.pid[perm])
