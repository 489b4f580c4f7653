"""Failure handling of the collision step through the C ABI, forced from the
host: a NaN planted in the input is reported by pic_sync as
PIC_ERR_NONFINITE under PIC_CHECK_FINITE (and the step still runs); a
workspace budget below a call's scratch gives PIC_ERR_NOMEM before anything
runs, the arrays unchanged; the context keeps working afterwards."""
import numpy as np
import pytest

from paper_2508_06771_amd import workloads
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2508_06771_amd import piccoll
    assert torch.cuda.is_available()
    c = piccoll.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_nan_injection_reported(ctx, dtype):
    import torch
    from paper_2508_06771_amd import piccoll
    tdt = torch.float32 if dtype == "f32" else torch.float64
    w = workloads.c2(1, n_cells=8, per_cell=3000, dtype=np.float32 if dtype == "f32" else np.float64)
    ctx.set_mcc(w.sigma0, w.n_neutral, 0.0)
    # clean input: no report
    tv, tc, tp = dev(w.v, tdt), dev(w.cell_of), dev(w.pid)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0,
                        flags=piccoll.FUSE_MCC | piccoll.CHECK_FINITE)
    ctx.sync()
    # one NaN component: reported with the check, silent without
    bad = w.v.copy()
    bad[1, 1234] = np.nan
    for fl, want in ((piccoll.CHECK_FINITE, piccoll.PIC_ERR_NONFINITE), (0, None)):
        tv, tc, tp = dev(bad, tdt), dev(w.cell_of), dev(w.pid)
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0,
                            flags=piccoll.FUSE_MCC | fl)
        if want is None:
            ctx.sync()
        else:
            with pytest.raises(piccoll.PicError) as e:
                ctx.sync()
            assert e.value.status == want
        assert np.isnan(host(tv)).any()
    # the latch is cleared by the report
    tv, tc, tp = dev(w.v, tdt), dev(w.cell_of), dev(w.pid)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=1,
                        flags=piccoll.CHECK_FINITE)
    ctx.sync()


def test_workspace_budget_gives_nomem(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    w = workloads.c2(2, n_cells=64, per_cell=5000)
    c2 = piccoll.Context(0)          # a fresh context: no scratch yet
    try:
        c2.set_workspace_limit(1 << 20)
        tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
        with pytest.raises(piccoll.PicError) as e:
            c2.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0)
        assert e.value.status == piccoll.PIC_ERR_NOMEM
        c2.sync()
        assert np.array_equal(host(tv), w.v) and np.array_equal(host(tc), w.cell_of)
        c2.set_workspace_limit(0)
        c2.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0)
        c2.sync()
        assert not np.array_equal(host(tv), w.v)
    finally:
        c2.close()
