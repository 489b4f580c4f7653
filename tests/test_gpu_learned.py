"""GPU parity of the learned sub-cycling gate against the oracle.

Features (FP32 from FP64 raw sums vs. the oracle's two-pass definition),
relaxation labels (closed-form h with erfcx vs. quadrature), the network's
forward pass and gradients (binary32 mode vs. FP64 backprop; bfloat16 mode
vs. the oracle's bfloat16-rounded FP64 backprop), Adam, and gated steps:
the first gated step equals a plain step bitwise, later steps equal the
oracle run with the gate's own skip / dt_scale decisions.
"""
import numpy as np
import pytest

import oracle
from oracle import physics
from paper_2508_06771_amd import workloads
from tests.gpu_util import dev, host, host_u32, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_06771_amd import piccoll
    c = piccoll.Context(0)
    yield c
    c.sync()
    c.close()


def sorted_workload(seed, sizes, dtype=np.float64):
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    v = workloads.maxwellian_beam(rng, sizes, dtype=dtype)
    w = workloads._finish(rng, "s", v, sizes, dtype, shuffle=False)
    cs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    return w, cs


def test_features(ctx):
    import torch
    w, cs = sorted_workload(1, [0, 1, 2, 50, 700, 3000, 12000])
    w.v[:, cs[5]:cs[6]] = workloads.bi_maxwellian(np.random.default_rng(2), 3000, 2.0, 0.5)
    mom = ctx.cell_moments(dev(w.v, torch.float64), dev(cs))
    feat, valid = ctx.features(mom)
    ctx.sync()
    ref = physics.cell_features(w.v, cs)
    ok = ~np.isnan(ref[:, 0])
    assert np.array_equal(host(valid).astype(bool), ok)
    g = host(feat)
    assert np.allclose(g[ok], ref[ok], rtol=2e-5, atol=2e-5)
    assert np.all(g[~ok] == 0)


def test_relaxation_labels(ctx):
    import torch
    w, cs = sorted_workload(3, [0, 1, 3, 40, 300, 301])
    dts = np.array([1.0, 1.0, 2.0, 1.0, 3.0, 1.0])
    r = ctx.relaxation(dev(w.v, torch.float64), dev(cs), dev(w.pid), dt=w.dt, lnL=w.lnL, seed=5,
                       step=7, replicas=3, dt_scale=dev(dts))
    ctx.sync()
    ref = physics.relaxation(w.v, cs, w.pid, dt=w.dt, lnL=w.lnL, seed=5, step=7, replicas=3,
                             dt_scale=dts)
    assert np.allclose(host(r), ref, rtol=1e-8, atol=1e-14)


def test_relaxation_labels_large_cells(ctx):
    """Cells beyond the small LDS sort (2,048 members) and beyond the large one
    (10,240 members, sorted in global scratch) give the oracle's label too."""
    import torch
    w, cs = sorted_workload(4, [2, 3000, 10300])
    r = ctx.relaxation(dev(w.v, torch.float32), dev(cs), dev(w.pid), dt=w.dt, lnL=w.lnL, seed=6,
                       step=2, replicas=1)
    ctx.sync()
    v32 = dev(w.v, torch.float32).cpu().numpy().astype(np.float64)
    ref = physics.relaxation(v32, cs, w.pid, dt=w.dt, lnL=w.lnL, seed=6, step=2, replicas=1)
    assert np.allclose(host(r), ref, rtol=1e-8, atol=1e-14)


def rand_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return physics.pack_params([rng.standard_normal(s) * scale for s in physics.mlp_init_shapes()])


GRAD_TENSORS = ("W1", "b1", "W2", "b2", "W3", "b3")


def assert_grad_elementwise(g, gr, rtol, atol_frac):
    """Every entry of every parameter tensor: |g - g_ref| <= rtol |g_ref| +
    atol_frac max |g_ref| over that tensor (so a small tensor such as the
    output bias is held to its own scale, not the whole vector's)."""
    for name, a, b in zip(GRAD_TENSORS, physics.unpack_params(np.asarray(g, np.float64)),
                          physics.unpack_params(np.asarray(gr, np.float64))):
        bound = rtol * np.abs(b) + atol_frac * np.max(np.abs(b))
        worst = np.max(np.abs(a - b) / np.maximum(bound, 1e-300))
        assert worst <= 1.0, (name, worst)


def test_mlp_forward_and_grad(ctx):
    import torch
    rng = np.random.default_rng(0)
    flat = rand_params(1)
    x = rng.standard_normal((1000, 8))
    y = (rng.uniform(size=1000) < 0.4).astype(np.float64)
    tp = dev(flat.astype(np.float32))
    tx = dev(x.astype(np.float32))
    ty = dev(y.astype(np.float32))
    x32 = x.astype(np.float32).astype(np.float64)
    p32 = flat.astype(np.float32).astype(np.float64)
    # binary32 mode vs FP64 backprop of the same (binary32-rounded) inputs
    prob = host(ctx.mlp_forward(tp, tx, bf16=False))
    g, loss = ctx.mlp_grad(tp, tx, ty, bf16=False)
    ctx.sync()
    pr, _ = physics.mlp_forward(physics.unpack_params(p32), x32)
    assert np.allclose(prob, pr, rtol=1e-5, atol=1e-6)
    lr, gr = physics.mlp_bce_grad(physics.unpack_params(p32), x32, y)
    gr = physics.pack_params(gr)
    assert np.linalg.norm(host(g) - gr) / np.linalg.norm(gr) < 1e-5
    assert_grad_elementwise(host(g), gr, rtol=1e-4, atol_frac=1e-5)
    assert abs(float(host(loss)[0]) - lr) < 1e-5 * abs(lr)
    # bfloat16 mode vs the oracle's bfloat16-rounded FP64 backprop
    prob16 = host(ctx.mlp_forward(tp, tx, bf16=True))
    g16, loss16 = ctx.mlp_grad(tp, tx, ty, bf16=True)
    ctx.sync()
    l16, gr16, pr16 = physics.mlp_bce_grad_bf16(p32, x32, y)
    assert np.max(np.abs(prob16 - pr16)) < 1e-2
    assert np.linalg.norm(host(g16) - gr16) / np.linalg.norm(gr16) < 1e-2
    assert_grad_elementwise(host(g16), gr16, rtol=3e-2, atol_frac=1e-2)
    assert abs(float(host(loss16)[0]) - l16) < 1e-2 * abs(l16)


def test_gate_infer(ctx):
    """Stand-alone decision: probabilities are the network's (binary32 mode
    against the oracle's FP64 forward of the same inputs), and skip / the
    deferred counts follow the rule exactly from the kernel's own
    probabilities over three calls (so k_max is reached)."""
    import torch
    rng = np.random.default_rng(5)
    flat = rand_params(2)
    flat[-1] = 1.5    # output bias: most cells want to skip
    x = rng.standard_normal((777, 8))
    tp = dev(flat.astype(np.float32))
    tx = dev(x.astype(np.float32))
    k = torch.zeros(777, dtype=torch.int32, device="cuda")
    k_ref = np.zeros(777, np.int64)
    thr, kmax = 0.6, 2
    pr, _ = physics.mlp_forward(physics.unpack_params(flat.astype(np.float32).astype(np.float64)),
                                x.astype(np.float32).astype(np.float64))
    sums = []
    for call in range(3):
        skip, prob = ctx.gate_infer(tx, tp, thr, kmax, k, bf16=False)
        ctx.sync()
        skip, prob, kk = host(skip).astype(bool), host(prob), host(k)
        assert np.allclose(prob, pr, rtol=1e-5, atol=1e-6)
        want = (prob > thr) & (k_ref < kmax)
        assert np.array_equal(skip, want), call
        k_ref = np.where(want, k_ref + 1, 0)
        assert np.array_equal(kk, k_ref), call
        sums.append(int(want.sum()))
    # cells that want to skip do so twice, then collide once (k_max = 2)
    assert 0 < sums[0] < 777 and sums[1] == sums[0] and sums[2] == 0


def test_adam_train_step(ctx):
    import torch
    rng = np.random.default_rng(3)
    flat = rand_params(4).astype(np.float32)
    x = rng.standard_normal((512, 8)).astype(np.float32)
    y = (rng.uniform(size=512) < 0.5).astype(np.float32)
    tp, tm, tv = dev(flat), torch.zeros(4801, device="cuda"), torch.zeros(4801, device="cuda")
    g, _ = ctx.mlp_grad(tp, dev(x), dev(y), bf16=False)
    gh = host(g).astype(np.float64)
    ctx.mlp_train_step(tp, tm, tv, 1, 1e-3, dev(x), dev(y), bf16=False)
    ctx.sync()
    out, m, v = physics.adam_update([flat.astype(np.float64)], [gh], [np.zeros(4801)],
                                    [np.zeros(4801)], 1, 1e-3)
    assert np.allclose(host(tp), out[0], rtol=1e-6, atol=1e-7)
    assert np.allclose(host(tm), m[0], rtol=1e-6, atol=1e-12)


def gated_setup(ctx, threshold):
    import torch
    w, cs = sorted_workload(5, [3000] * 24 + [0, 1, 5, 600, 2500, 5000, 9000, 12000], np.float32)
    params = dev(rand_params(6, 0.3).astype(np.float32))
    ctx.gate_config(params, threshold, k_max=3, judge_fraction=0.2, tolerance=1e-3, replicas=2)
    ctx.gate_reset()
    ctx.set_mcc(w.sigma0, 1.0, 0.0)
    return w, cs, params


def test_gated_steps_match_oracle_with_gate_decisions(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    w, cs, params = gated_setup(ctx, threshold=0.3)
    fl = piccoll.GATE | piccoll.FUSE_MCC
    tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    # step 0: no moments yet, every cell collides: equals a plain step bitwise
    pv, pc, pp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0, flags=fl)
    ctx.coulomb_collide(pv, pc, pp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0,
                        flags=piccoll.FUSE_MCC)
    ctx.sync()
    assert torch.equal(tv, pv)
    k_prev = np.zeros(w.n_cells, np.int32)
    skipped_any = False
    for step in (1, 2, 3):
        v_in = host(tv).astype(np.float64)
        _, _, _, mom_in = ctx.gate_state(w.n_cells)
        mom_in = host(mom_in)
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=step, flags=fl)
        skip, k, prob, mom = ctx.gate_state(w.n_cells)
        ctx.sync()
        skip, k, prob = host(skip).astype(bool), host(k), host(prob)
        skipped_any |= bool(skip.any())
        # the gate's probabilities are the network applied to last step's features
        feat, valid = ctx.features(dev(mom_in))
        pr = host(ctx.mlp_forward(params, feat, bf16=True))
        ctx.sync()
        vm = host(valid).astype(bool)
        assert np.allclose(prob[vm], pr[vm], atol=1e-6)
        dts = np.where(skip, 1.0, k_prev + 1.0)
        assert np.array_equal(k, np.where(skip, k_prev + 1, 0))
        vr, cr, prr = v_in.copy(), w.cell_of.copy(), w.pid.copy()
        oracle.step(vr, cr, prr, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=step, mcc=True,
                    sigma0=w.sigma0, n_neutral=1.0, skip=skip.astype(np.uint8), dt_scale=dts)
        assert rel_err(host(tv).astype(np.float64), vr) < 1e-5
        # moments for the next decision are those of the new state
        assert np.allclose(host(mom), oracle.cell_moments(host(tv).astype(np.float64), cs),
                           rtol=1e-9, atol=1e-6)
        k_prev = k
    assert skipped_any
    st = ctx.gate_stats()
    assert st["steps"] == 4 and st["have_moments"] == 1 and st["judged"] > 0


def test_gated_graph_equals_eager(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    fl = piccoll.GATE | piccoll.FUSE_MCC
    w, cs, params = gated_setup(ctx, threshold=0.3)
    A = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
    ctx.run_steps(*A, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step0=0, nsteps=5, flags=fl)
    ctx.sync()
    sa = ctx.gate_stats()
    w, cs, params = gated_setup(ctx, threshold=0.3)
    B = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
    for k in range(5):
        ctx.coulomb_collide(*B, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step=k, flags=fl)
    ctx.sync()
    assert torch.equal(A[0], B[0])
    assert ctx.gate_stats() == sa


def test_gate_moment_refresh_interval(ctx):
    """With a refresh interval of 3 the gate's moment sums are those of the
    post-step state on the first gated step and every third step, and are
    left as they were in between."""
    import torch
    from paper_2508_06771_amd import piccoll
    w, cs, params = gated_setup(ctx, threshold=0.3)
    ctx.gate_refresh(3)
    try:
        fl = piccoll.GATE | piccoll.FUSE_MCC
        tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
        last = None
        for step in range(7):
            ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=step,
                                flags=fl)
            _, _, _, mom = ctx.gate_state(w.n_cells)
            ctx.sync()
            mom = host(mom)
            if step == 0 or step % 3 == 0:
                ref = oracle.cell_moments(host(tv).astype(np.float64), cs)
                assert np.allclose(mom, ref, rtol=1e-9, atol=1e-6), step
            else:
                assert np.array_equal(mom, last), step
            last = mom
    finally:
        ctx.gate_refresh(1)


def test_gate_switches_off_on_false_skips(ctx):
    """A gate that skips everything (threshold 0) on anisotropic cells is
    judged wrong and switches itself off; then every cell collides."""
    import torch
    from paper_2508_06771_amd import piccoll
    rng = np.random.default_rng(8)
    sizes = np.full(400, 2000)
    v = workloads.bi_maxwellian(rng, int(sizes.sum()), t_par=3.0, t_perp=0.5, dtype=np.float32)
    w = workloads._finish(rng, "a", v, sizes, np.float32, shuffle=False)
    params = dev(rand_params(9).astype(np.float32))
    params[4800] = 50.0     # logit bias: probability ~1 for every cell
    ctx.gate_config(params, 0.0, k_max=8, judge_fraction=0.25, tolerance=1e-4, replicas=1)
    ctx.gate_reset()
    tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    for k in range(3):
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=3, step=k,
                            flags=piccoll.GATE)
    st = ctx.gate_stats()
    assert st["disabled"] == 1 and st["false_skip"] > 0
    before = st["collided"]
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=3, step=3, flags=piccoll.GATE)
    assert ctx.gate_stats()["collided"] - before == w.n_cells


def _tpar_over_tperp(v, cs):
    """Per-cell T_par / T_perp (z parallel) of storage in cell order, FP64."""
    v = v.astype(np.float64)
    N = np.diff(cs).astype(np.float64)
    s1 = np.add.reduceat(v, cs[:-1], axis=1) / N
    s2 = np.add.reduceat(v * v, cs[:-1], axis=1) / N
    T = s2 - s1 * s1
    return T[2] / (0.5 * (T[0] + T[1]))


def test_trained_gate_gains_over_plain(ctx, tmp_path):
    """What the trained network gains over the plain operator.  A gate is
    trained here on the GPU by the library's own kernels (the trainer's
    default trajectories of the Maxwellian + beam workload), then the same 24
    steps run from the same mixed-cell state (32,768 cells x 2,000 electrons:
    70% near-Maxwellian, 15% Maxwellian + beam, 15% anisotropic) plainly and
    gated, as graph replays: the gate defers a large share of the cell-steps
    and the gated steps take less wall time, with an energy drift no worse than
    plain's and the anisotropic cells' T_par / T_perp relaxing as in the plain
    run to within 3% of the relaxation itself."""
    import json
    import torch
    from paper_2508_06771_amd import piccoll, train_gate
    out = tmp_path / "gate.npy"
    train_gate.main(["--out", str(out)])
    params = dev(np.load(out))
    meta = json.load(open(tmp_path / "gate.json"))
    w = workloads.c5(3, n_cells=32768)
    K = 24
    res = {}
    try:
        for mode in ("plain", "gated"):
            v, c, p = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
            fl = 0
            if mode == "gated":
                ctx.gate_config(params, meta["threshold"], k_max=8, judge_fraction=0.01,
                                tolerance=meta["tolerance"], replicas=8, bf16=True)
                ctx.gate_refresh(4)
                ctx.gate_reset()
                fl = piccoll.GATE
            ctx.coulomb_collide(v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0, flags=fl)
            ctx.sync()
            cs = np.concatenate([[0], np.cumsum(np.bincount(host(c), minlength=w.n_cells))])
            v0 = host(v)
            # warm the graph, then time K replays from the same state
            st0 = ctx.gate_stats() if mode == "gated" else None
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.run_steps(v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step0=1, nsteps=K,
                          flags=fl | piccoll.ASSUME_SORTED)
            e1.record()
            ctx.sync()
            torch.cuda.synchronize()
            v1 = host(v)
            en0 = (v0.astype(np.float64) ** 2).sum()
            res[mode] = {
                "ms": e0.elapsed_time(e1) / K,
                "drift": abs((v1.astype(np.float64) ** 2).sum() - en0) / en0,
                "r0": _tpar_over_tperp(v0, cs), "r1": _tpar_over_tperp(v1, cs),
                "stats": ctx.gate_stats() if mode == "gated" else None,
                "stats0": st0,
            }
    finally:
        ctx.gate_refresh(1)
    g, pl = res["gated"], res["plain"]
    st, s0 = g["stats"], g["stats0"]
    sk = st["skipped"] - s0["skipped"]
    skipped = sk / (sk + st["collided"] - s0["collided"])
    print("trained gate:", meta, "skipped", skipped, "ms/step gated", g["ms"], "plain", pl["ms"],
          "drift", g["drift"], pl["drift"], flush=True)
    assert st["disabled"] == 0
    assert skipped > 0.2, skipped
    assert g["ms"] < 0.95 * pl["ms"], (g["ms"], pl["ms"])
    assert g["drift"] <= max(2.0 * pl["drift"], 1e-6), (g["drift"], pl["drift"])
    aniso = w.meta["kind"] == 2
    relax = np.abs(pl["r1"] - pl["r0"])[aniso].mean()
    diff = np.abs(g["r1"] - pl["r1"])[aniso].mean()
    assert diff < 0.03 * relax, (diff, relax)


# ---------------------------------------------------------------- analytic gate


def test_analytic_relaxation_matches_oracle(ctx):
    """The moment-based relaxation estimate from the library's FP64 one-pass
    sums against the oracle's two-pass features: ragged and degenerate cells
    (0, 1 and 2 members give NaN or a value as the oracle does), densities."""
    import torch
    w, cs = sorted_workload(9, [0, 1, 2, 37, 500, 2000, 3000, 777, 4097, 10001], np.float32)
    dens = np.linspace(0.5, 2.0, w.n_cells)
    tv = dev(w.v, torch.float32)
    mom = ctx.cell_moments(tv, dev(cs))
    for K, d in ((8, None), (2, dens)):
        r = host(ctx.analytic_relaxation(mom, dt=w.dt, lnL=w.lnL, replicas=K,
                                         density=None if d is None else dev(d)))
        ctx.sync()
        ref = physics.analytic_relaxation(w.v.astype(np.float64), cs, dt=w.dt, lnL=w.lnL,
                                          replicas=K, density=d)
        assert np.array_equal(np.isnan(r), np.isnan(ref))
        ok = ~np.isnan(ref)
        assert ok.sum() >= 8
        assert np.allclose(r[ok], ref[ok], rtol=1e-8, atol=0)


def test_analytic_gate_decisions_and_steps(ctx):
    """The analytic gate: its stored score is the estimate over the tolerance
    from last step's moments, a cell is skipped only when that score is below
    the threshold (and not judged, and under k_max), and the step equals the
    oracle run with the gate's own skip / dt_scale decisions."""
    import torch
    from paper_2508_06771_amd import piccoll
    w, cs = sorted_workload(5, [3000] * 24 + [0, 1, 5, 600, 2500, 5000, 9000, 12000], np.float32)
    ctx.gate_config_analytic(1.0, k_max=3, judge_fraction=0.2, tolerance=1e-3, replicas=2)
    ctx.gate_reset()
    ctx.set_mcc(w.sigma0, 1.0, 0.0)
    fl = piccoll.GATE | piccoll.FUSE_MCC
    tv, tc, tp = dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)
    ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=0, flags=fl)
    _, _, _, mom0 = ctx.gate_state(w.n_cells)
    q0 = host(ctx.analytic_relaxation(mom0, dt=w.dt, lnL=w.lnL, replicas=2)) / 1e-3
    ctx.sync()
    thr = float(np.nanmedian(q0))
    ctx.gate_config_analytic(thr, k_max=3, judge_fraction=0.2, tolerance=1e-3, replicas=2)
    k_prev = np.zeros(w.n_cells, np.int32)
    skipped_any = False
    try:
        for step in (1, 2, 3):
            v_in = host(tv).astype(np.float64)
            _, _, _, mom_in = ctx.gate_state(w.n_cells)
            r_in = host(ctx.analytic_relaxation(mom_in, dt=w.dt, lnL=w.lnL, replicas=2))
            ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=step,
                                flags=fl)
            skip, k, prob, mom = ctx.gate_state(w.n_cells)
            ctx.sync()
            skip, k, prob = host(skip).astype(bool), host(k), host(prob)
            valid = ~np.isnan(r_in)
            assert np.allclose(prob[valid], r_in[valid] / 1e-3, rtol=1e-6, atol=0)
            assert np.all(prob[~valid] == 0.0)
            want = valid & (prob < np.float32(thr)) & (k_prev < 3)
            assert not np.any(skip & ~want)
            assert (want & ~skip).sum() <= 0.5 * max(1, want.sum())   # judged: 20% of cells
            skipped_any |= bool(skip.any())
            dts = np.where(skip, 1.0, k_prev + 1.0)
            assert np.array_equal(k, np.where(skip, k_prev + 1, 0))
            vr, cr, prr = v_in.copy(), w.cell_of.copy(), w.pid.copy()
            oracle.step(vr, cr, prr, w.n_cells, dt=w.dt, lnL=w.lnL, seed=1, step=step, mcc=True,
                        sigma0=w.sigma0, n_neutral=1.0, skip=skip.astype(np.uint8), dt_scale=dts)
            assert rel_err(host(tv).astype(np.float64), vr) < 1e-5
            k_prev = k
        assert skipped_any
        st = ctx.gate_stats()
        assert st["steps"] == 4 and st["judged"] > 0
    finally:
        ctx.gate_reset()


def test_analytic_gate_graph_equals_eager(ctx):
    import torch
    from paper_2508_06771_amd import piccoll
    fl = piccoll.GATE | piccoll.FUSE_MCC
    w, cs = sorted_workload(7, [3000] * 24 + [0, 1, 5, 600, 2500, 5000, 9000, 12000], np.float32)
    ctx.set_mcc(w.sigma0, 1.0, 0.0)
    out = []
    for graph in (True, False):
        ctx.gate_config_analytic(1e3, k_max=3, judge_fraction=0.2, tolerance=1e-3, replicas=2)
        ctx.gate_reset()
        A = [dev(w.v, torch.float32), dev(w.cell_of), dev(w.pid)]
        if graph:
            ctx.run_steps(*A, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step0=0, nsteps=5, flags=fl)
        else:
            for k in range(5):
                ctx.coulomb_collide(*A, w.n_cells, dt=w.dt, lnL=w.lnL, seed=2, step=k, flags=fl)
        ctx.sync()
        out.append((A[0], ctx.gate_stats()))
    assert torch.equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]
    assert out[0][1]["skipped"] > 0
    ctx.gate_reset()


def test_short_form_train_step_counts_adam_steps(ctx):
    """mlp_train_step equals pic_mlp_train_step (bf16) with t = 1, 2, ... on the
    same parameters, and restarts at t = 1 for another parameter array."""
    import torch
    rng = np.random.default_rng(8)
    flat = rand_params(9).astype(np.float32)
    x = dev(rng.standard_normal((700, 8)).astype(np.float32))
    y = dev((rng.uniform(size=700) < 0.6).astype(np.float32))
    pa, state = dev(flat), torch.zeros(2 * 4801, device="cuda")
    pb, m, v = dev(flat), torch.zeros(4801, device="cuda"), torch.zeros(4801, device="cuda")
    for t in (1, 2, 3):
        la = ctx.train_step(x, y, pa, state, 2e-3)
        lb = ctx.mlp_train_step(pb, m, v, t, 2e-3, x, y, bf16=True)
        ctx.sync()
        assert torch.equal(pa, pb) and torch.equal(la, lb)
        assert torch.equal(state[:4801], m) and torch.equal(state[4801:], v)
    pc, state_c = dev(flat), torch.zeros(2 * 4801, device="cuda")
    pd, md, vd = dev(flat), torch.zeros(4801, device="cuda"), torch.zeros(4801, device="cuda")
    ctx.train_step(x, y, pc, state_c, 2e-3)
    ctx.mlp_train_step(pd, md, vd, 1, 2e-3, x, y, bf16=True)
    ctx.sync()
    assert torch.equal(pc, pd)


def test_gated_binary64_large_cells_match_oracle(ctx):
    """Binary64 gated steps on cells of the binary64 lean pass (4,097..10,240
    members) and smaller ones: the deferred cells' accumulated time step
    (dt_scale) and the skips are applied as the oracle applies the gate's own
    decisions, to 1e-12."""
    import torch
    from paper_2508_06771_amd import piccoll
    w, cs = sorted_workload(12, [6000] * 6 + [9000, 4500, 10240, 3000, 0, 1, 7], np.float64)
    ctx.gate_config_analytic(1e3, k_max=2, judge_fraction=0.2, tolerance=1e-3, replicas=2)
    ctx.gate_reset()
    ctx.set_mcc(w.sigma0, 1.0, 0.0)
    fl = piccoll.GATE | piccoll.FUSE_MCC
    tv, tc, tp = dev(w.v, torch.float64), dev(w.cell_of), dev(w.pid)
    k_prev = np.zeros(w.n_cells, np.int32)
    try:
        ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=3, step=0, flags=fl)
        ctx.sync()
        skipped_any = collided_late = False
        for step in (1, 2, 3, 4):
            v_in = host(tv).copy()
            ctx.coulomb_collide(tv, tc, tp, w.n_cells, dt=w.dt, lnL=w.lnL, seed=3, step=step,
                                flags=fl)
            skip, k, _, _ = ctx.gate_state(w.n_cells)
            ctx.sync()
            skip, k = host(skip).astype(bool), host(k)
            skipped_any |= bool(skip.any())
            collided_late |= bool((~skip & (k_prev > 0)).any())
            dts = np.where(skip, 1.0, k_prev + 1.0)
            vr, cr, prr = v_in.copy(), w.cell_of.copy(), w.pid.copy()
            oracle.step(vr, cr, prr, w.n_cells, dt=w.dt, lnL=w.lnL, seed=3, step=step, mcc=True,
                        sigma0=w.sigma0, n_neutral=1.0, skip=skip.astype(np.uint8), dt_scale=dts)
            assert rel_err(host(tv), vr) < 1e-12, step
            k_prev = k
        assert skipped_any and collided_late
    finally:
        ctx.gate_reset()
