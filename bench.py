#!/usr/bin/env python3
"""Electron collision step throughput on one MI355X.

Workload (default): 4096 cells x 10,000 electrons (40.96M), binary32 SoA
velocities, 95% Maxwellian + 5% cold beam at 3 v_th, one step = Coulomb
(Takizuka & Abe pairing within each cell) + null-collision MCC (sigma0 E^-1/2,
P_null = 0.01) fused into the same pass, lnLambda = 10, dt = 0.01 tau_e.
Storage starts unsorted; the first warm-up step re-bins it (timed separately
as rebin_step_ms), the timed steps run on storage already in cell order, as a
step of a collision-only loop does.

Prints one JSON line: whole-job throughput (electron updates per second with
inputs resident in HBM), the dominant kernel's roofline figures from HIP
events on the library's stream, the energy drift over the timed steps, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "electron collision updates/sec at 1 MI355X; % HBM peak; energy drift"

# algorithmic bytes per electron per step (binary32 SoA)
BYTES_CHECK = 4          # order check: read cell_of
BYTES_COLLIDE = 4 + 12 + 12   # collide pass: read pid + v, write v


def energy(v):
    return float((v.double() ** 2).sum().item()) * 0.5


def copy_probe(torch, nbytes=1 << 31, iters=10):
    """Plain device copy of a known size: achievable HBM bandwidth (STREAM-style)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(iters):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / iters
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


def cpu_baseline(target_s=10.0, n_cells=512):
    """FP64 oracle on the first n_cells cells of the same workload (all host threads)."""
    import numpy as np

    import oracle
    from paper_2508_06771_amd import workloads
    w = workloads.c2(0, n_cells=n_cells, per_cell=10000)
    v = w.v.astype(np.float64)
    c, p = w.cell_of.copy(), w.pid.copy()
    oracle.step(v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=0, mcc=True,
                sigma0=w.sigma0, n_neutral=w.n_neutral)   # re-bin step, untimed
    steps, t0 = 0, time.perf_counter()
    while True:
        oracle.step(v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=1 + steps, mcc=True,
                    sigma0=w.sigma0, n_neutral=w.n_neutral)
        steps += 1
        el = time.perf_counter() - t0
        if el >= target_s and steps >= 3:
            break
    return {"value": w.n * steps / el, "unit": "electron-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n_cells} of 4096 cells x 10,000 electrons ({w.n} electrons), "
                      f"{steps} steady-state steps in {el:.1f} s, Coulomb + MCC, FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-kernel-timing", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the collision step has no cross-GPU exchange "
              "(replicated cells would add only an O(cells) all-reduce outside this path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_06771_amd import piccoll, workloads

    w = workloads.c2(0)
    v = torch.from_numpy(w.v).cuda()
    cell = torch.from_numpy(w.cell_of).cuda()
    pid = torch.from_numpy(w.pid.view(np.int32)).cuda()
    n = w.n
    del w.v
    ctx = piccoll.Context(0)
    ctx.set_mcc(w.sigma0, w.n_neutral, 0.0)
    flags = piccoll.FUSE_MCC

    def step(k):
        ctx.coulomb_collide(v, cell, pid, w.n_cells, dt=w.dt, lnL=w.lnL, seed=0, step=k,
                            flags=flags)

    torch.cuda.synchronize()
    s0, e0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    step(0)                              # re-binning step (storage starts unsorted)
    e0.record()
    ctx.sync()
    rebin_ms = s0.elapsed_time(e0)
    for k in range(1, max(args.warmup, 1)):
        step(k)
    ctx.sync()
    E0 = energy(v)
    k0 = max(args.warmup, 1)

    timing = not args.no_kernel_timing
    if timing:
        ctx.time_kernels(True)
        ctx.kernel_times()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for k in range(args.steps):
        step(k0 + k)
    e.record()
    torch.cuda.synchronize()
    ms_total = s.elapsed_time(e)
    ctx.sync()
    kt = ctx.kernel_times() if timing else {}
    ctx.time_kernels(False)
    E1 = energy(v)

    ms_step = ms_total / args.steps
    value = n / (ms_step * 1e-3)
    step_gbs = n * (BYTES_CHECK + BYTES_COLLIDE) / (ms_step * 1e-3) / 1e9

    roof = None
    if "class3" in kt:
        kms, kcnt = kt["class3"]
        kavg = kms / kcnt
        achieved = n * BYTES_COLLIDE / (kavg * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_collide<float,1024,10> (cells of 4097..10240 members)",
                "kernel_avg_ms": round(kavg, 5),
                "bytes_per_launch": n * BYTES_COLLIDE}

    copy_gbs, _ = copy_probe(torch)
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "electron-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4096 cells x 10,000 electrons (40.96M), FP32 SoA, Maxwellian + "
                               "5% cold beam, Coulomb (Takizuka-Abe) + fused null-collision MCC",
                   "n_electrons": n, "n_cells": w.n_cells, "dt_over_tau_e": 0.01,
                   "lnLambda": w.lnL, "p_null": 0.01},
        "hbm_frac_step": round(step_gbs / HBM_PEAK_GBS, 4),
        "step_algorithmic_gbs": round(step_gbs, 1),
        "algorithmic_bytes_per_electron": BYTES_CHECK + BYTES_COLLIDE,
        "copy_probe_gbs": round(copy_gbs, 1),
        "rebin_step_ms": round(rebin_ms, 4),
        "energy_drift": abs(E1 - E0) / E0,
        "kernel_ms_per_step": {k: round(t / c, 5) for k, (t, c) in kt.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
