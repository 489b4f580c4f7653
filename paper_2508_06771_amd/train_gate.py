"""Trains the learned sub-cycling gate on the GPU, on trajectories of the
Maxwellian + cold-beam workload (Coulomb + null collisions) and of the mixed
workload (near-Maxwellian, beam and bi-Maxwellian cells; Coulomb only).

    python -m paper_2508_06771_amd.train_gate --out paper_2508_06771_amd/gate_params.npy

Samples: every `--every` steps, each cell's eight features and its expected
one-step relaxation r (pic_relaxation, averaged over re-pairings).  Two
Maxwellian + beam trajectories with 10,000 and 2,000 electrons per cell and
one mixed trajectory with 2,000 (seed 2: the mixed workload's seed 0 is the
benchmark's and seed 1 its threshold calibration's) cover the cell
populations the gate is used on.  Label: r < tolerance.
The network is trained with binary cross-entropy and Adam (bfloat16
products, binary32 master weights); the skip threshold is the smallest one
whose skipped held-out cells contain at most `--max-false` cells at or above
the tolerance.  Writes the parameters (.npy, binary32) and a JSON summary.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import gate, piccoll, workloads


def trajectory(ctx, n_cells, per_cell, steps, every, replicas, seed):
    w = workloads.c2(seed, n_cells=n_cells, per_cell=per_cell)
    v = torch.from_numpy(w.v).cuda()
    c = torch.from_numpy(w.cell_of).cuda()
    p = torch.from_numpy(w.pid.view(np.int32)).cuda()
    ctx.set_mcc(w.sigma0, w.n_neutral, 0.0)
    return gate.collect(ctx, v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, steps=steps, every=every,
                        replicas=replicas, seed=seed, flags=piccoll.FUSE_MCC)


def mixed_trajectory(ctx, n_cells, steps, every, replicas, seed):
    w = workloads.c5(seed, n_cells=n_cells)
    v = torch.from_numpy(w.v).cuda()
    c = torch.from_numpy(w.cell_of).cuda()
    p = torch.from_numpy(w.pid.view(np.int32)).cuda()
    return gate.collect(ctx, v, c, p, w.n_cells, dt=w.dt, lnL=w.lnL, steps=steps, every=every,
                        replicas=replicas, seed=seed)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "gate_params.npy"))
    ap.add_argument("--cells", type=int, default=512)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--replicas", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--max-false", type=float, default=0.02)
    ap.add_argument("--mixed-cells", type=int, default=8192,
                    help="cells of the mixed-workload trajectory (0: none)")
    args = ap.parse_args(argv)
    t0 = time.time()
    ctx = piccoll.Context(0)
    parts = [trajectory(ctx, args.cells, 10000, args.steps, args.every, args.replicas, 1),
             trajectory(ctx, 4 * args.cells, 2000, args.steps, args.every, args.replicas, 2)]
    if args.mixed_cells:
        parts.append(mixed_trajectory(ctx, args.mixed_cells, args.steps, args.every, args.replicas, 2))
    data = gate.Dataset(torch.cat([d.x for d in parts]), torch.cat([d.r for d in parts]))
    ctx.sync()
    S = data.x.shape[0]
    rng = np.random.default_rng(0)
    perm = torch.from_numpy(rng.permutation(S)).cuda()
    nval = S // 5
    val, tr = perm[:nval], perm[nval:]
    dtr = gate.Dataset(data.x[tr].contiguous(), data.r[tr].contiguous())
    dva = gate.Dataset(data.x[val].contiguous(), data.r[val].contiguous())
    params, hist = gate.train(ctx, dtr, args.tol, epochs=args.epochs, batch=args.batch,
                              lr=args.lr, bf16=True, seed=0, scale_inputs=True)
    prob = ctx.mlp_forward(params, dva.x, bf16=True)
    ctx.sync()
    yv = (dva.r < args.tol).cpu().numpy()
    pv = prob.cpu().numpy()
    acc = float(((pv > 0.5) == yv).mean())
    thr = gate.tune_threshold(prob, dva.r, args.tol, args.max_false)
    skip = pv > thr
    summary = {
        "samples": S, "parts": [int(d.x.shape[0]) for d in parts], "train": int(tr.numel()), "val": int(nval),
        "label_positive_fraction": float((data.r < args.tol).float().mean().item()),
        "tolerance": args.tol, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
        "val_accuracy_at_0.5": acc, "majority_baseline": float(max(yv.mean(), 1 - yv.mean())),
        "threshold": thr, "val_skip_fraction": float(skip.mean()),
        "val_false_skip_fraction": float((~yv[skip]).mean()) if skip.any() else 0.0,
        "seconds": time.time() - t0,
    }
    np.save(args.out, params.cpu().numpy().astype(np.float32))
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
