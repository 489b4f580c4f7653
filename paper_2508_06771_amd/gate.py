"""Training and tuning of the learned sub-cycling gate (host orchestration).

Every numerical step runs in the HIP library: trajectories (coulomb_collide
with moment sums), features (pic_features), labels (pic_relaxation:
expected one-step relaxation of the temperature tensor, averaged over
re-pairings), and the network's forward, backward and Adam steps
(pic_mlp_forward / pic_mlp_train_step).  This module only loops, shuffles
sample indices and picks the decision threshold.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import piccoll

PARAMS = piccoll.MLP_PARAMS


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-initialised 8-64-64-1 network, flat binary32 layout of the library."""
    g = torch.Generator().manual_seed(seed)
    w1 = torch.randn(8, 64, generator=g) * math.sqrt(2 / 8)
    w2 = torch.randn(64, 64, generator=g) * math.sqrt(2 / 64)
    w3 = torch.randn(64, 1, generator=g) * math.sqrt(1 / 64)
    flat = torch.cat([w1.reshape(-1), torch.zeros(64), w2.reshape(-1), torch.zeros(64),
                      w3.reshape(-1), torch.zeros(1)])
    assert flat.numel() == PARAMS
    return flat.to(device=device, dtype=torch.float32).contiguous()


@dataclass
class Dataset:
    x: torch.Tensor      # (S, 8) features, device
    r: torch.Tensor      # (S,) expected relative relaxation per step, device float64


def collect(ctx: "piccoll.Context", v, cell_of, pid, n_cells: int, *, dt: float, lnL: float,
            steps: int, every: int, replicas: int = 8, seed: int = 0, step0: int = 0,
            flags: int = 0) -> Dataset:
    """Runs `steps` collision steps; every `every` steps records each cell's
    features and its relaxation label (storage stays in cell order after the
    first step)."""
    xs, rs = [], []
    mom = torch.zeros((n_cells, 14), dtype=torch.float64, device=v.device)
    ctx.set_moments_out(mom)
    for k in range(steps):
        ctx.coulomb_collide(v, cell_of, pid, n_cells, dt=dt, lnL=lnL, seed=seed, step=step0 + k,
                            flags=flags | piccoll.MOMENTS)
        if (k + 1) % every == 0:
            cs, _ = ctx.bin_cells(cell_of, n_cells)
            feat, valid = ctx.features(mom)
            r = ctx.relaxation(v, cs, pid, dt=dt, lnL=lnL, seed=seed, step=step0 + k + 1,
                               replicas=replicas)
            keep = valid.bool()
            xs.append(feat[keep].clone())
            rs.append(r[keep].clone())
    ctx.set_moments_out(None)
    return Dataset(torch.cat(xs), torch.cat(rs))


def train(ctx: "piccoll.Context", data: Dataset, tol: float, *, epochs: int = 20,
          batch: int = 4096, lr: float = 3e-3, bf16: bool = True, seed: int = 0,
          params: torch.Tensor | None = None, scale_inputs: bool = False):
    """Binary cross-entropy training of P(relaxation < tol) with Adam.
    scale_inputs: train on each feature divided by its standard deviation
    over the training set (better conditioned: the anisotropy features span
    a few hundredths), then fold the scales into the first layer's weights,
    so the returned network takes the plain features.
    Returns (params, per-epoch mean losses)."""
    y = (data.r < tol).to(torch.float32)
    S = data.x.shape[0]
    x = data.x
    if scale_inputs:
        sd = data.x.double().std(dim=0).clamp_min(1e-3).to(torch.float32)
        x = (data.x / sd).contiguous()
    params = init_params(seed, data.x.device) if params is None else params
    m = torch.zeros_like(params)
    vv = torch.zeros_like(params)
    rng = np.random.default_rng(seed)
    t, hist = 0, []
    for _ in range(epochs):
        perm = torch.from_numpy(rng.permutation(S)).to(data.x.device)
        losses = []
        for b0 in range(0, S - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = x[idx].contiguous()
            yb = y[idx].contiguous()
            t += 1
            losses.append(ctx.mlp_train_step(params, m, vv, t, lr, xb, yb, bf16=bf16))
        hist.append(float(torch.stack(losses).mean().item()))
    if scale_inputs:
        # W1 is row-major [8][64]: row i multiplies feature i
        params[:512].view(8, 64).div_(sd.view(8, 1))
    return params, hist


def tune_threshold(prob: torch.Tensor, r: torch.Tensor, tol: float, max_false: float = 0.02):
    """Smallest threshold whose skipped set has at most a max_false fraction of
    cells at or above the tolerance (on held-out samples)."""
    p = prob.double().cpu().numpy()
    bad = (r >= tol).cpu().numpy()
    order = np.argsort(-p)
    cum_bad = np.cumsum(bad[order])
    frac = cum_bad / np.arange(1, p.size + 1)
    ok = np.flatnonzero(frac <= max_false)
    if ok.size == 0:
        return 1.0
    k = ok[-1]
    return float(p[order][k]) - 1e-7
