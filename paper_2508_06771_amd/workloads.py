"""Seeded synthetic particle populations for the electron collision step.

This module holds no part of the collision method: it only draws initial
velocities and cell assignments with numpy's PCG64 generator, so that the
GPU library and the FP64 oracle can be fed the same inputs.  The populations
stand in for the paper's argon discharge workloads (whose cross-section data
are not available); their shapes follow the paper's regime of many particles
per cell (hundreds to tens of thousands).

Velocities are in units of the thermal speed, v_th = sqrt(T/m) = 1, so a
Maxwellian has unit variance per component.  Storage starts in a random
order (unsorted particles, as the paper's solver keeps them): cell ids are a
random permutation of the repeated cell ids, and pid[l] = l.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def tau_e(T: float = 1.0, n: float = 1.0, lnL: float = 10.0) -> float:
    """Braginskii electron collision time in code units (m_e = 1, e^4 = 1)."""
    return 3.0 * T ** 1.5 / (4.0 * math.sqrt(2.0 * math.pi) * n * lnL)


LNL = 10.0
DT = 0.01 * tau_e(1.0, 1.0, LNL)           # 2.992067e-4
P_NULL = 0.01                               # null-collision probability per step
SIGMA0 = -math.log1p(-P_NULL) / (math.sqrt(2.0) * DT)   # with n_neutral = 1
N_NEUTRAL = 1.0


@dataclass
class Workload:
    name: str
    v: np.ndarray            # (3, n) SoA
    cell_of: np.ndarray      # int32 (n,)
    pid: np.ndarray          # uint32 (n,)
    n_cells: int
    dt: float = DT
    lnL: float = LNL
    mcc: bool = False
    sigma0: float = SIGMA0
    n_neutral: float = N_NEUTRAL
    mass_ratio: float = 0.0
    steps: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.cell_of.size)


def _finish(rng, name, v_cellorder, counts, dtype, shuffle=True, **kw):
    n = int(counts.sum())
    cell = np.repeat(np.arange(counts.size, dtype=np.int32), counts)
    if shuffle and n > 0:
        perm = rng.permutation(n)
        cell = cell[perm]
        v = np.empty((3, n), dtype=dtype)
        for c in range(3):
            v[c] = v_cellorder[c][perm]
    else:
        v = np.ascontiguousarray(v_cellorder, dtype=dtype)
    pid = np.arange(n, dtype=np.uint32)
    return Workload(name=name, v=np.ascontiguousarray(v), cell_of=np.ascontiguousarray(cell),
                    pid=pid, n_cells=int(counts.size), **kw)


def bi_maxwellian(rng, n, t_par=1.5, t_perp=0.75, dtype=np.float64):
    """Zero-drift bi-Maxwellian, parallel axis z.  The defaults give
    T_par = 2 T_perp with (T_par + 2 T_perp) / 3 = 1."""
    v = rng.standard_normal((3, n), dtype=np.float64)
    v[0:2] *= math.sqrt(t_perp)
    v[2] *= math.sqrt(t_par)
    return v.astype(dtype, copy=False)


def c1(seed: int = 0, n_cells: int = 64, per_cell: int = 256, dtype=np.float64) -> Workload:
    """64 cells x 256 electrons, bi-Maxwellian T_par = 2 T_perp, 100 steps."""
    rng = np.random.default_rng(seed)
    counts = np.full(n_cells, per_cell, dtype=np.int64)
    v = bi_maxwellian(rng, int(counts.sum()), dtype=dtype)
    return _finish(rng, "c1_bimaxwellian", v, counts, dtype, steps=100)


def maxwellian_beam(rng, counts, beam_frac=0.05, beam_v=3.0, dtype=np.float32):
    """Per cell: (1 - beam_frac) isotropic unit Maxwellian + beam_frac cold
    beam at v = (0, 0, beam_v) (zero spread)."""
    n = int(counts.sum())
    v = rng.standard_normal((3, n), dtype=np.float32 if dtype == np.float32 else np.float64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    nb = np.rint(counts * beam_frac).astype(np.int64)
    # beam members: the last nb[j] slots of every cell
    mask = np.zeros(n, dtype=bool)
    idx = np.repeat(starts + counts - nb, nb) + (np.arange(nb.sum()) - np.repeat(
        np.concatenate([[0], np.cumsum(nb)[:-1]]), nb))
    mask[idx] = True
    v[0, mask] = 0.0
    v[1, mask] = 0.0
    v[2, mask] = beam_v
    return v.astype(dtype, copy=False)


def c2(seed: int = 0, n_cells: int = 4096, per_cell: int = 10000, dtype=np.float32) -> Workload:
    """4096 cells x 10,000 electrons: 95% Maxwellian + 5% cold beam at 3 v_th,
    Coulomb + null-collision MCC with sigma = sigma0 E^-1/2, 1000 steps."""
    rng = np.random.default_rng(seed)
    counts = np.full(n_cells, per_cell, dtype=np.int64)
    v = maxwellian_beam(rng, counts, dtype=dtype)
    return _finish(rng, "c2_maxwellian_beam", v, counts, dtype, mcc=True, steps=1000)


C3_SIGMA = 0.9193


def c3_counts(rng, n_cells=16384, median=2000, sigma=C3_SIGMA, lo=10, hi=200000):
    z = rng.standard_normal(n_cells)
    return np.clip(np.rint(median * np.exp(sigma * z)), lo, hi).astype(np.int64)


def c3(seed: int = 0, n_cells: int = 16384, median: int = 2000, hi: int = 200000,
       dtype=np.float32) -> Workload:
    """Log-normal cell populations (median 2000, clipped to [10, 200000]),
    Maxwellian + beam velocities as in c2."""
    rng = np.random.default_rng(seed)
    counts = c3_counts(rng, n_cells, median=median, hi=hi)
    v = maxwellian_beam(rng, counts, dtype=dtype)
    return _finish(rng, "c3_lognormal_cells", v, counts, dtype, mcc=True, steps=1)


def c4(seed: int = 0, n_cells: int = 32768, per_cell: int = 3052, dtype=np.float32) -> Workload:
    """32,768 cells x 3,052 electrons, the c1 bi-Maxwellian, 10,000 steps."""
    rng = np.random.default_rng(seed)
    counts = np.full(n_cells, per_cell, dtype=np.int64)
    v = bi_maxwellian(rng, int(counts.sum()), dtype=dtype)
    return _finish(rng, "c4_precision", v, counts, dtype, steps=10000)


def c5(seed: int = 0, n_cells: int = 65536, per_cell: int = 2000, dtype=np.float32) -> Workload:
    """70% near-Maxwellian cells (T_par / T_perp ~ U[1, 1.05]); 15% Maxwellian
    + 5% beam; 15% bi-Maxwellian with T_par / T_perp ~ U[1, 4] (along z).
    Per-cell temperature normalised to (T_par + 2 T_perp) / 3 = 1."""
    rng = np.random.default_rng(seed)
    counts = np.full(n_cells, per_cell, dtype=np.int64)
    kind = rng.choice(3, size=n_cells, p=[0.70, 0.15, 0.15])
    ratio = np.where(kind == 0, rng.uniform(1.0, 1.05, n_cells),
                     np.where(kind == 2, rng.uniform(1.0, 4.0, n_cells), 1.0))
    t_perp = 3.0 / (ratio + 2.0)
    t_par = ratio * t_perp
    n = int(counts.sum())
    v = rng.standard_normal((3, n), dtype=np.float64)
    sp = np.repeat(np.sqrt(t_perp), counts)
    sz = np.repeat(np.sqrt(t_par), counts)
    v[0] *= sp
    v[1] *= sp
    v[2] *= sz
    beam_cells = np.flatnonzero(kind == 1)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    nb = int(round(per_cell * 0.05))
    for j in beam_cells:
        e = starts[j] + counts[j]
        v[0:2, e - nb:e] = 0.0
        v[2, e - nb:e] = 3.0
    w = _finish(rng, "c5_mixed_cells", v.astype(dtype), counts, dtype, mcc=False, steps=1)
    w.meta["kind"] = kind
    w.meta["ratio"] = ratio
    return w


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


def dsmc_table() -> dict:
    """Synthetic cross sections for the electron-heavy channels C1..C4 (the
    paper's argon cross sections come from LXCat, not available here), in
    code units (E = |v|^2 / 2 with thermal speed 1): thresholds in the ratio
    of argon's 11.55 / 15.76 / 4.21 eV (excitation / ionization / two-step
    ionization) with the two-step threshold at E = 1; a Ramsauer-like elastic
    minimum.  Piecewise cubic Hermite on shared breakpoints:
    coef[c, p, q] multiplies (E - breaks[p])^q."""
    breaks = np.array([0.0, 0.25, 0.5, 1.0, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0])
    thr = np.array([0.0, 3.74, 2.74, 1.0])
    y = np.array([
        [2.0, 0.8, 0.5, 1.0, 2.0, 2.5, 2.2, 1.8, 1.5, 1.2, 1.0],      # C1 elastic
        [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.05, 0.3, 0.5, 0.7, 0.75],     # C2 ionization
        [0.0, 0.0, 0.0, 0.0, 0.0, 0.02, 0.15, 0.3, 0.32, 0.28, 0.25],  # C3 excitation
        [0.0, 0.0, 0.0, 0.0, 1.0, 1.5, 1.6, 1.5, 1.3, 1.1, 1.0],       # C4 two-step ionization
    ])
    P = breaks.size - 1
    coef = np.zeros((4, P, 4))
    for c in range(4):
        m = np.gradient(y[c], breaks)
        for p in range(P):
            h = breaks[p + 1] - breaks[p]
            d = (y[c, p + 1] - y[c, p]) / h
            coef[c, p] = [y[c, p], m[p], (3 * d - 2 * m[p] - m[p + 1]) / h,
                          (m[p] + m[p + 1] - 2 * d) / (h * h)]
    return {"breaks": breaks, "coef": coef, "thr": thr}
