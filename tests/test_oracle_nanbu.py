"""Pins of the oracle's Nanbu Coulomb operator.

* The deflection's cosine has mean exp(-s) (a property of Nanbu's
  distribution, checked on samples), and its distribution function is
  (exp(A c) - exp(-A)) / (2 sinh A) (Kolmogorov-Smirnov).
* A(s) tends to 1/s for small s and to 3 exp(-s) for large s.
* Each pair keeps its momentum and kinetic energy.
* With s = 2 s2 (s2 the Takizuka-Abe variance) the initial isotropisation of
  a bi-Maxwellian follows the same rate ODE as the Takizuka-Abe operator
  (within 3% at dt = 0.001 tau_e): the reading of s is pinned by the
  physics, not by the code.
* A Maxwellian stays Maxwellian.
"""
import math

import numpy as np
from scipy import stats

import oracle
from oracle import physics
from paper_2508_06771_amd import workloads


def cos_samples(s, m=40_000, seed=0):
    A = oracle.nanbu_A(s)
    U = (np.random.default_rng(seed).integers(0, 2 ** 23, m) + 0.5) / 2 ** 23
    return A, 1.0 - np.array([oracle.nanbu_omc(A, float(u)) for u in U])


def test_mean_cosine_is_exp_minus_s():
    for s in (0.003, 0.05, 0.3, 1.0, 2.5, 6.0, 15.0):
        A, c = cos_samples(s)
        sd = c.std() / math.sqrt(c.size)
        assert abs(c.mean() - math.exp(-s)) < 5 * sd + 1e-12, (s, c.mean(), math.exp(-s))


def test_cosine_distribution_ks():
    for s in (0.1, 1.0, 4.0):
        A, c = cos_samples(s, m=20_000, seed=1)

        def cdf(x):
            return np.expm1(A * (x + 1.0)) / np.expm1(2.0 * A)

        assert stats.kstest(c, cdf).pvalue > 1e-4


def test_limits_of_A():
    for s in (1e-6, 1e-4, 1e-3):
        assert math.isclose(oracle.nanbu_A(s), 1.0 / s, rel_tol=2 * s)
    for s in (12.0, 20.0, 40.0):
        assert math.isclose(oracle.nanbu_A(s), 3.0 * math.exp(-s), rel_tol=1e-8)


def sorted_population(w):
    order = np.argsort(w.cell_of, kind="stable")
    v = np.ascontiguousarray(w.v[:, order], dtype=np.float64)
    pid = w.pid[order]
    cs = np.searchsorted(w.cell_of[order], np.arange(w.n_cells + 1)).astype(np.int32)
    return v, pid, cs


def test_pair_conservation():
    w = workloads.c1(3, n_cells=16)
    v, pid, cs = sorted_population(w)
    v0 = v.copy()
    oracle.nanbu(v, cs, pid, 0.05, 10.0, 7, 1)
    sorted_, partner = oracle.pairs(cs, pid, 7, 1)
    a = np.nonzero(partner > np.arange(v.shape[1]))[0]
    b = partner[a]
    assert np.any(v != v0)
    p0, p1 = v0[:, a] + v0[:, b], v[:, a] + v[:, b]
    assert np.max(np.abs(p1 - p0)) < 1e-13 * (1 + np.max(np.abs(p0)))
    e0 = (v0[:, a] ** 2).sum(0) + (v0[:, b] ** 2).sum(0)
    e1 = (v[:, a] ** 2).sum(0) + (v[:, b] ** 2).sum(0)
    assert np.max(np.abs(e1 / e0 - 1)) < 1e-13


def temperatures(v):
    c = v - v.mean(axis=1, keepdims=True)
    return float(np.mean(c[2] ** 2)), float(0.5 * np.mean(c[0] ** 2 + c[1] ** 2))


def test_initial_relaxation_matches_rate():
    dt = 0.1 * workloads.DT
    w = workloads.c1(0, n_cells=2000)
    v, pid, cs = sorted_population(w)
    t0 = temperatures(v)
    for k in range(50):
        oracle.nanbu(v, cs, pid, dt, w.lnL, 0, k)
    t1 = temperatures(v)
    opa, ope = physics.isotropisation_rk4(t0[0], t0[1], dt, 50)
    m = (t1[0] - t1[1]) - (t0[0] - t0[1])
    o = (opa[-1] - ope[-1]) - (opa[0] - ope[0])
    assert abs(m / o - 1) < 0.03, m / o


def test_maxwellian_is_stationary():
    rng = np.random.default_rng(5)
    M, per = 64, 256
    v = rng.standard_normal((3, M * per))
    cs = np.arange(0, M * per + 1, per, dtype=np.int32)
    pid = np.arange(M * per, dtype=np.uint32)
    for k in range(50):
        oracle.nanbu(v, cs, pid, workloads.DT, 10.0, 2, k)
    for i in range(3):
        assert stats.kstest(v[i], "norm").pvalue > 1e-3
