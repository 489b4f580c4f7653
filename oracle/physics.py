"""Closed forms, quadratures and small dense references in plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Braginskii electron collision time and the temperature-isotropisation rate
  of a bi-Maxwellian (NRL Plasma Formulary, relaxation rates), integrated
  with classical RK4.  These pin the Takizuka & Abe operator's rate.
* Moments of the Takizuka & Abe scattering angle over the Gaussian delta:
  g(s2) = E[1 - cos Theta] and h(s2) = E[sin^2 Theta], by adaptive
  quadrature.
* Per-cell features (eight Galilean-invariant moments) computed directly
  from velocities with a two-pass central-moment definition.
* The learned-gate label: the expected one-step change of a cell's
  temperature tensor, averaged over independent re-pairings; and its
  estimate from the moments alone (the analytic gate).
* A dense FP64 reference of the 8-64-64-1 gate network: forward, binary
  cross-entropy, backward by the chain rule, and Adam.

Code units: m_e = 1, (e^2 / 4 pi eps0)^2 = 1, temperatures as m <v_i^2>.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate

# ---------------------------------------------------------------- rates


def tau_e(T: float = 1.0, n: float = 1.0, lnL: float = 10.0) -> float:
    """Braginskii electron collision time 3 sqrt(m) T^1.5 / (4 sqrt(2 pi) n e^4 lnL)."""
    return 3.0 * T ** 1.5 / (4.0 * math.sqrt(2.0 * math.pi) * n * lnL)


def nu_isotropisation(Tpar: float, Tperp: float, n: float = 1.0, lnL: float = 10.0) -> float:
    """Relaxation rate nu_T of dT_perp/dt = -nu_T (T_perp - T_par) for like
    particles: 2 sqrt(pi) n lnL / (sqrt(m) T_par^1.5) * A^-2 [-3 + (A+3) F(A)],
    A = T_perp / T_par - 1, F = atan(sqrt A)/sqrt A (A > 0) or
    atanh(sqrt(-A))/sqrt(-A) (A < 0)."""
    A = Tperp / Tpar - 1.0
    pref = 2.0 * math.sqrt(math.pi) * n * lnL / Tpar ** 1.5
    if abs(A) < 1e-4:
        # series of A^-2 [-3 + (A+3) F(A)] = 4/15 - 8 A / 35 + ...
        return pref * (4.0 / 15.0 - 8.0 * A / 35.0 + 4.0 * A * A / 21.0)
    if A > 0:
        F = math.atan(math.sqrt(A)) / math.sqrt(A)
    else:
        F = math.atanh(math.sqrt(-A)) / math.sqrt(-A)
    return pref * (-3.0 + (A + 3.0) * F) / (A * A)


def isotropisation_rk4(Tpar0: float, Tperp0: float, dt: float, steps: int, n: float = 1.0,
                       lnL: float = 10.0, substeps: int = 20):
    """Integrate dTperp/dt = -nu (Tperp - Tpar), dTpar/dt = -2 dTperp/dt with RK4.
    Returns arrays (Tpar, Tperp) of length steps + 1 sampled every dt."""

    def rhs(y):
        tpa, tpe = y
        dtpe = -nu_isotropisation(tpa, tpe, n, lnL) * (tpe - tpa)
        return np.array([-2.0 * dtpe, dtpe])

    y = np.array([Tpar0, Tperp0], dtype=np.float64)
    h = dt / substeps
    out = [y.copy()]
    for _ in range(steps):
        for _ in range(substeps):
            k1 = rhs(y)
            k2 = rhs(y + 0.5 * h * k1)
            k3 = rhs(y + 0.5 * h * k2)
            k4 = rhs(y + h * k3)
            y = y + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        out.append(y.copy())
    out = np.array(out)
    return out[:, 0], out[:, 1]


# ---------------------------------------------------------------- angle moments


def _gauss_expect(f, s2: float) -> float:
    """E[f(delta)] for delta ~ N(0, s2), f even; adaptive quadrature in delta."""
    s = math.sqrt(s2)
    norm = 1.0 / (s * math.sqrt(2.0 * math.pi))

    def integrand(d):
        return f(d) * norm * math.exp(-0.5 * d * d / s2)

    hi = 12.0 * s
    pts = [p for p in (0.5, 1.0, 2.0) if p < hi]
    with warnings.catch_warnings():
        # at extreme s2 the requested 1e-12 is below round-off; the result is
        # still the best available estimate
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(integrand, 0.0, hi, points=pts or None, limit=400,
                                epsabs=0.0, epsrel=1e-12)
    return 2.0 * val


def g_angle(s2: float) -> float:
    """E[1 - cos Theta] = E[2 delta^2 / (1 + delta^2)]."""
    return _gauss_expect(lambda d: 2.0 * d * d / (1.0 + d * d), s2)


def h_angle(s2: float) -> float:
    """E[sin^2 Theta] = E[4 delta^2 / (1 + delta^2)^2]."""
    return _gauss_expect(lambda d: 4.0 * d * d / (1.0 + d * d) ** 2, s2)


# ---------------------------------------------------------------- features


def cell_features(v: np.ndarray, cell_start: np.ndarray) -> np.ndarray:
    """Eight features per cell, from the cell's velocities (two passes):
    ln N, ln T, T_xx/T - 1, T_yy/T - 1, T_zz/T - 1, ||offdiag T||_F / T,
    |q| / (N T^1.5) with q = 1/2 sum |c|^2 c, <|c|^4> / (15 T^2) - 1,
    where c = v - mean(v), T_ab = <c_a c_b>, T = tr(T) / 3.
    Cells with fewer than 2 members or T <= 0 get NaN rows."""
    M = cell_start.size - 1
    out = np.full((M, 8), np.nan)
    for j in range(M):
        lo, hi = int(cell_start[j]), int(cell_start[j + 1])
        N = hi - lo
        if N < 2:
            continue
        c = v[:, lo:hi] - v[:, lo:hi].mean(axis=1, keepdims=True)
        Tt = (c @ c.T) / N
        T = np.trace(Tt) / 3.0
        if not T > 0:
            continue
        off = math.sqrt(2.0 * (Tt[0, 1] ** 2 + Tt[0, 2] ** 2 + Tt[1, 2] ** 2))
        c2 = (c * c).sum(axis=0)
        q = 0.5 * (c2[None, :] * c).sum(axis=1)
        out[j] = [math.log(N), math.log(T), Tt[0, 0] / T - 1.0, Tt[1, 1] / T - 1.0, Tt[2, 2] / T - 1.0,
                  off / T,
                  np.linalg.norm(q) / (N * T ** 1.5), (c2 * c2).mean() / (15.0 * T * T) - 1.0]
    return out


# ---------------------------------------------------------------- label


def expected_pair_change(u: np.ndarray, s2: np.ndarray) -> np.ndarray:
    """E over (delta, Phi) of the change of v_a v_a^T + v_b v_b^T for pairs with
    relative velocity u (k, 3): 1/4 h(s2) (|u|^2 I - 3 u u^T).  Returns (k, 3, 3)."""
    h = np.array([h_angle(float(x)) for x in s2])
    uu = (u * u).sum(axis=1)
    t = uu[:, None, None] * np.eye(3)[None] - 3.0 * u[:, :, None] * u[:, None, :]
    return 0.25 * h[:, None, None] * t


def relaxation(v, cell_start, pid, *, dt, lnL, seed, step, replicas, density=None,
               dt_scale=None):
    """r_j = ||(1/K) sum over K re-pairings of sum_pairs 1/4 h(s2) (|u|^2 I - 3 u u^T)||_F
    / (N_j T_j), with the oracle's re-pairings (domain 3, c3 = replica) and h by
    quadrature.  Plain loops; meant for small inputs."""
    import oracle
    M = cell_start.size - 1
    acc = np.zeros((M, 3, 3))
    for rep in range(replicas):
        u, cell = oracle.repair_u(v, cell_start, pid, seed, step, rep)
        for k in range(u.shape[0]):
            j = int(cell[k])
            dens = 1.0 if density is None else float(density[j])
            dts = 1.0 if dt_scale is None else float(dt_scale[j])
            uu = float(u[k] @ u[k])
            if uu == 0.0:
                continue
            s2 = 8 * math.pi * dens * lnL * dt * dts / uu ** 1.5
            acc[j] += expected_pair_change(u[k:k + 1], np.array([s2]))[0]
    r = np.zeros(M)
    for j in range(M):
        lo, hi = int(cell_start[j]), int(cell_start[j + 1])
        N = hi - lo
        if N < 2:
            continue
        c = v[:, lo:hi] - v[:, lo:hi].mean(axis=1, keepdims=True)
        T = float((c * c).sum()) / (3 * N)
        r[j] = np.linalg.norm(acc[j] / replicas) / (N * T)
    return r


# ---------------------------------------------------------------- analytic gate


def _psi(v: float) -> float:
    """psi(v) = G'(v)/v - G''(v) for the Rosenbluth potential G(v) = E|v - w|
    of a unit Maxwellian, G = (v + 1/v) erf(v/sqrt2) + sqrt(2/pi) exp(-v^2/2):
    psi = (1/v - 3/v^3) erf(v/sqrt2) + 3 sqrt(2/pi) exp(-v^2/2) / v^2.
    E_w[(I - 3 u^ u^T) / |u|] over u = v - w equals -psi(|v|) (I - 3 v^ v^T)."""
    from scipy.special import erf
    if v < 1e-2:   # series: the closed form cancels near 0
        return math.sqrt(2.0 / math.pi) * v * v * (2.0 / 15.0 - v * v / 35.0)
    return (1.0 / v - 3.0 / v ** 3) * erf(v / math.sqrt(2.0)) + \
        3.0 * math.sqrt(2.0 / math.pi) * math.exp(-0.5 * v * v) / (v * v)


def pairing_noise_constants():
    """(6 E[psi^2], 6 E[psi v^2]^2 / E[v^4]) over a unit Maxwellian, by quadrature.
    The second is 10 / (25 pi): the part of the pair sum's pairing-independent
    fluctuation that the sample's second-moment anisotropy explains."""
    dens = lambda v: 4.0 * math.pi * v * v * (2.0 * math.pi) ** -1.5 * math.exp(-0.5 * v * v)
    e2, _ = integrate.quad(lambda v: _psi(v) ** 2 * dens(v), 0.0, 40.0, limit=400, epsrel=1e-12)
    e1, _ = integrate.quad(lambda v: _psi(v) * v * v * dens(v), 0.0, 40.0, limit=400, epsrel=1e-12)
    return 6.0 * e2, 6.0 * e1 * e1 / 15.0


def analytic_relaxation(v, cell_start, *, dt, lnL, replicas, density=None):
    """Estimate of the label r_j from the cell's moments alone (no pairing),
    the baseline the learned gate is compared with:
        r_pred^2 = r_aniso^2 + r_floor^2,
        r_aniso = 3 nu_0 dt ||A||_F,
        r_floor^2 = (c / T^1.5)^2 / N * (a - b + (3/2 - a) / K),
    with c = 8 pi n lnL dt, (a, b) = pairing_noise_constants().
    A = T_ab / T - I is the traceless part of the temperature tensor in units
    of T = tr(T_ab) / 3 (its diagonal and off-diagonal norm are features 2-5
    of cell_features).  Linearised about isotropy the
    traceless part decays at 3 nu_0 (for a bi-Maxwellian, T_par - T_perp
    decays at 3 nu_T), nu_0 = (8 sqrt(pi) / 15) n lnL / T^1.5 the
    small-anisotropy limit of nu_isotropisation.  The floor is the spread of
    the pair sum of an isotropic Maxwellian cell in the small-angle limit
    h = 4 s^2, where a pair adds c (I - 3 u^ u^T) / |u|: split into the
    pairing-independent part sum_a g(v_a) (variance a N (c/T^1.5)^2 T^2, of
    which the fraction b/a is the second-moment anisotropy already in r_aniso)
    and the pairing part (variance (3/2 - a) N (...)^2, E|u|^-2 = 1/(2T),
    divided by K by the average over re-pairings).  Slow pairs, whose angle
    is not small, make the floor an overestimate at larger dt.  NaN for cells
    without features."""
    a, b = pairing_noise_constants()
    f = cell_features(v, cell_start)
    M = cell_start.size - 1
    out = np.full(M, np.nan)
    for j in range(M):
        if np.isnan(f[j, 0]):
            continue
        N = math.exp(f[j, 0])
        T = math.exp(f[j, 1])
        n = 1.0 if density is None else float(density[j])
        a2 = f[j, 2] ** 2 + f[j, 3] ** 2 + f[j, 4] ** 2 + f[j, 5] ** 2
        nu0 = 8.0 * math.sqrt(math.pi) / 15.0 * n * lnL / T ** 1.5
        r_aniso = 3.0 * nu0 * dt * math.sqrt(a2)
        c = 8.0 * math.pi * n * lnL * dt / T ** 1.5
        r_floor2 = c * c / N * (a - b + (1.5 - a) / replicas)
        out[j] = math.sqrt(r_aniso ** 2 + r_floor2)
    return out


# ---------------------------------------------------------------- gate MLP (FP64)


def bf16_round(a):
    """Round to bfloat16 (nearest, ties to even) via binary32, returned as float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack_params(flat):
    flat = np.asarray(flat, dtype=np.float64)
    W1 = flat[0:512].reshape(8, 64)
    b1 = flat[512:576]
    W2 = flat[576:4672].reshape(64, 64)
    b2 = flat[4672:4736]
    W3 = flat[4736:4800].reshape(64, 1)
    b3 = flat[4800:4801]
    return [W1, b1, W2, b2, W3, b3]


def pack_params(params):
    return np.concatenate([p.reshape(-1) for p in params])


def mlp_bce_grad_bf16(flat, x, y):
    """Mean BCE and gradient with the products of bfloat16-rounded operands
    (weights, inputs, activations and back-propagated deltas), FP64 arithmetic."""
    W1, b1, W2, b2, W3, b3 = unpack_params(flat)
    r = bf16_round
    W1r, W2r, W3r = r(W1), r(W2), r(W3)
    B = x.shape[0]
    xr = r(x)
    z1 = xr @ W1r + b1
    a1 = r(np.maximum(z1, 0.0))
    z2 = a1 @ W2r + b2
    a2 = r(np.maximum(z2, 0.0))
    z3 = (a2 @ W3r + b3)[:, 0]
    p = 1.0 / (1.0 + np.exp(-z3))
    loss = np.mean(np.maximum(z3, 0) - z3 * y + np.log1p(np.exp(-np.abs(z3))))
    d3 = r((p - y) / B)
    gW3 = a2.T @ d3[:, None]
    gb3 = np.array([d3.sum()])
    d2 = r(np.where(z2 > 0, W3r[:, 0][None, :] * d3[:, None], 0.0))
    gW2 = a1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = r(np.where(z1 > 0, d2 @ W2r.T, 0.0))
    gW1 = xr.T @ d1
    gb1 = d1.sum(axis=0)
    return loss, pack_params([gW1, gb1, gW2, gb2, gW3, gb3]), p


def mlp_init_shapes():
    return [(8, 64), (64,), (64, 64), (64,), (64, 1), (1,)]


def mlp_forward(params, x):
    W1, b1, W2, b2, W3, b3 = params
    z1 = x @ W1 + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2 + b2
    a2 = np.maximum(z2, 0.0)
    z3 = a2 @ W3 + b3
    p = 1.0 / (1.0 + np.exp(-z3[:, 0]))
    return p, (x, z1, a1, z2, a2, z3)


def mlp_bce_grad(params, x, y):
    """Mean binary cross-entropy and its gradient for logits z3."""
    W1, b1, W2, b2, W3, b3 = params
    p, (x, z1, a1, z2, a2, z3) = mlp_forward(params, x)
    B = x.shape[0]
    z = z3[:, 0]
    loss = np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z))))
    dz3 = ((p - y) / B)[:, None]
    gW3 = a2.T @ dz3
    gb3 = dz3.sum(axis=0)
    da2 = dz3 @ W3.T
    dz2 = da2 * (z2 > 0)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(axis=0)
    da1 = dz2 @ W2.T
    dz1 = da1 * (z1 > 0)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_update(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; t counts from 1."""
    outp, outm, outv = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mhat = mm / (1 - b1 ** t)
        vhat = vv / (1 - b2 ** t)
        outp.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        outm.append(mm)
        outv.append(vv)
    return outp, outm, outv
