"""FP64 CPU oracle for the electron collision step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It shares no code with the GPU library: the C source
``oracle.c`` is compiled on its own with gcc, and this module is a ctypes
wrapper around it plus plain numpy routines in :mod:`oracle.physics`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-shared", "-fPIC",
           _SRC, "-o", _LIB, "-lm"]


def build() -> str:
    """Compile oracle.c into liboracle.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = GCC_CMD[:-3] + ["-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.orc_philox.argtypes = [u32p, u32p, u32p]
        L.orc_philox.restype = None
        L.orc_philox_fill.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, u32p,
                                      C.c_int64, u32p]
        L.orc_philox_fill.restype = None
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_bin_cells.argtypes = [i32p, C.c_int64, C.c_int32, i32p, i32p]
        L.orc_bin_cells.restype = C.c_int
        L.orc_pairs.argtypes = [i32p, u32p, C.c_int32, C.c_uint64, C.c_uint64, i32p, i32p]
        L.orc_pairs.restype = C.c_int
        L.orc_ta_delta.argtypes = [f64p, C.c_double, C.c_double, C.c_double, C.c_double, f64p]
        L.orc_ta_delta.restype = None
        L.orc_mcc_exact_count.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double]
        L.orc_mcc_exact_count.restype = C.c_int64
        L.orc_mcc_exact.argtypes = [f64p, u32p, C.c_int64, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_uint64, C.c_uint64, C.c_void_p]
        L.orc_mcc_exact.restype = C.c_int
        L.orc_step_triplet.argtypes = [f64p, C.c_int64, i32p, u32p, C.c_int32, C.c_double,
                                       C.c_double, C.c_void_p, C.c_uint64, C.c_uint64]
        L.orc_step_triplet.restype = C.c_int
        L.orc_step_weighted.argtypes = [f64p, C.c_void_p, C.c_int64, i32p, u32p, C.c_int32,
                                        C.c_double, C.c_double, C.c_void_p, C.c_uint64,
                                        C.c_uint64, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_step_weighted.restype = C.c_int
        L.orc_nanbu_A.argtypes = [C.c_double]
        L.orc_nanbu_A.restype = C.c_double
        L.orc_nanbu_omc.argtypes = [C.c_double, C.c_double]
        L.orc_nanbu_omc.restype = C.c_double
        L.orc_nanbu.argtypes = [f64p, C.c_int64, i32p, u32p, C.c_int32, C.c_double, C.c_double,
                                C.c_void_p, C.c_uint64, C.c_uint64]
        L.orc_nanbu.restype = C.c_int
        L.orc_recombine.argtypes = [f64p, f64p, u32p, C.c_void_p, C.c_int64, i32p, C.c_int32,
                                    C.c_double, C.c_uint64, C.c_uint64, C.c_void_p]
        L.orc_recombine.restype = C.c_int
        L.orc_p2c.argtypes = [f64p, C.c_int32, i32p, C.c_int64, C.c_int32, f64p]
        L.orc_p2c.restype = C.c_int64
        L.orc_dsmc_sigma.argtypes = [C.c_int32, C.c_double, C.c_int32, f64p, f64p, f64p]
        L.orc_dsmc_sigma.restype = C.c_double
        L.orc_dsmc.argtypes = [f64p, C.c_int64, i32p, u32p, C.c_void_p, C.c_void_p, C.c_double,
                               C.c_double, C.c_double, C.c_int32, f64p, f64p, f64p, C.c_double,
                               C.c_uint64, C.c_uint64, C.c_uint32, f64p, C.c_int64, u32p, i32p,
                               C.POINTER(C.c_int64), C.c_void_p]
        L.orc_dsmc.restype = C.c_int
        L.orc_ta_s2.argtypes = [C.c_double] * 4
        L.orc_ta_s2.restype = C.c_double
        L.orc_mcc_threshold.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_mcc_threshold.restype = C.c_uint64
        L.orc_mcc.argtypes = [f64p, u32p, C.c_int64, C.c_double, C.c_double, C.c_double,
                              C.c_double, C.c_uint64, C.c_uint64, C.c_void_p]
        L.orc_mcc.restype = C.c_int
        L.orc_step.argtypes = [f64p, i32p, u32p, C.c_int64, C.c_int32, C.POINTER(Params),
                               C.c_void_p]
        L.orc_step.restype = C.c_int
        L.orc_conserve_cells.argtypes = [f64p, C.c_int64, i32p, C.c_int32, f64p]
        L.orc_conserve_cells.restype = C.c_int
        L.orc_cell_moments.argtypes = [f64p, C.c_int64, i32p, C.c_int32, f64p]
        L.orc_cell_moments.restype = C.c_int
        L.orc_repair_u.argtypes = [f64p, C.c_int64, i32p, C.c_int32, u32p, C.c_uint64,
                                   C.c_uint64, C.c_uint32, f64p, i32p]
        L.orc_repair_u.restype = C.c_int64
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("lnL", C.c_double), ("density", C.c_void_p),
                ("seed", C.c_uint64), ("step", C.c_uint64), ("conserve", C.c_int32),
                ("mcc", C.c_int32), ("sigma0", C.c_double), ("n_neutral", C.c_double),
                ("mass_ratio", C.c_double), ("dt_scale", C.c_void_p), ("skip", C.c_void_p)]


def _ptr(a):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------- RNG
def philox(ctr, key):
    """One Philox4x32-10 block: ctr = 4 words, key = 2 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(c, k, out)
    return out


def philox_fill(seed: int, step: int, domain: int, c0, c3: int = 0) -> np.ndarray:
    c0 = np.ascontiguousarray(c0, dtype=np.uint32)
    out = np.zeros((c0.size, 4), np.uint32)
    lib().orc_philox_fill(seed, step, domain, c3, c0, c0.size, out.reshape(-1))
    return out


def u01(x) -> np.ndarray:
    """((x >> 9) + 0.5) * 2^-23 -- exact in binary32 and binary64."""
    x = np.asarray(x, dtype=np.uint32)
    return ((x >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


# ---------------------------------------------------------------- binning / pairing
def bin_cells(cell_of, n_cells: int):
    cell_of = np.ascontiguousarray(cell_of, dtype=np.int32)
    cs = np.zeros(n_cells + 1, np.int32)
    order = np.zeros(max(cell_of.size, 1), np.int32)
    rc = lib().orc_bin_cells(cell_of, cell_of.size, n_cells, cs, order)
    if rc:
        raise ValueError(f"orc_bin_cells failed: {rc}")
    return cs, order[:cell_of.size]


def pairs(cell_start, pid, seed: int, step: int):
    """Returns (sorted_slots, partner) for storage already in cell order."""
    cs = np.ascontiguousarray(cell_start, dtype=np.int32)
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    n = int(cs[-1])
    srt = np.zeros(max(n, 1), np.int32)
    par = np.zeros(max(n, 1), np.int32)
    rc = lib().orc_pairs(cs, pid, cs.size - 1, seed, step, srt, par)
    if rc:
        raise ValueError(f"orc_pairs failed: {rc}")
    return srt[:n], par[:n]


# ---------------------------------------------------------------- collision pieces
def ta_delta(u, s2: float, U1: float, U2: float, U3: float) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    du = np.zeros(3, np.float64)
    lib().orc_ta_delta(u, s2, U1, U2, U3, du)
    return du


def ta_s2(umag: float, density: float, lnL: float, dt: float) -> float:
    return lib().orc_ta_s2(umag, density, lnL, dt)


def mcc_threshold(dt: float, sigma0: float, n_neutral: float) -> int:
    return int(lib().orc_mcc_threshold(dt, sigma0, n_neutral))


def mcc_exact_count(n: int, dt: float, sigma0: float, n_neutral: float) -> int:
    return int(lib().orc_mcc_exact_count(n, dt, sigma0, n_neutral))


def mcc_exact(v, pid, dt, sigma0, n_neutral, mass_ratio, seed, step):
    """Exact-count null-collision step in place on v (3, n) float64; returns
    the selected flags."""
    n = v.shape[1]
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    flags = np.zeros(max(n, 1), np.uint8)
    rc = lib().orc_mcc_exact(v.reshape(-1), pid, n, dt, sigma0, n_neutral, mass_ratio, seed, step,
                             flags.ctypes.data)
    if rc:
        raise ValueError(f"orc_mcc_exact failed: {rc}")
    return flags[:n]


def step_triplet(v, cell_start, pid, dt, lnL, seed, step, density=None):
    """One Takizuka-Abe step with the triplet for odd cells, in place on v
    (3, n) float64, storage in cell order."""
    n = v.shape[1]
    cell_start = np.ascontiguousarray(cell_start, dtype=np.int32)
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    d = None if density is None else np.ascontiguousarray(density, dtype=np.float64)
    rc = lib().orc_step_triplet(v.reshape(-1), n, cell_start, pid, cell_start.size - 1, dt, lnL,
                                None if d is None else d.ctypes.data, seed, step)
    if rc:
        raise ValueError(f"orc_step_triplet failed: {rc}")


def step_weighted(v, w, cell_start, pid, dt, lnL, seed, step, density=None, mcc=False,
                  sigma0=0.0, n_neutral=0.0, mass_ratio=0.0):
    """One Takizuka-Abe step of variable-weight particles (weights w, (n,)
    float64), in place on v (3, n) float64, storage in cell order."""
    n = v.shape[1]
    cell_start = np.ascontiguousarray(cell_start, dtype=np.int32)
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = None if density is None else np.ascontiguousarray(density, dtype=np.float64)
    rc = lib().orc_step_weighted(v.reshape(-1), w.ctypes.data, n, cell_start, pid,
                                 cell_start.size - 1, dt, lnL, None if d is None else d.ctypes.data,
                                 seed, step, int(bool(mcc)), sigma0, n_neutral, mass_ratio)
    if rc:
        raise ValueError(f"orc_step_weighted failed: {rc}")


def nanbu_A(s: float) -> float:
    return float(lib().orc_nanbu_A(s))


def nanbu_omc(A: float, U: float) -> float:
    return float(lib().orc_nanbu_omc(A, U))


def nanbu(v, cell_start, pid, dt, lnL, seed, step, density=None):
    """One Nanbu Coulomb step in place on v (3, n) float64, storage in cell order."""
    n = v.shape[1]
    cell_start = np.ascontiguousarray(cell_start, dtype=np.int32)
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    d = None if density is None else np.ascontiguousarray(density, dtype=np.float64)
    rc = lib().orc_nanbu(v.reshape(-1), n, cell_start, pid, cell_start.size - 1, dt, lnL,
                         None if d is None else d.ctypes.data, seed, step)
    if rc:
        raise ValueError(f"orc_nanbu failed: {rc}")


def recombine(v, w, pid, primary, cell_start, eps, seed, step):
    """Recombination C5 in place on v (3, n) and w (n,) float64, storage in
    cell order; returns the per-cell event counts."""
    n = v.shape[1]
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    primary = np.ascontiguousarray(primary, dtype=np.uint8)
    cell_start = np.ascontiguousarray(cell_start, dtype=np.int32)
    M = cell_start.size - 1
    ev = np.zeros(max(M, 1), np.int32)
    rc = lib().orc_recombine(v.reshape(-1), w, pid, primary.ctypes.data, n, cell_start, M, eps,
                             seed, step, ev.ctypes.data)
    if rc:
        raise ValueError(f"orc_recombine failed: {rc}")
    return ev[:M]


def p2c(q, cell_of, n_cells: int):
    """Per-cell sums (n_cells, nq) of the rows of q (nq, n); returns (sums,
    number of skipped out-of-range ids)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    nq, n = q.shape
    cell_of = np.ascontiguousarray(cell_of, dtype=np.int32)
    out = np.zeros((n_cells, nq), np.float64)
    bad = lib().orc_p2c(q.reshape(-1), nq, cell_of, n, n_cells, out.reshape(-1))
    return out, int(bad)


def mcc(v, pid, dt, sigma0, n_neutral, mass_ratio, seed, step, return_flags=False):
    """Stand-alone null-collision step, in place on v (3, n) float64."""
    n = v.shape[1]
    pid = np.ascontiguousarray(pid, dtype=np.uint32)
    flags = np.zeros(max(n, 1), np.uint8) if return_flags else None
    rc = lib().orc_mcc(v.reshape(-1), pid, n, dt, sigma0, n_neutral, mass_ratio, seed, step,
                       _ptr(flags))
    if rc:
        raise ValueError(f"orc_mcc failed: {rc}")
    return flags[:n] if return_flags else None


def step(v, cell_of, pid, n_cells: int, *, dt: float, lnL: float, seed: int, step: int,
         density=None, conserve=False, mcc=False, sigma0=0.0, n_neutral=0.0,
         mass_ratio=0.0, dt_scale=None, skip=None):
    """One full collision step in place.  v: (3, n) float64 C-contiguous,
    cell_of int32, pid uint32 -- all permuted into stable cell order.
    Returns cell_start."""
    assert v.dtype == np.float64 and v.flags.c_contiguous and v.shape[0] == 3
    n = v.shape[1]
    assert cell_of.dtype == np.int32 and pid.dtype == np.uint32
    dens = None if density is None else np.ascontiguousarray(density, np.float64)
    dts = None if dt_scale is None else np.ascontiguousarray(dt_scale, np.float64)
    sk = None if skip is None else np.ascontiguousarray(skip, np.uint8)
    p = Params(dt, lnL, _ptr(dens), seed, step, int(bool(conserve)), int(bool(mcc)), sigma0,
               n_neutral, mass_ratio, _ptr(dts), _ptr(sk))
    cs = np.zeros(n_cells + 1, np.int32)
    rc = lib().orc_step(v.reshape(-1), cell_of, pid, n, n_cells, C.byref(p), cs.ctypes.data)
    if rc:
        raise ValueError(f"orc_step failed: {rc}")
    return cs


def conserve_cells(v, cell_start, before):
    """Per-cell correction in place; before = (M, 5) sums N, sum v (3), sum |v|^2."""
    cs = np.ascontiguousarray(cell_start, dtype=np.int32)
    lib().orc_conserve_cells(v.reshape(-1), v.shape[1], cs, cs.size - 1,
                             np.ascontiguousarray(before, np.float64).reshape(-1))


def cell_moments(v, cell_start) -> np.ndarray:
    cs = np.ascontiguousarray(cell_start, dtype=np.int32)
    out = np.zeros((cs.size - 1, 14), np.float64)
    lib().orc_cell_moments(np.ascontiguousarray(v, np.float64).reshape(-1), v.shape[1], cs,
                           cs.size - 1, out.reshape(-1))
    return out


def repair_u(v, cell_start, pid, seed: int, step: int, replica: int):
    cs = np.ascontiguousarray(cell_start, dtype=np.int32)
    n = v.shape[1]
    u = np.zeros((max(n // 2, 1), 3), np.float64)
    cell = np.zeros(max(n // 2, 1), np.int32)
    k = lib().orc_repair_u(np.ascontiguousarray(v, np.float64).reshape(-1), n, cs, cs.size - 1,
                           np.ascontiguousarray(pid, np.uint32), seed, step, replica,
                           u.reshape(-1), cell)
    if k < 0:
        raise MemoryError("orc_repair_u")
    return u[:k], cell[:k]


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------- DSMC-Coll (C1..C4)
def dsmc_sigma(c: int, E: float, table) -> float:
    """Cross section of channel c (0..3) at energy E from a table dict with
    float64 arrays 'breaks' [P+1], 'coef' [4, P, 4], 'thr' [4]."""
    return lib().orc_dsmc_sigma(c, E, table["coef"].shape[1], table["breaks"],
                                np.ascontiguousarray(table["coef"]).reshape(-1), table["thr"])


def dsmc(v, cell_of, pid, *, dt: float, table, seed: int, step: int, pid_base: int,
         n_gas=None, n_meta=None, ng0: float = 1.0, nm0: float = 0.0, mass_ratio: float = 0.0,
         cap: int = 0):
    """DSMC-Coll step in place on v (3, n) float64.  Returns (channel per
    particle, 0 = none, 1..4 = C1..C4; new electrons' v (3, k), pid, cell)."""
    n = v.shape[1]
    cell_of = np.ascontiguousarray(cell_of, np.int32)
    pid = np.ascontiguousarray(pid, np.uint32)
    cap = max(int(cap), 1)
    vn = np.zeros((3, cap), np.float64)
    pn = np.zeros(cap, np.uint32)
    cn = np.zeros(cap, np.int32)
    cnt = C.c_int64(0)
    chan = np.zeros(max(n, 1), np.uint8)
    ng = None if n_gas is None else np.ascontiguousarray(n_gas, np.float64)
    nm = None if n_meta is None else np.ascontiguousarray(n_meta, np.float64)
    rc = lib().orc_dsmc(v.reshape(-1), n, cell_of, pid, _ptr(ng), _ptr(nm), ng0, nm0, dt,
                        table["coef"].shape[1], table["breaks"],
                        np.ascontiguousarray(table["coef"]).reshape(-1), table["thr"], mass_ratio,
                        seed, step, pid_base, vn.reshape(-1), cap, pn, cn, C.byref(cnt),
                        chan.ctypes.data)
    if rc:
        raise ValueError("orc_dsmc: more new electrons than cap")
    k = cnt.value
    return chan[:n], vn[:, :k], pn[:k], cn[:k]
