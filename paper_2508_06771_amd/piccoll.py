"""ctypes binding of libpiccoll.so -- argument marshalling only.

Every step of the collision path runs in the HIP library; this module checks
tensor dtypes, devices and contiguity, passes raw device pointers and the
current torch stream, and turns status codes into exceptions.  There is no
CPU fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpiccoll.so")

PIC_F32, PIC_F64 = 0, 1
CONSERVE_FIX = 1 << 0
FUSE_MCC = 1 << 1
GATE = 1 << 2
ASSUME_SORTED = 1 << 3
MOMENTS = 1 << 4
CHECK_FINITE = 1 << 5
PIC_ERR_ARG, PIC_ERR_RANGE, PIC_ERR_NOMEM, PIC_ERR_STATE, PIC_ERR_NONFINITE = 1, 2, 4, 6, 7
# limits of coulomb_collide_noalloc (its fixed scratch and the LDS classes)
NOALLOC_MAX_CELLS = 65536
NOALLOC_MAX_CELL_F32 = 10240
NOALLOC_MAX_CELL_F64 = 6144

_STATUS = {0: "PIC_OK", 1: "PIC_ERR_ARG", 2: "PIC_ERR_RANGE", 3: "PIC_ERR_HIP",
           4: "PIC_ERR_NOMEM", 5: "PIC_ERR_DTYPE", 6: "PIC_ERR_STATE", 7: "PIC_ERR_NONFINITE"}


class PicError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)} ({status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run paper_2508_06771_amd/build.py "
                          "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, u64, u32, f64 = (C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_uint32,
                                   C.c_double)
    sig = {
        "pic_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
        "pic_destroy": ([vp], None),
        "pic_strerror": ([C.c_int], C.c_char_p),
        "pic_sync": ([vp], C.c_int),
        "pic_set_stream": ([vp, vp], C.c_int),
        "pic_bin_cells": ([vp, vp, i64, i32, vp, vp], C.c_int),
        "coulomb_collide_noalloc": ([vp, C.c_int, vp, vp, vp, i64, i32, f64, f64, vp, u64, u64,
                                     u32], C.c_int),
        "coulomb_collide": ([vp, C.c_int, vp, vp, vp, i64, i32, f64, f64, vp, u64, u64, u32],
                            C.c_int),
        "pic_set_mcc": ([vp, f64, f64, f64], C.c_int),
        "pic_set_moments_out": ([vp, vp], C.c_int),
        "mcc_null_collide": ([vp, C.c_int, vp, vp, i64, f64, f64, f64, f64, u64, u64, vp],
                             C.c_int),
        "pic_philox": ([vp, u64, u64, u32, u32, vp, i64, vp], C.c_int),
        "mcc_null_collide_exact": ([vp, C.c_int, vp, vp, i64, f64, f64, f64, f64, u64, u64, vp],
                                   C.c_int),
        "p2c_sums": ([vp, C.c_int, vp, C.c_int32, vp, i64, C.c_int32, vp], C.c_int),
        "recombine": ([vp, C.c_int, vp, vp, vp, vp, i64, vp, C.c_int32, f64, u64, u64, vp], C.c_int),
        "coulomb_collide_nanbu": ([vp, C.c_int, vp, vp, i64, vp, C.c_int32, f64, f64, vp, u64, u64],
                                  C.c_int),
        "coulomb_collide_triplet": ([vp, C.c_int, vp, vp, i64, vp, C.c_int32, f64, f64, vp, u64, u64],
                                    C.c_int),
        "coulomb_collide_weighted": ([vp, C.c_int, vp, vp, vp, i64, vp, C.c_int32, f64, f64, vp, u64,
                                      u64, u32], C.c_int),
        "coulomb_pairs": ([vp, vp, vp, i32, u64, u64, vp, vp], C.c_int),
        "pic_cell_moments": ([vp, C.c_int, vp, i64, vp, i32, vp], C.c_int),
        "pic_unsort": ([vp, C.c_int, vp, vp, vp, i64], C.c_int),
        "pic_run_steps": ([vp, C.c_int, vp, vp, vp, i64, i32, f64, f64, vp, u64, u64, i64, u32],
                          C.c_int),
        "pic_features": ([vp, vp, i32, vp, vp], C.c_int),
        "pic_relaxation": ([vp, C.c_int, vp, i64, vp, vp, i32, f64, f64, vp, vp, u64, u64, i32, vp],
                           C.c_int),
        "pic_mlp_forward": ([vp, vp, vp, i32, C.c_int, vp], C.c_int),
        "pic_mlp_grad": ([vp, vp, vp, vp, i32, C.c_int, vp, vp], C.c_int),
        "pic_mlp_train_step": ([vp, vp, vp, vp, i32, C.c_float, vp, vp, i32, C.c_int, vp], C.c_int),
        "mlp_train_step": ([vp, vp, vp, i32, vp, vp, C.c_float, vp], C.c_int),
        "pic_gate_config": ([vp, vp, C.c_float, i32, f64, f64, i32, C.c_int], C.c_int),
        "pic_gate_config_analytic": ([vp, C.c_float, i32, f64, f64, i32], C.c_int),
        "pic_analytic_relaxation": ([vp, vp, i32, f64, f64, vp, i32, vp], C.c_int),
        "pic_gate_reset": ([vp], C.c_int),
        "pic_gate_stats": ([vp, C.POINTER(C.c_int64)], C.c_int),
        "pic_gate_state": ([vp, vp, vp, vp, vp], C.c_int),
        "pic_conserve_reset": ([vp], C.c_int),
        "pic_gate_refresh": ([vp, i32], C.c_int),
        "gate_infer": ([vp, vp, i32, vp, C.c_float, i32, C.c_int, vp, vp, vp], C.c_int),
        "pic_set_dsmc": ([vp, i32, vp, vp, vp, f64], C.c_int),
        "dsmc_collide": ([vp, C.c_int, vp, vp, vp, i64, i32, vp, vp, f64, f64, f64, u64, u64, u32, vp,
                          vp, vp, i64, vp, vp], C.c_int),
        "pic_autotune": ([vp, C.c_int, vp, vp, vp, i64, i32, f64, f64, u32, vp], C.c_int),
        "pic_set_schedule": ([vp, C.c_int, C.c_int], C.c_int),
        "pic_set_workspace_limit": ([vp, C.c_size_t], C.c_int),
        "pic_time_kernels": ([vp, C.c_int], C.c_int),
        "pic_kernel_times": ([vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()

EXPORTED = ["pic_create", "pic_destroy", "pic_strerror", "pic_sync", "pic_set_stream",
            "pic_bin_cells", "coulomb_collide", "pic_set_mcc", "pic_set_moments_out",
            "mcc_null_collide", "pic_philox", "coulomb_pairs", "pic_cell_moments", "pic_unsort",
            "pic_time_kernels", "pic_kernel_times", "pic_run_steps", "pic_features",
            "pic_relaxation", "pic_mlp_forward", "pic_mlp_grad", "pic_mlp_train_step",
            "mlp_train_step", "pic_gate_config", "pic_gate_config_analytic",
            "pic_analytic_relaxation", "pic_gate_reset", "pic_gate_stats", "pic_gate_state",
            "pic_autotune",
            "pic_conserve_reset", "pic_gate_refresh", "gate_infer", "pic_set_dsmc", "dsmc_collide",
            "mcc_null_collide_exact", "p2c_sums", "recombine", "coulomb_collide_nanbu",
            "coulomb_collide_triplet", "coulomb_collide_noalloc", "coulomb_collide_weighted", "pic_set_schedule",
            "pic_set_workspace_limit"]

MLP_PARAMS = 4801
GATE_STATS = ["steps", "skipped", "collided", "judged", "judged_want", "false_skip", "disabled",
              "have_moments"]

KT_SLOTS = ["class0", "class1", "class2", "class3", "huge", "check", "queue", "sort", "mcc", "gate",
            "relax", "deferred", "moments", "dsmc", "p2c", "recombine", "nanbu", "triplet", "weighted",
            "all"]


def _dt(v: torch.Tensor) -> int:
    if v.dtype == torch.float32:
        return PIC_F32
    if v.dtype == torch.float64:
        return PIC_F64
    raise TypeError(f"velocities must be float32 or float64, got {v.dtype}")


def _p(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on a HIP device")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _chk(rc: int, where: str):
    if rc != 0:
        raise PicError(rc, where)


class Context:
    """One library context bound to a device; calls go on torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        with torch.cuda.device(device):
            s = torch.cuda.current_stream().cuda_stream
            _chk(lib.pic_create(C.byref(h), device, C.c_void_p(s)), "pic_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib.pic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _chk(lib.pic_set_stream(self._h, C.c_void_p(s)), "pic_set_stream")

    def sync(self):
        _chk(lib.pic_sync(self._h), "pic_sync")

    # -------------------------------------------------------------- binning
    def bin_cells(self, cell_of: torch.Tensor, n_cells: int):
        assert cell_of.dtype == torch.int32
        self._stream()
        n = cell_of.numel()
        cs = torch.empty(n_cells + 1, dtype=torch.int32, device=cell_of.device)
        order = torch.empty(max(n, 1), dtype=torch.int32, device=cell_of.device)
        _chk(lib.pic_bin_cells(self._h, _p(cell_of), n, n_cells, _p(cs), _p(order)),
             "pic_bin_cells")
        return cs, order[:n]

    # -------------------------------------------------------------- collision step
    def set_mcc(self, sigma0: float, n_neutral: float, mass_ratio: float = 0.0):
        _chk(lib.pic_set_mcc(self._h, sigma0, n_neutral, mass_ratio), "pic_set_mcc")

    def conserve_reset(self):
        _chk(lib.pic_conserve_reset(self._h), "pic_conserve_reset")

    def set_moments_out(self, out):
        if out is not None:
            assert out.dtype == torch.float64
        _chk(lib.pic_set_moments_out(self._h, _p(out)), "pic_set_moments_out")

    def coulomb_collide(self, v: torch.Tensor, cell_of: torch.Tensor, pid: torch.Tensor,
                        n_cells: int, *, dt: float, lnL: float, seed: int, step: int,
                        density=None, flags: int = 0):
        assert v.dim() == 2 and v.shape[0] == 3
        assert cell_of.dtype == torch.int32 and pid.dtype in (torch.int32, torch.uint32)
        if density is not None:
            assert density.dtype == torch.float64 and density.numel() == n_cells
        self._stream()
        _chk(lib.coulomb_collide(self._h, _dt(v), _p(v), _p(cell_of), _p(pid), v.shape[1],
                                 n_cells, dt, lnL, _p(density), seed, step, flags),
             "coulomb_collide")

    def coulomb_collide_noalloc(self, v: torch.Tensor, cell_of: torch.Tensor, pid: torch.Tensor,
                                n_cells: int, *, dt: float, lnL: float, seed: int, step: int,
                                density=None, flags: int = 0):
        """coulomb_collide on storage already in cell order, with the library's
        fixed per-GPU scratch (no device allocation)."""
        assert v.dim() == 2 and v.shape[0] == 3
        assert cell_of.dtype == torch.int32 and pid.dtype in (torch.int32, torch.uint32)
        if density is not None:
            assert density.dtype == torch.float64 and density.numel() == n_cells
        self._stream()
        _chk(lib.coulomb_collide_noalloc(self._h, _dt(v), _p(v), _p(cell_of), _p(pid), v.shape[1],
                                         n_cells, dt, lnL, _p(density), seed, step, flags),
             "coulomb_collide_noalloc")

    def set_workspace_limit(self, nbytes: int):
        """Cap on the context's scratch memory (0: none)."""
        _chk(lib.pic_set_workspace_limit(self._h, nbytes), "pic_set_workspace_limit")

    def set_schedule(self, dtype, schedule: int):
        """0: one launch per size class; 1: one persistent launch, smallest
        class one wave per cell; 2: one persistent launch, whole workgroups."""
        d = PIC_F32 if dtype in (torch.float32, "f32") else PIC_F64
        _chk(lib.pic_set_schedule(self._h, d, schedule), "pic_set_schedule")

    def run_steps(self, v: torch.Tensor, cell_of: torch.Tensor, pid: torch.Tensor, n_cells: int,
                  *, dt: float, lnL: float, seed: int, step0: int, nsteps: int, density=None,
                  flags: int = 0):
        """nsteps steps; after the first, replays of a captured HIP graph."""
        assert v.dim() == 2 and v.shape[0] == 3
        assert cell_of.dtype == torch.int32 and pid.dtype in (torch.int32, torch.uint32)
        self._stream()
        _chk(lib.pic_run_steps(self._h, _dt(v), _p(v), _p(cell_of), _p(pid), v.shape[1], n_cells,
                               dt, lnL, _p(density), seed, step0, nsteps, flags), "pic_run_steps")

    def mcc_null_collide(self, v: torch.Tensor, pid: torch.Tensor, *, dt: float, sigma0: float,
                         n_neutral: float, mass_ratio: float, seed: int, step: int,
                         candidates: bool = False):
        self._stream()
        n = v.shape[1]
        cand = torch.empty(max(n, 1), dtype=torch.uint8, device=v.device) if candidates else None
        _chk(lib.mcc_null_collide(self._h, _dt(v), _p(v), _p(pid), n, dt, sigma0, n_neutral,
                                  mass_ratio, seed, step, _p(cand)), "mcc_null_collide")
        return cand[:n] if candidates else None

    def mcc_null_collide_exact(self, v: torch.Tensor, pid: torch.Tensor, *, dt: float,
                               sigma0: float, n_neutral: float, mass_ratio: float, seed: int,
                               step: int, selected: bool = False):
        self._stream()
        n = v.shape[1]
        sel = torch.empty(max(n, 1), dtype=torch.uint8, device=v.device) if selected else None
        _chk(lib.mcc_null_collide_exact(self._h, _dt(v), _p(v), _p(pid), n, dt, sigma0, n_neutral,
                                        mass_ratio, seed, step, _p(sel)),
             "mcc_null_collide_exact")
        return sel[:n] if selected else None

    def nanbu(self, v: torch.Tensor, pid: torch.Tensor, cell_start: torch.Tensor, *, dt: float,
              lnL: float, seed: int, step: int, density=None):
        """One Nanbu Coulomb step in place on v (cell-sorted storage)."""
        self._stream()
        _chk(lib.coulomb_collide_nanbu(self._h, _dt(v), _p(v), _p(pid), v.shape[1], _p(cell_start),
                                       cell_start.numel() - 1, dt, lnL, _p(density), seed, step),
             "coulomb_collide_nanbu")

    def triplet(self, v: torch.Tensor, pid: torch.Tensor, cell_start: torch.Tensor, *, dt: float,
                lnL: float, seed: int, step: int, density=None):
        """One Takizuka-Abe step with the triplet for odd cells, in place on v
        (cell-sorted storage)."""
        self._stream()
        _chk(lib.coulomb_collide_triplet(self._h, _dt(v), _p(v), _p(pid), v.shape[1], _p(cell_start),
                                         cell_start.numel() - 1, dt, lnL, _p(density), seed, step),
             "coulomb_collide_triplet")

    def weighted(self, v: torch.Tensor, w: torch.Tensor, pid: torch.Tensor,
                 cell_start: torch.Tensor, *, dt: float, lnL: float, seed: int, step: int,
                 density=None, flags: int = 0):
        """One Takizuka-Abe step of variable-weight particles in place on v
        (cell-sorted storage; w of v's dtype, not modified)."""
        assert w.dtype == v.dtype and w.numel() == v.shape[1]
        self._stream()
        _chk(lib.coulomb_collide_weighted(self._h, _dt(v), _p(v), _p(w), _p(pid), v.shape[1],
                                          _p(cell_start), cell_start.numel() - 1, dt, lnL,
                                          _p(density), seed, step, flags),
             "coulomb_collide_weighted")

    def recombine(self, v: torch.Tensor, w: torch.Tensor, pid: torch.Tensor, primary: torch.Tensor,
                  cell_start: torch.Tensor, *, eps: float, seed: int, step: int, events=False):
        """Recombination C5 in place on v and w (cell-sorted storage)."""
        self._stream()
        n = v.shape[1]
        M = cell_start.numel() - 1
        if w.dtype != v.dtype:
            raise TypeError("weights must have the velocity dtype")
        ev = torch.empty(M, dtype=torch.int32, device=v.device) if events else None
        _chk(lib.recombine(self._h, _dt(v), _p(v), _p(w), _p(pid), _p(primary), n, _p(cell_start), M,
                           eps, seed, step, _p(ev)), "recombine")
        return ev

    def p2c_sums(self, q: torch.Tensor, cell_of: torch.Tensor, n_cells: int, out=None):
        """Per-cell sums of the rows of q (nq, n) over the particles of each cell."""
        self._stream()
        nq, n = q.shape
        if out is None:
            out = torch.empty((n_cells, nq), dtype=torch.float64, device=q.device)
        _chk(lib.p2c_sums(self._h, _dt(q), _p(q), nq, _p(cell_of), n, n_cells, _p(out)), "p2c_sums")
        return out

    # -------------------------------------------------------------- learned gate
    def features(self, moments: torch.Tensor):
        self._stream()
        M = moments.shape[0]
        feat = torch.empty((M, 8), dtype=torch.float32, device=moments.device)
        valid = torch.empty(M, dtype=torch.uint8, device=moments.device)
        _chk(lib.pic_features(self._h, _p(moments), M, _p(feat), _p(valid)), "pic_features")
        return feat, valid

    def relaxation(self, v: torch.Tensor, cell_start: torch.Tensor, pid: torch.Tensor, *, dt: float,
                   lnL: float, seed: int, step: int, replicas: int = 8, density=None,
                   dt_scale=None):
        self._stream()
        M = cell_start.numel() - 1
        r = torch.empty(M, dtype=torch.float64, device=v.device)
        _chk(lib.pic_relaxation(self._h, _dt(v), _p(v), v.shape[1], _p(cell_start), _p(pid), M, dt,
                                lnL, _p(density), _p(dt_scale), seed, step, replicas, _p(r)),
             "pic_relaxation")
        return r

    def analytic_relaxation(self, moments: torch.Tensor, *, dt: float, lnL: float, replicas: int = 8,
                            density=None):
        self._stream()
        M = moments.shape[0]
        r = torch.empty(M, dtype=torch.float64, device=moments.device)
        _chk(lib.pic_analytic_relaxation(self._h, _p(moments), M, dt, lnL, _p(density), replicas, _p(r)),
             "pic_analytic_relaxation")
        return r

    def mlp_forward(self, params: torch.Tensor, x: torch.Tensor, bf16: bool = True):
        self._stream()
        prob = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _chk(lib.pic_mlp_forward(self._h, _p(params), _p(x), x.shape[0], int(bf16), _p(prob)),
             "pic_mlp_forward")
        return prob

    def set_dsmc(self, table: dict, mass_ratio: float = 0.0):
        """Cross-section table: float64 numpy arrays 'breaks' [P+1], 'coef'
        [4, P, 4] (coefficient of (E - breaks[p])^q), 'thr' [4]."""
        br = np.ascontiguousarray(table["breaks"], np.float64)
        co = np.ascontiguousarray(table["coef"], np.float64)
        th = np.ascontiguousarray(table["thr"], np.float64)
        f64p = C.POINTER(C.c_double)
        _chk(lib.pic_set_dsmc(self._h, co.shape[1], br.ctypes.data_as(f64p), co.ctypes.data_as(f64p),
                              th.ctypes.data_as(f64p), mass_ratio), "pic_set_dsmc")

    def dsmc_collide(self, v: torch.Tensor, cell_of: torch.Tensor, pid: torch.Tensor, n_cells: int,
                     *, dt: float,
                     seed: int, step: int, pid_base: int, v_new: torch.Tensor, pid_new: torch.Tensor,
                     cell_new: torch.Tensor, count: torch.Tensor, n_gas=None, n_meta=None,
                     n_gas0: float = 1.0, n_meta0: float = 0.0, channel_out=None):
        """DSMC-Coll step in place; new electrons appended to v_new (3, cap)
        at count (int64 device scalar, advanced)."""
        self._stream()
        assert count.dtype == torch.int64 and v_new.dtype == v.dtype
        _chk(lib.dsmc_collide(self._h, _dt(v), _p(v), _p(cell_of), _p(pid), v.shape[1], n_cells,
                              _p(n_gas),
                              _p(n_meta), n_gas0, n_meta0, dt, seed, step, pid_base, _p(v_new),
                              _p(pid_new), _p(cell_new), v_new.shape[1], _p(count), _p(channel_out)),
             "dsmc_collide")

    def gate_infer(self, feat: torch.Tensor, params: torch.Tensor, threshold: float, k_max: int,
                   k_acc: torch.Tensor, bf16: bool = True):
        """(skip uint8, prob float32); k_acc (int32, device) is updated in place."""
        self._stream()
        assert k_acc.dtype == torch.int32 and feat.dtype == torch.float32
        n = feat.shape[0]
        skip = torch.empty(n, dtype=torch.uint8, device=feat.device)
        prob = torch.empty(n, dtype=torch.float32, device=feat.device)
        _chk(lib.gate_infer(self._h, _p(feat), n, _p(params), threshold, k_max, int(bf16), _p(skip),
                            _p(k_acc), _p(prob)), "gate_infer")
        return skip, prob

    def mlp_grad(self, params, x, y, bf16: bool = True):
        self._stream()
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _chk(lib.pic_mlp_grad(self._h, _p(params), _p(x), _p(y), x.shape[0], int(bf16), _p(grad),
                              _p(loss)), "pic_mlp_grad")
        return grad, loss

    def mlp_train_step(self, params, m, v, t: int, lr: float, x, y, bf16: bool = True):
        self._stream()
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _chk(lib.pic_mlp_train_step(self._h, _p(params), _p(m), _p(v), t, lr, _p(x), _p(y),
                                    x.shape[0], int(bf16), _p(loss)), "pic_mlp_train_step")
        return loss

    def train_step(self, feat, label, w_master, adam_state, lr: float):
        """mlp_train_step: bfloat16 step, Adam moments in adam_state (2 x 4801),
        step count kept by the context per w_master."""
        self._stream()
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _chk(lib.mlp_train_step(self._h, _p(feat), _p(label), feat.shape[0], _p(w_master),
                                _p(adam_state), lr, _p(loss)), "mlp_train_step")
        return loss

    def gate_config(self, params, threshold: float, k_max: int = 8, judge_fraction: float = 0.01,
                    tolerance: float = 1e-3, replicas: int = 8, bf16: bool = True):
        self._gate_params = params     # the library keeps the pointer
        _chk(lib.pic_gate_config(self._h, _p(params), threshold, k_max, judge_fraction, tolerance,
                                 replicas, int(bf16)), "pic_gate_config")

    def gate_config_analytic(self, threshold: float, k_max: int = 8, judge_fraction: float = 0.01,
                             tolerance: float = 1e-3, replicas: int = 8):
        self._gate_params = None
        _chk(lib.pic_gate_config_analytic(self._h, threshold, k_max, judge_fraction, tolerance,
                                          replicas), "pic_gate_config_analytic")

    def gate_refresh(self, every: int):
        _chk(lib.pic_gate_refresh(self._h, int(every)), "pic_gate_refresh")

    def gate_reset(self):
        _chk(lib.pic_gate_reset(self._h), "pic_gate_reset")

    def gate_stats(self):
        out = (C.c_int64 * 8)()
        _chk(lib.pic_gate_stats(self._h, out), "pic_gate_stats")
        return dict(zip(GATE_STATS, list(out)))

    def gate_state(self, n_cells: int, device="cuda"):
        self._stream()
        skip = torch.empty(n_cells, dtype=torch.uint8, device=device)
        k = torch.empty(n_cells, dtype=torch.int32, device=device)
        prob = torch.empty(n_cells, dtype=torch.float32, device=device)
        mom = torch.empty((n_cells, 14), dtype=torch.float64, device=device)
        _chk(lib.pic_gate_state(self._h, _p(skip), _p(k), _p(prob), _p(mom)), "pic_gate_state")
        return skip, k, prob, mom

    def autotune(self, v, cell_of, pid, n_cells: int, *, dt: float, lnL: float, flags: int = 0):
        """Picks class thresholds / grid sizes for this state (scratch copy); returns the index."""
        self._stream()
        ch = C.c_int32(-1)
        _chk(lib.pic_autotune(self._h, _dt(v), _p(v), _p(cell_of), _p(pid), v.shape[1], n_cells, dt,
                              lnL, flags, C.byref(ch)), "pic_autotune")
        return ch.value

    # -------------------------------------------------------------- measurement
    def time_kernels(self, on: bool):
        _chk(lib.pic_time_kernels(self._h, int(on)), "pic_time_kernels")

    def kernel_times(self):
        """{slot: (total_ms, launches)} since the previous call."""
        ms = (C.c_double * 20)()
        cnt = (C.c_int64 * 20)()
        _chk(lib.pic_kernel_times(self._h, ms, cnt), "pic_kernel_times")
        return {KT_SLOTS[s]: (ms[s], cnt[s]) for s in range(len(KT_SLOTS)) if cnt[s]}

    # -------------------------------------------------------------- test exports
    def philox(self, seed: int, step: int, domain: int, c0: torch.Tensor, c3: int = 0):
        self._stream()
        out = torch.empty((max(c0.numel(), 1), 4), dtype=torch.int32, device=c0.device)
        _chk(lib.pic_philox(self._h, seed, step, domain, c3, _p(c0), c0.numel(), _p(out)),
             "pic_philox")
        return out[:c0.numel()]

    def pairs(self, cell_start: torch.Tensor, pid: torch.Tensor, seed: int, step: int):
        self._stream()
        n = pid.numel()
        srt = torch.empty(max(n, 1), dtype=torch.int32, device=pid.device)
        par = torch.empty(max(n, 1), dtype=torch.int32, device=pid.device)
        _chk(lib.coulomb_pairs(self._h, _p(cell_start), _p(pid), cell_start.numel() - 1, seed,
                               step, _p(srt), _p(par)), "coulomb_pairs")
        return srt[:n], par[:n]

    def cell_moments(self, v: torch.Tensor, cell_start: torch.Tensor):
        self._stream()
        M = cell_start.numel() - 1
        out = torch.empty((M, 14), dtype=torch.float64, device=v.device)
        _chk(lib.pic_cell_moments(self._h, _dt(v), _p(v), v.shape[1], _p(cell_start), M,
                                  _p(out)), "pic_cell_moments")
        return out

    def unsort(self, v: torch.Tensor, pid: torch.Tensor, cell_of: torch.Tensor):
        self._stream()
        _chk(lib.pic_unsort(self._h, _dt(v), _p(v), _p(pid), _p(cell_of), v.shape[1]),
             "pic_unsort")
