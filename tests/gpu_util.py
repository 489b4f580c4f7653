"""Helpers shared by the GPU parity tests (marshalling only)."""
import numpy as np
import torch


def dev(a: np.ndarray, dtype=None) -> torch.Tensor:
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def host_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def rel_err(v_gpu: np.ndarray, v_ref: np.ndarray, vth: float = 1.0) -> float:
    """max_l ||v_gpu - v_ref||_inf / max(||v_ref||_2, 1e-3 v_th) over particles l."""
    num = np.max(np.abs(v_gpu - v_ref), axis=0)
    den = np.maximum(np.linalg.norm(v_ref, axis=0), 1e-3 * vth)
    return float(np.max(num / den)) if num.size else 0.0
