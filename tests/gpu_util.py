"""Helpers shared by the GPU tests: host-side level layout and oracle caches."""
from __future__ import annotations

import functools

import numpy as np
import torch

import workloads as W


def pitch(n: int) -> int:
    # the library pads rows to a multiple of 16 elements (checked against the library)
    return ((n + 1) + 15) // 16 * 16


def level_np(dim: int, n: int, compact: np.ndarray) -> np.ndarray:
    """Compact interior vector -> padded level layout, built independently on the host."""
    P = pitch(n)
    m = n - 1
    if dim == 2:
        lv = np.zeros((n + 1, P))
        lv[1:n, 1:n] = compact.reshape(m, m)
    else:
        lv = np.zeros((n + 1, n + 1, P))
        lv[1:n, 1:n, 1:n] = compact.reshape(m, m, m)
    return lv.ravel()


def compact_np(dim: int, n: int, level: np.ndarray) -> np.ndarray:
    P = pitch(n)
    if dim == 2:
        return level.reshape(n + 1, P)[1:n, 1:n].ravel().copy()
    return level.reshape(n + 1, n + 1, P)[1:n, 1:n, 1:n].ravel().copy()


def to_dev(a: np.ndarray, dtype=torch.float64) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def dev_level(dim, n, compact, dtype=torch.float64):
    return to_dev(level_np(dim, n, compact), dtype)


def host_compact(dim, n, t: torch.Tensor) -> np.ndarray:
    return compact_np(dim, n, t.double().cpu().numpy())


def rel_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@functools.lru_cache(maxsize=None)
def oracle_hierarchy(problem: W.Problem):
    from oracle.fmg import Hierarchy
    return Hierarchy(problem)


def m_norm(M, v):
    return float(np.sqrt(abs(v @ (M @ v))))
