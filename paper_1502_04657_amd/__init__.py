"""MI355X (gfx950) full multigrid eigensolver for Gross-Pitaevskii-type nonlinear
eigenvalue problems (Jia, Xie, Xie, Xu, arXiv:1502.04657).

The compute path is libfmgeig.so (HIP kernels behind the C ABI of include/fmgeig.h).
This module only marshals arguments: PyTorch tensors provide device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _ffi
from ._ffi import FMG_FP64, FMG_MIXED, fmg_options, fmg_problem, fmg_result

__all__ = ["solve", "workspace_bytes", "Solver", "FmgError", "ops", "lib", "to_c_problem", "to_c_options"]


class FmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfmgeig error {code}: {msg}")
        self.code = code


def lib():
    return _ffi.load()


def _check(rc):
    if rc != 0:
        raise FmgError(rc, lib().fmg_last_error().decode())


def to_c_problem(p) -> fmg_problem:
    cp = fmg_problem()
    cp.dim, cp.n_coarse, cp.n_refine = int(p.dim), int(p.n_coarse), int(p.n_refine)
    w = list(p.w_quad) + [0.0] * (3 - len(p.w_quad))
    for k in range(3):
        cp.w_quad[k] = float(w[k])
    cp.w_const = float(p.w_const)
    cp.zeta = float(p.zeta)
    return cp


def to_c_options(o) -> fmg_options:
    co = fmg_options()
    co.tol_lambda = float(o.tol_lambda)
    co.m, co.p = int(o.m), int(o.p)
    co.nu_pre, co.nu_post = int(o.nu_pre), int(o.nu_post)
    co.max_final_steps = int(o.max_final_steps)
    co.newton_max_iter = int(getattr(o, "newton_max_iter", 40))
    co.newton_tol = float(getattr(o, "scf_tol", 1e-13))
    co.precision = FMG_MIXED if o.precision == "mixed" else FMG_FP64
    return co


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def workspace_bytes(problem, options) -> int:
    n = C.c_size_t()
    _check(lib().fmg_workspace_bytes(C.byref(to_c_problem(problem)), C.byref(to_c_options(options)), C.byref(n)))
    return n.value


@dataclasses.dataclass
class Result:
    lam: float
    lambda_rq: float
    norm: float
    dlambda: float
    status: int
    levels: int
    steps_total: int
    newton_total: int
    seconds: float
    history: list
    factor_total: int = 0


class Solver:
    """Holds a device workspace for repeated solves of one problem shape."""

    def __init__(self, problem, options, device="cuda"):
        self.problem, self.options = problem, options
        self.cp, self.co = to_c_problem(problem), to_c_options(options)
        self.ws_bytes = workspace_bytes(problem, options)
        self.ws = torch.empty(self.ws_bytes // 8 + 64, dtype=torch.float64, device=device)
        n = problem.n_coarse << problem.n_refine
        self.ndof = (n - 1) ** problem.dim
        self.device = device

    def solve(self, u_out: torch.Tensor | None = None, stream=None, check=True):
        if u_out is None:
            u_out = torch.empty(self.ndof, dtype=torch.float64, device=self.device)
        res = fmg_result()
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        rc = lib().fmg_solve(C.byref(self.cp), C.byref(self.co), C.c_void_p(aligned),
                             C.c_size_t(self.ws_bytes), _stream(stream), _ptr(u_out),
                             C.c_int64(u_out.numel()), C.byref(res))
        if check:
            _check(rc)
        out = Result(res.lambda_, res.lambda_rq, res.norm, res.dlambda, res.status, res.levels, res.steps_total,
                     res.newton_total, res.seconds, list(res.history[: res.history_len]), res.factor_total)
        return out, u_out


def solve(problem, options, device="cuda", check=True):
    return Solver(problem, options, device).solve(check=check)


from . import ops  # noqa: E402  (needs the helpers above)
