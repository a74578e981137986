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

__all__ = ["solve", "solve_alloc", "workspace_bytes", "footprint_bytes", "Solver", "batch_solve", "BatchPlan", "Server", "FmgError", "ops", "lib",
           "to_c_problem", "to_c_options"]


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
    a = list(getattr(p, "diffusion", (1.0, 1.0, 1.0))) + [1.0] * 3
    for k in range(3):
        cp.diffusion[k] = float(a[k])
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
    co.newton_fixed_iters = int(getattr(o, "newton_fixed_iters", 0))
    co.smoother = _ffi.FMG_SMOOTH_CG if getattr(o, "smoother", "sgs") == "cg" else _ffi.FMG_SMOOTH_SGS
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
    wait_seconds: float = 0.0
    residual: float = 0.0
    gamma_est: float = -1.0


def _result(res: fmg_result) -> "Result":
    return Result(res.lambda_, res.lambda_rq, res.norm, res.dlambda, res.status, res.levels, res.steps_total,
                  res.newton_total, res.seconds, list(res.history[: res.history_len]), res.factor_total,
                  res.wait_seconds, res.residual, res.gamma_est)


def footprint_bytes(problem, options) -> int:
    """Device bytes one solve holds (admission footprint); raises for invalid input."""
    n = lib().fmg_footprint_bytes(C.byref(to_c_problem(problem)), C.byref(to_c_options(options)))
    if n == 0:
        raise FmgError(_ffi.FMG_EINVAL, "invalid problem or options")
    return n


def _ndof(problem) -> int:
    n = problem.n_coarse << problem.n_refine
    return (n - 1) ** problem.dim


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
        return _result(res), u_out


def solve(problem, options, device="cuda", check=True):
    return Solver(problem, options, device).solve(check=check)


def solve_alloc(problem, options, u_out=None, stream=None, check=True):
    """fmg_solve_alloc: the library allocates and frees the workspace.  u_out may be a CUDA
    or a CPU tensor (float64, (n-1)^dim elements); a new CUDA tensor when None."""
    if u_out is None:
        u_out = torch.empty(_ndof(problem), dtype=torch.float64, device="cuda")
    assert u_out.dtype == torch.float64 and u_out.is_contiguous()
    res = fmg_result()
    rc = lib().fmg_solve_alloc(C.byref(to_c_problem(problem)), C.byref(to_c_options(options)), _stream(stream),
                               _ptr(u_out), C.c_int64(u_out.numel()), C.byref(res))
    if check:
        _check(rc)
    return _result(res), u_out


def batch_solve(problems, options, device="cuda", stream=None, check=True):
    """fmg_batch_solve over lists of problems and options (one options object is reused for
    every problem).  Returns ([Result], [u tensors])."""
    k = len(problems)
    opts = options if isinstance(options, (list, tuple)) else [options] * k
    cps = (fmg_problem * k)(*[to_c_problem(p) for p in problems])
    cos = (fmg_options * k)(*[to_c_options(o) for o in opts])
    us = [torch.empty(_ndof(p), dtype=torch.float64, device=device) for p in problems]
    ptrs = (C.c_void_p * k)(*[u.data_ptr() for u in us])
    lens = (C.c_int64 * k)(*[u.numel() for u in us])
    res = (fmg_result * k)()
    rc = lib().fmg_batch_solve(k, cps, cos, _stream(stream), ptrs, lens, res)
    if check:
        _check(rc)
    return [_result(r) for r in res], us


class BatchPlan:
    """fmg_batch_plan_*: a batch set up once (one pool, each instance's kernel sequence
    captured into HIP graphs) and replayed by run().  Output tensors are allocated once and
    reused by every run."""

    def __init__(self, problems, options, device="cuda", stream=None):
        k = len(problems)
        opts = options if isinstance(options, (list, tuple)) else [options] * k
        cps = (fmg_problem * k)(*[to_c_problem(p) for p in problems])
        cos = (fmg_options * k)(*[to_c_options(o) for o in opts])
        self.problems = list(problems)
        h = lib().fmg_batch_plan_create(k, cps, cos, _stream(stream))
        if not h:
            raise FmgError(_ffi.FMG_EINVAL, lib().fmg_last_error().decode())
        self._h = h
        self.us = [torch.empty(_ndof(p), dtype=torch.float64, device=device) for p in problems]
        self._ptrs = (C.c_void_p * k)(*[u.data_ptr() for u in self.us])
        self._lens = (C.c_int64 * k)(*[u.numel() for u in self.us])

    def run(self, check=True):
        """Replay every instance; returns ([Result], [u tensors]) (the tensors are the plan's
        and are overwritten by the next run)."""
        k = len(self.problems)
        res = (fmg_result * k)()
        rc = lib().fmg_batch_plan_run(self._h, self._ptrs, self._lens, res)
        if check:
            _check(rc)
        return [_result(r) for r in res], self.us

    def close(self):
        if self._h:
            lib().fmg_batch_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """fmg_server_*: continuous batching of eigensolve requests within an HBM budget."""

    def __init__(self, hbm_budget=0, max_slots=8, stream=None, device="cuda"):
        self.device = device
        self._stream = _stream(stream)
        h = lib().fmg_server_create(C.c_size_t(hbm_budget), max_slots, self._stream)
        if not h:
            raise FmgError(_ffi.FMG_ENOMEM, lib().fmg_last_error().decode())
        self._h = C.c_void_p(h)
        self._problems = {}

    def submit(self, problem, options) -> int:
        t = C.c_uint64()
        _check(lib().fmg_server_submit(self._h, C.byref(to_c_problem(problem)), C.byref(to_c_options(options)),
                                       C.byref(t)))
        self._problems[t.value] = problem
        return t.value

    def poll(self, ticket, want_u=True, check=True):
        """None while pending; else (Result, u or None)."""
        p = self._problems[ticket]
        u = torch.empty(_ndof(p), dtype=torch.float64, device=self.device) if want_u else None
        res = fmg_result()
        rc = lib().fmg_server_poll(self._h, C.c_uint64(ticket), C.byref(res),
                                   C.c_void_p(u.data_ptr()) if u is not None else None,
                                   C.c_int64(u.numel() if u is not None else 0))
        if rc == _ffi.FMG_PENDING:
            return None
        del self._problems[ticket]
        if check:
            _check(rc)
        return _result(res), u

    def close(self):
        if self._h:
            lib().fmg_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from . import ops  # noqa: E402  (needs the helpers above)
