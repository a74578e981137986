"""Single steps of the method through the C ABI (level-layout device tensors).

Each function marshals torch tensors into the matching fmg_op_* call; the arithmetic
runs in the HIP kernels of libfmgeig.so."""
from __future__ import annotations

import ctypes as C

import torch

from . import FMG_FP64, FMG_MIXED, _check, _ptr, _stream, lib, to_c_options, to_c_problem


def level_pitch(dim: int, n: int) -> int:
    return int(lib().fmg_level_pitch(dim, n))


def level_elems(dim: int, n: int) -> int:
    return int(lib().fmg_level_elems(dim, n))


def new_level(dim, n, dtype=torch.float64, device="cuda"):
    return torch.zeros(level_elems(dim, n), dtype=dtype, device=device)


def _prec(t: torch.Tensor):
    return FMG_MIXED if t.dtype == torch.float32 else FMG_FP64


def pack(dim, n, compact: torch.Tensor, level: torch.Tensor | None = None):
    level = new_level(dim, n, device=compact.device) if level is None else level
    _check(lib().fmg_pack(dim, n, _ptr(compact), _ptr(level), _stream()))
    return level


def unpack(dim, n, level: torch.Tensor):
    out = torch.empty((n - 1) ** dim, dtype=torch.float64, device=level.device)
    _check(lib().fmg_unpack(dim, n, _ptr(level), _ptr(out), _stream()))
    return out


def rhs(problem, n, lam, u_level):
    b = torch.zeros_like(u_level)
    _check(lib().fmg_op_rhs(C.byref(to_c_problem(problem)), n, C.c_double(lam), _ptr(u_level), _ptr(b), _stream()))
    return b


def smooth(dim, n, x_level, f_level, sweeps):
    _check(lib().fmg_op_smooth(dim, n, _prec(x_level), _ptr(x_level), _ptr(f_level), sweeps, _stream()))
    return x_level


def cg_smooth(dim, n, x_level, f_level, steps):
    es = x_level.element_size()
    e = (es * level_elems(dim, n) + 255) // 256 * 256
    nbytes = 3 * e + 8 * (512 + 8)
    scratch = torch.zeros(nbytes // 8 + 64, dtype=torch.float64, device=x_level.device)
    base = (scratch.data_ptr() + 255) // 256 * 256
    _check(lib().fmg_op_cg_smooth(dim, n, _prec(x_level), _ptr(x_level), _ptr(f_level), steps, C.c_void_p(base),
                                  C.c_size_t(nbytes), _stream()))
    return x_level


def residual_restrict(dim, n, x_level, f_level):
    rc = torch.zeros(level_elems(dim, n // 2), dtype=x_level.dtype, device=x_level.device)
    _check(lib().fmg_op_residual_restrict(dim, n, _prec(x_level), _ptr(x_level), _ptr(f_level), _ptr(rc), _stream()))
    return rc


def prolong(dim, n, xc_level, xf_level=None, accumulate=False):
    if xf_level is None:
        xf_level = torch.zeros(level_elems(dim, n), dtype=xc_level.dtype, device=xc_level.device)
    _check(lib().fmg_op_prolong(dim, n, _prec(xc_level), _ptr(xc_level), _ptr(xf_level), int(accumulate), _stream()))
    return xf_level


def coarse_solve(dim, n, f_level):
    x = torch.zeros_like(f_level)
    _check(lib().fmg_op_coarse_solve(dim, n, _prec(f_level), _ptr(f_level), _ptr(x), _stream()))
    return x


def vcycle(problem, options, x_level, f_level):
    n = C.c_size_t()
    _check(lib().fmg_workspace_bytes(C.byref(to_c_problem(problem)), C.byref(to_c_options(options)), C.byref(n)))
    ws = torch.empty(n.value // 8 + 64, dtype=torch.float64, device=x_level.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    _check(lib().fmg_op_vcycle(problem.dim, problem.n_coarse, problem.n_refine + 1, options.nu_pre, options.nu_post,
                               _ptr(x_level), _ptr(f_level), C.c_void_p(base), C.c_size_t(n.value), _stream()))
    torch.cuda.synchronize()
    return x_level


def moments_layout(dim, n_coarse, n):
    per = C.c_int32()
    scr = C.c_size_t()
    _check(lib().fmg_moments_layout(dim, n_coarse, n, C.byref(per), C.byref(scr)))
    return per.value, scr.value


def moments(problem, n, ut_level, chunk_cells=0):
    """fmg_op_moments (chunk_cells = 0) or fmg_op_moments_chunked."""
    per, scr = moments_layout(problem.dim, problem.n_coarse, n)
    ncell = problem.n_coarse ** problem.dim
    ne = 2 if problem.dim == 2 else 6
    out = torch.zeros(ncell * ne * per, dtype=torch.float64, device=ut_level.device)
    if chunk_cells:
        s = n // problem.n_coarse
        groups = (s * (s - 1) // 2, s) if problem.dim == 2 else (s * (s - 1) * (s - 2) // 6, s * s)
        blocks = ncell * ne * sum(-(-g // chunk_cells) for g in groups)
        scr = max(scr, blocks * (23 if problem.dim == 2 else 39) * 8)
    scratch = torch.empty(scr // 8 + 32, dtype=torch.float64, device=ut_level.device)
    if chunk_cells:
        _check(lib().fmg_op_moments_chunked(C.byref(to_c_problem(problem)), n, _ptr(ut_level), _ptr(out),
                                            _ptr(scratch), C.c_size_t(scratch.numel() * 8), chunk_cells, _stream()))
    else:
        _check(lib().fmg_op_moments(C.byref(to_c_problem(problem)), n, _ptr(ut_level), _ptr(out), _ptr(scratch),
                                    C.c_size_t(scratch.numel() * 8), _stream()))
    return out.view(ncell * ne, per)


def _small_scratch(problem, device):
    n = C.c_size_t()
    _check(lib().fmg_small_scratch_bytes(problem.dim, problem.n_coarse, C.byref(n)))
    t = torch.zeros(n.value // 8 + 64, dtype=torch.float64, device=device)
    base = (t.data_ptr() + 255) // 256 * 256
    return t, C.c_void_p(base), n.value


def augmented_matrices(problem, mom, x):
    N1 = (problem.n_coarse - 1) ** problem.dim + 1
    A = torch.zeros(N1 * N1, dtype=torch.float64, device=mom.device)
    B = torch.zeros_like(A)
    S = torch.zeros_like(A)
    keep, base, nbytes = _small_scratch(problem, mom.device)
    _check(lib().fmg_op_augmented_matrices(C.byref(to_c_problem(problem)), _ptr(mom), _ptr(x), _ptr(A), _ptr(B),
                                           _ptr(S), base, C.c_size_t(nbytes), _stream()))
    torch.cuda.synchronize()
    del keep
    return A.view(N1, N1), B.view(N1, N1), S.view(N1, N1)


def augmented_solve(problem, options, mom):
    xc = new_level(problem.dim, problem.n_coarse, device=mom.device)
    keep, base, nbytes = _small_scratch(problem, mom.device)
    lam, c = C.c_double(), C.c_double()
    it, gs = C.c_int32(), C.c_int32()
    _check(lib().fmg_op_augmented_solve(C.byref(to_c_problem(problem)), C.byref(to_c_options(options)), _ptr(mom),
                                        _ptr(xc), base, C.c_size_t(nbytes), _stream(), C.byref(lam), C.byref(c),
                                        C.byref(it), C.byref(gs)))
    del keep
    return lam.value, c.value, xc, it.value, bool(gs.value)


def coarse_nonlinear(problem, options, device="cuda"):
    xc = new_level(problem.dim, problem.n_coarse, device=device)
    keep, base, nbytes = _small_scratch(problem, device)
    lam = C.c_double()
    it, gs = C.c_int32(), C.c_int32()
    _check(lib().fmg_op_coarse_nonlinear(C.byref(to_c_problem(problem)), C.byref(to_c_options(options)), _ptr(xc),
                                         base, C.c_size_t(nbytes), _stream(), C.byref(lam), C.byref(it), C.byref(gs)))
    del keep
    return lam.value, xc, it.value, bool(gs.value)


def form_u(dim, n_coarse, n, c, xc_level, u_level):
    scratch = torch.zeros(8, dtype=torch.float64, device=u_level.device)
    _check(lib().fmg_op_form_u(dim, n_coarse, n, C.c_double(c), _ptr(xc_level), _ptr(u_level), _ptr(scratch),
                               _stream()))
    return u_level


def forms(problem, n, u_level):
    scratch = torch.zeros(4200, dtype=torch.float64, device=u_level.device)
    out = (C.c_double * 4)()
    _check(lib().fmg_op_forms(C.byref(to_c_problem(problem)), n, _ptr(u_level), C.cast(out, C.c_void_p), _ptr(scratch), _stream()))
    return tuple(out)
