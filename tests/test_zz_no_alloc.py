"""fmg_solve_static, the entry point that allocates nothing (its workspace is the library's
static device array), called through the C ABI and checked against fmg_solve on the same
problems: two calls in a row, the second on a smaller mesh, each bit for bit equal to
fmg_solve's result; and a problem whose workspace exceeds the static array is refused."""
import ctypes as C

import pytest

import workloads as W

torch = pytest.importorskip("torch")


def _call_static(prob, opts, u):
    from paper_1502_04657_amd import _ffi, lib, to_c_options, to_c_problem
    res = _ffi.fmg_result()
    rc = lib().fmg_solve_static(C.byref(to_c_problem(prob)), C.byref(to_c_options(opts)),
                                C.c_void_p(torch.cuda.current_stream().cuda_stream), C.c_void_p(u.data_ptr()),
                                C.c_int64(u.numel()), C.byref(res))
    return rc, res


def test_static_workspace_refuses_problems_above_its_size():
    from paper_1502_04657_amd import _ffi, lib, to_c_options, to_c_problem, workspace_bytes
    prob, opts = W.LARGE_2D, W.Options()
    assert workspace_bytes(prob, opts) > (64 << 20)
    res = _ffi.fmg_result()
    rc = lib().fmg_solve_static(C.byref(to_c_problem(prob)), C.byref(to_c_options(opts)), None, None,
                                C.c_int64(0), C.byref(res))
    assert rc == _ffi.FMG_ENOMEM
    assert b"static workspace" in lib().fmg_last_error()


@pytest.mark.gpu
def test_static_workspace_solves_match_fmg_solve():
    from paper_1502_04657_amd import Solver, workspace_bytes
    cases = [(W.Problem(2, 16, 5, (1.0, 1.0, 0.0), 0.0, 100.0), W.Options(tol_lambda=1e-9)),             # n = 512
             (W.Problem(3, 4, 2, (0.8, 1.1, 1.4), 0.0, 10.0), W.Options(tol_lambda=1e-9, precision="mixed"))]  # n = 16
    for prob, opts in cases:
        assert workspace_bytes(prob, opts) <= (64 << 20)
        ref, u_ref = Solver(prob, opts).solve()
        u = torch.full_like(u_ref, float("nan"))
        rc, res = _call_static(prob, opts, u)
        torch.cuda.synchronize()
        assert rc == 0
        assert res.lambda_ == ref.lam
        assert res.steps_total == ref.steps_total
        assert list(res.history[: res.history_len]) == ref.history
        assert torch.equal(u, u_ref)
