"""The library's per-launch measurement hooks (fmg_profile_begin / fmg_profile_end) record
the finest-level launches of each kernel kind during whole solves, with the algorithmic bytes
and units of work their declaration states."""
import ctypes as C

import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _profiled(prob, opts, kind, solves=2):
    from paper_1502_04657_amd import Solver, _ffi, lib
    s = Solver(prob, opts)
    u = torch.empty(s.ndof, dtype=torch.float64, device="cuda")
    s.solve(u)
    torch.cuda.synchronize()
    assert lib().fmg_profile_begin(kind, 256) == 0
    res = []
    try:
        for _ in range(solves):
            res.append(s.solve(u)[0])
    finally:
        prof = _ffi.fmg_kernel_profile()
        assert lib().fmg_profile_end(C.byref(prof)) == 0
    return prof, res


@pytest.mark.parametrize("kind_name, per_node_bytes", [("FMG_PROF_RHS3D", 16.0), ("FMG_PROF_MOMENTS3D", 8.0),
                                                       ("FMG_PROF_VPRE3D_F64", 24.0),
                                                       ("FMG_PROF_VPOST3D_F64", None)])
def test_3d_hooks_record_finest_launches(kind_name, per_node_bytes):
    from paper_1502_04657_amd import _ffi
    prob = W.Problem(3, 4, 5, (1.0, 1.0, 1.0), 0.0, 10.0)            # n = 128: fused passes apply
    kind = getattr(_ffi, kind_name)
    prof, res = _profiled(prob, W.Options(tol_lambda=1e-9), kind)
    n = prob.n_fine
    nf, ncs = (n - 1) ** 3, (n // 2 - 1) ** 3
    assert prof.launches >= 2 and prof.seconds > 0.0
    per = prof.bytes / prof.launches
    if per_node_bytes is None:
        assert per == pytest.approx(8.0 * (3 * nf + ncs))
    else:
        assert per == pytest.approx(per_node_bytes * nf)
    units = prof.units / prof.launches
    assert units == pytest.approx(float(n) ** 3 if kind_name == "FMG_PROF_MOMENTS3D" else float(nf))
    # the hook does not change the solve
    assert res[0].lam == res[1].lam


def test_2d_hook_records_wide_tile_post_passes():
    from paper_1502_04657_amd import _ffi
    prob = W.Problem(2, 16, 5, (1.0, 1.0, 0.0), 0.0, 100.0)          # n = 512
    prof, _ = _profiled(prob, W.Options(tol_lambda=1e-9), _ffi.FMG_PROF_VPOST2D_F64)
    nf, ncs = 511 ** 2, 255 ** 2
    assert prof.launches >= 2
    assert prof.bytes / prof.launches == pytest.approx(8.0 * (3 * nf + ncs))
