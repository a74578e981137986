"""The C-ABI library loads and exports every function include/fmgeig.h declares (no GPU
needed: nothing here launches a kernel), and the pure host-side entry points behave."""
import ctypes as C
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmgeig.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fmg_[a-z_0-9]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1502_04657_amd import _ffi
    return _ffi.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fmg_solve", "fmg_workspace_bytes", "fmg_op_rhs", "fmg_op_smooth", "fmg_op_moments",
                 "fmg_op_augmented_solve", "fmg_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1502_04657_amd import _ffi
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _ffi.SIGNATURES, f"binding lacks {name}"


def test_workspace_bytes_and_validation(lib):
    from paper_1502_04657_amd import to_c_options, to_c_problem
    n = C.c_size_t()
    p, o = to_c_problem(W.LARGE_2D), to_c_options(W.Options())
    assert lib.fmg_workspace_bytes(C.byref(p), C.byref(o), C.byref(n)) == 0
    # u and b on every level plus the V-cycle arrays below the top: about 27 bytes/dof
    assert 20 * W.LARGE_2D.dofs() < n.value < 60 * W.LARGE_2D.dofs()
    o_mixed = to_c_options(W.Options(precision="mixed"))
    m = C.c_size_t()
    assert lib.fmg_workspace_bytes(C.byref(p), C.byref(o_mixed), C.byref(m)) == 0
    bad = to_c_problem(W.Problem(4, 8, 2))
    assert lib.fmg_workspace_bytes(C.byref(bad), C.byref(o), C.byref(n)) == -1
    assert b"dim" in lib.fmg_last_error()
    bad = to_c_problem(W.Problem(2, 8, 2, zeta=-1.0))
    assert lib.fmg_workspace_bytes(C.byref(bad), C.byref(o), C.byref(n)) == -1
    bad = to_c_problem(W.Problem(2, 8, 2, zeta=float("nan")))
    assert lib.fmg_workspace_bytes(C.byref(bad), C.byref(o), C.byref(n)) == -1
    bad_o = to_c_options(W.Options(m=0))
    assert lib.fmg_workspace_bytes(C.byref(p), C.byref(bad_o), C.byref(n)) == -1
    bad_o = to_c_options(W.Options(newton_fixed_iters=-1))
    assert lib.fmg_workspace_bytes(C.byref(p), C.byref(bad_o), C.byref(n)) == -1
    bad_o = to_c_options(W.Options(newton_fixed_iters=1000))
    assert lib.fmg_workspace_bytes(C.byref(p), C.byref(bad_o), C.byref(n)) == -1
    assert b"newton_fixed_iters" in lib.fmg_last_error()


def test_level_layout(lib):
    assert lib.fmg_level_pitch(2, 8) == 16
    assert lib.fmg_level_pitch(2, 2048) == 2064
    assert lib.fmg_level_elems(2, 8) == 9 * 16
    assert lib.fmg_level_elems(3, 8) == 9 * 9 * 16
    assert lib.fmg_level_elems(5, 8) == -1


def test_solve_rejects_bad_sizes_before_touching_the_device(lib):
    from paper_1502_04657_amd import _ffi, to_c_options, to_c_problem
    p, o = to_c_problem(W.SMALL_2D), to_c_options(W.Options())
    res = _ffi.fmg_result()
    # wrong u_len is rejected on the host
    rc = lib.fmg_solve(C.byref(p), C.byref(o), C.c_void_p(256), C.c_size_t(1 << 30), None, C.c_void_p(256),
                       C.c_int64(5), C.byref(res))
    assert rc == -1 and b"u_len" in lib.fmg_last_error()
    # too small a workspace
    rc = lib.fmg_solve(C.byref(p), C.byref(o), C.c_void_p(256), C.c_size_t(16), None, C.c_void_p(256),
                       C.c_int64(127 * 127), C.byref(res))
    assert rc == -2


def test_footprint_is_the_aligned_workspace(lib):
    from paper_1502_04657_amd import to_c_options, to_c_problem
    for prob, opt in ((W.LARGE_2D, W.Options()), (W.SMALL_2D, W.Options(precision="mixed")),
                      (W.LARGE_3D, W.Options(tol_lambda=1e-9))):
        p, o = to_c_problem(prob), to_c_options(opt)
        n = C.c_size_t()
        assert lib.fmg_workspace_bytes(C.byref(p), C.byref(o), C.byref(n)) == 0
        f = lib.fmg_footprint_bytes(C.byref(p), C.byref(o))
        assert f % 256 == 0 and n.value <= f < n.value + 256
        assert lib.fmg_footprint_bytes(C.byref(p), C.byref(o)) == f   # pure
    bad = to_c_problem(W.Problem(2, 1, 3))
    assert lib.fmg_footprint_bytes(C.byref(bad), C.byref(to_c_options(W.Options()))) == 0


def test_allocator_hooks_must_come_in_pairs(lib):
    alloc_t = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
    fake = alloc_t(lambda n, ctx: None)
    assert lib.fmg_set_allocator(C.cast(fake, C.c_void_p), None, None) == -1
    assert b"both" in lib.fmg_last_error()
    assert lib.fmg_set_allocator(None, None, None) == 0


def test_batch_validates_every_instance_before_any_work(lib):
    from paper_1502_04657_amd import _ffi, to_c_options, to_c_problem
    k = 3
    probs = (_ffi.fmg_problem * k)(to_c_problem(W.SMALL_2D), to_c_problem(W.Problem(2, 8, 2)),
                                   to_c_problem(W.Problem(2, 8, 2, zeta=-2.0)))
    opts = (_ffi.fmg_options * k)(*[to_c_options(W.Options())] * k)
    ptrs = (C.c_void_p * k)(256, 256, 256)
    res = (_ffi.fmg_result * k)()
    # the third instance is invalid: rejected on the host, nothing allocated or launched
    lens = (C.c_int64 * k)(127 ** 2, 31 ** 2, 31 ** 2)
    assert lib.fmg_batch_solve(k, probs, opts, None, ptrs, lens, res) == -1
    assert b"instance 2" in lib.fmg_last_error()
    # a wrong length
    probs[2] = to_c_problem(W.Problem(2, 8, 2))
    lens[1] = 5
    assert lib.fmg_batch_solve(k, probs, opts, None, ptrs, lens, res) == -1
    assert b"instance 1" in lib.fmg_last_error() and b"u_len" in lib.fmg_last_error()
    assert lib.fmg_batch_solve(0, None, None, None, None, None, None) == 0
    assert lib.fmg_batch_solve(-1, None, None, None, None, None, None) == -1


def test_diffusion_coefficient_is_validated(lib):
    """A = diag(diffusion): each entry finite and > 0, or all zero (the identity)."""
    from paper_1502_04657_amd import _ffi, to_c_problem, to_c_options
    o = to_c_options(W.Options())
    nb = C.c_size_t()
    for a, ok in (((1.0, 2.0, 0.5), True), ((0.0, 0.0, 0.0), True), ((1.0, -1.0, 1.0), False),
                  ((1.0, float("nan"), 1.0), False), ((0.0, 1.0, 1.0), False)):
        p = to_c_problem(W.Problem(2, 8, 2))
        for k in range(3):
            p.diffusion[k] = a[k]
        rc = lib.fmg_workspace_bytes(C.byref(p), C.byref(o), C.byref(nb))
        assert (rc == 0) == ok, a
    # the third entry is ignored in 2D
    p = to_c_problem(W.Problem(2, 8, 2, diffusion=(1.0, 2.0, -5.0)))
    assert lib.fmg_workspace_bytes(C.byref(p), C.byref(o), C.byref(nb)) == 0


def test_batch_plan_validates_before_any_device_work(lib):
    from paper_1502_04657_amd import _ffi
    assert lib.fmg_batch_plan_create(0, None, None, None) is None
    assert b"count" in lib.fmg_last_error()
    probs = (_ffi.fmg_problem * 1)()
    opts = (_ffi.fmg_options * 1)()
    probs[0].dim = 4                                   # invalid dimension
    assert lib.fmg_batch_plan_create(1, probs, opts, None) is None
    assert b"instance 0" in lib.fmg_last_error()
    assert lib.fmg_batch_plan_run(None, None, None, None) == _ffi.FMG_EINVAL
    lib.fmg_batch_plan_destroy(None)


def test_small_level_tile_choice_round_trips(lib):
    """The tuning field of the 3D small levels' LDS tiles: 0 selects the default (on), 1 and
    -1 are kept, anything else is refused and changes nothing."""
    import ctypes as C
    from paper_1502_04657_amd import _ffi
    saved = _ffi.fmg_tuning()
    assert lib.fmg_get_tuning(C.byref(saved)) == 0
    try:
        for v, want in ((0, 1), (-1, -1), (1, 1)):
            t = _ffi.fmg_tuning()
            assert lib.fmg_get_tuning(C.byref(t)) == 0
            t.vtile3d = v
            assert lib.fmg_set_tuning(C.byref(t)) == 0
            got = _ffi.fmg_tuning()
            assert lib.fmg_get_tuning(C.byref(got)) == 0 and got.vtile3d == want
        t.vtile3d = 2
        assert lib.fmg_set_tuning(C.byref(t)) == _ffi.FMG_EINVAL
        got = _ffi.fmg_tuning()
        assert lib.fmg_get_tuning(C.byref(got)) == 0 and got.vtile3d == 1
    finally:
        assert lib.fmg_set_tuning(C.byref(saved)) == 0


def test_profile_requests_are_validated(lib):
    """Unknown kinds and bad capacities are refused before any event is created, and ending
    a profile that was never begun is an error."""
    from paper_1502_04657_amd import _ffi
    for kind, cap in ((0, 8), (6, 8), (_ffi.FMG_PROF_MOMENTS3D, 0), (_ffi.FMG_PROF_RHS3D, -1)):
        assert lib.fmg_profile_begin(kind, cap) == _ffi.FMG_EINVAL
    assert lib.fmg_profile_end(None) == _ffi.FMG_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of fmg_problem, fmg_options and fmg_result have the field offsets
    and sizes a C compiler gives the header's structs."""
    from paper_1502_04657_amd import _ffi
    structs = {"fmg_problem": _ffi.fmg_problem, "fmg_options": _ffi.fmg_options, "fmg_result": _ffi.fmg_result,
               "fmg_tuning": _ffi.fmg_tuning, "fmg_kernel_profile": _ffi.fmg_kernel_profile}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fmgeig.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            cname = "lambda" if fname == "lambda_" else fname
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {cname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        sname, field, val = line.split()
        cls = structs[sname]
        got = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), line
