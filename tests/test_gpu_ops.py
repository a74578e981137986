"""GPU parity of every step of the hot path against the oracle, step by step, through the
C ABI: layout, smoother, residual/restriction, prolongation, coarse solve, V-cycle,
right-hand side (3.4), Rayleigh-quotient forms, moments and augmented matrices of (3.6),
the two small nonlinear solves and the formation of u.  FP64 results must agree to
~1e-12 relative (only the summation order differs); FP32 kernels to single precision."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from tests.gpu_util import (compact_np, dev_level, host_compact, level_np, oracle_hierarchy, pitch, rel_err,
                            to_dev)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ops():
    from paper_1502_04657_amd import ops as o
    return o


def _mesh_ops(dim, n, W_=None):
    from oracle import fem
    from oracle.mesh import Mesh
    m = Mesh(dim, n)
    return m, fem.stiffness(m)


# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim, n", [(2, 7), (2, 100), (3, 5), (3, 20)])
def test_pack_unpack_and_pitch(ops, dim, n):
    assert ops.level_pitch(dim, n) == pitch(n)
    c = W.random_interior(dim, n, seed=1)
    lv = ops.pack(dim, n, to_dev(c))
    assert np.array_equal(lv.cpu().numpy(), level_np(dim, n, c))
    assert np.array_equal(ops.unpack(dim, n, lv).cpu().numpy(), c)


@pytest.mark.parametrize("dim, n, sweeps", [(2, 6, 2), (2, 40, 1), (2, 130, 2), (3, 4, 2), (3, 12, 2), (3, 19, 1)])
def test_smoother_matches_red_black_sgs(ops, dim, n, sweeps):
    from oracle.mg import Level, sgs_sweep
    m, K = _mesh_ops(dim, n)
    lv = Level(m, K)
    x0 = W.random_interior(dim, n, seed=2)
    f = W.random_interior(dim, n, seed=3)
    xo = x0.copy()
    for _ in range(sweeps):
        sgs_sweep(lv, xo, f)
    xg = ops.smooth(dim, n, dev_level(dim, n, x0), dev_level(dim, n, f), sweeps)
    assert rel_err(host_compact(dim, n, xg), xo) < 1e-13
    # FP32 variant
    x32 = ops.smooth(dim, n, dev_level(dim, n, x0, torch.float32), dev_level(dim, n, f, torch.float32), sweeps)
    assert rel_err(host_compact(dim, n, x32), xo) < 2e-5


@pytest.mark.parametrize("dim, n", [(2, 8), (2, 98), (2, 132), (3, 8), (3, 22)])
def test_residual_restriction(ops, dim, n):
    from oracle import fem
    from oracle.mesh import Mesh
    mf, K = _mesh_ops(dim, n)
    P = fem.prolongation(mf, Mesh(dim, n // 2))
    x = W.random_interior(dim, n, seed=4)
    f = W.random_interior(dim, n, seed=5)
    ref = P.T @ (f - K @ x)
    rc = ops.residual_restrict(dim, n, dev_level(dim, n, x), dev_level(dim, n, f))
    assert rel_err(host_compact(dim, n // 2, rc), ref) < 1e-13
    rc32 = ops.residual_restrict(dim, n, dev_level(dim, n, x, torch.float32), dev_level(dim, n, f, torch.float32))
    assert rel_err(host_compact(dim, n // 2, rc32), ref) < 1e-5


@pytest.mark.parametrize("dim, n", [(2, 8), (2, 98), (3, 8), (3, 22)])
def test_prolongation(ops, dim, n):
    from oracle import fem
    from oracle.mesh import Mesh
    P = fem.prolongation(Mesh(dim, n), Mesh(dim, n // 2))
    xc = W.random_interior(dim, n // 2, seed=6)
    xf0 = W.random_interior(dim, n, seed=7)
    got = ops.prolong(dim, n, dev_level(dim, n // 2, xc))
    assert rel_err(host_compact(dim, n, got), P @ xc) < 1e-14
    acc = ops.prolong(dim, n, dev_level(dim, n // 2, xc), dev_level(dim, n, xf0), accumulate=True)
    assert rel_err(host_compact(dim, n, acc), xf0 + P @ xc) < 1e-14


@pytest.mark.parametrize("dim, n", [(2, 2), (2, 8), (2, 16), (2, 32), (3, 2), (3, 4), (3, 8), (3, 16)])
def test_coarse_solve_is_exact(ops, dim, n):
    _, K = _mesh_ops(dim, n)
    f = W.random_interior(dim, n, seed=8)
    ref = sla.cho_solve(sla.cho_factor(K.toarray()), f)
    x = ops.coarse_solve(dim, n, dev_level(dim, n, f))
    assert rel_err(host_compact(dim, n, x), ref) < 1e-13
    x32 = ops.coarse_solve(dim, n, dev_level(dim, n, f, torch.float32))
    assert rel_err(host_compact(dim, n, x32), ref) < 1e-5


@pytest.mark.parametrize("dim, nc, levels", [(2, 8, 3), (2, 16, 4), (2, 12, 4), (2, 6, 7), (3, 4, 3), (3, 2, 4),
                                             (3, 3, 4), (3, 4, 5), (3, 5, 4)])
def test_vcycle(ops, dim, nc, levels):
    from oracle.mg import MGHierarchy
    from paper_1502_04657_amd import lib
    H = MGHierarchy(dim, nc, levels)
    n = nc << (levels - 1)
    x0 = W.random_interior(dim, n, seed=9)
    f = W.random_interior(dim, n, seed=10)
    ref = H.vcycle(levels - 1, x0, f, 2, 2)
    prob = W.Problem(dim, nc, levels - 1)
    got = ops.vcycle(prob, W.Options(), dev_level(dim, n, x0), dev_level(dim, n, f))
    assert rel_err(host_compact(dim, n, got), ref) < 1e-12
    # the fused (temporally blocked) and unfused kernel sequences give identical bits
    lib().fmg_set_fused_vcycle(0)
    try:
        unf = ops.vcycle(prob, W.Options(), dev_level(dim, n, x0), dev_level(dim, n, f))
    finally:
        lib().fmg_set_fused_vcycle(1)
    assert torch.equal(got, unf)
    for nu in (0, 1):
        a = ops.vcycle(prob, W.Options(nu_pre=nu, nu_post=nu + 1), dev_level(dim, n, x0), dev_level(dim, n, f))
        lib().fmg_set_fused_vcycle(0)
        try:
            b = ops.vcycle(prob, W.Options(nu_pre=nu, nu_post=nu + 1), dev_level(dim, n, x0), dev_level(dim, n, f))
        finally:
            lib().fmg_set_fused_vcycle(1)
        assert torch.equal(a, b)
        assert rel_err(host_compact(dim, n, a), H.vcycle(levels - 1, x0, f, nu, nu + 1)) < 1e-12


@pytest.mark.parametrize("nc, levels", [(12, 8), (10, 7), (16, 8)])
def test_fused_vcycle_large_levels_bitwise(ops, nc, levels):
    """Levels above the small-tile threshold (64 x 32 tiles, ragged last tiles) give the
    same bits as the unfused kernel sequence."""
    from paper_1502_04657_amd import lib
    n = nc << (levels - 1)
    x0 = W.random_interior(2, n, seed=21)
    f = W.random_interior(2, n, seed=22)
    prob = W.Problem(2, nc, levels - 1)
    got = ops.vcycle(prob, W.Options(), dev_level(2, n, x0), dev_level(2, n, f))
    lib().fmg_set_fused_vcycle(0)
    try:
        unf = ops.vcycle(prob, W.Options(), dev_level(2, n, x0), dev_level(2, n, f))
    finally:
        lib().fmg_set_fused_vcycle(1)
    assert torch.equal(got, unf)
    assert bool(torch.isfinite(got).all())


@pytest.mark.parametrize("nc, levels", [(8, 5), (16, 4), (12, 4), (16, 2), (10, 6)])
@pytest.mark.parametrize("wide_min, bottom_max", [(64, 64), (128, -1), (512, 16), (0, 0)])
def test_fused_vcycle_2d_tuning_bitwise(ops, nc, levels, wide_min, bottom_max):
    """Every run-time choice of the 2D passes (the level from which the wide tiles are used,
    the largest level of the one-workgroup bottom, up to n = 64) gives the bits of the
    unfused kernel sequence."""
    import ctypes as C
    from paper_1502_04657_amd import _ffi, lib
    saved = _ffi.fmg_tuning()
    assert lib().fmg_get_tuning(C.byref(saved)) == 0
    t = _ffi.fmg_tuning()
    C.memmove(C.byref(t), C.byref(saved), C.sizeof(t))
    t.vpass2d_wide_min_n, t.vbottom2d_max_n = wide_min, bottom_max
    assert lib().fmg_set_tuning(C.byref(t)) == 0
    n = nc << (levels - 1)
    x0 = W.random_interior(2, n, seed=41)
    f = W.random_interior(2, n, seed=42)
    prob = W.Problem(2, nc, levels - 1)
    try:
        got = ops.vcycle(prob, W.Options(), dev_level(2, n, x0), dev_level(2, n, f))
        lib().fmg_set_fused_vcycle(0)
        unf = ops.vcycle(prob, W.Options(), dev_level(2, n, x0), dev_level(2, n, f))
    finally:
        lib().fmg_set_fused_vcycle(1)
        assert lib().fmg_set_tuning(C.byref(saved)) == 0
    assert bool(torch.isfinite(got).all())
    assert torch.equal(got, unf)


@pytest.mark.parametrize("nc, levels", [(4, 6), (6, 5), (3, 6), (5, 5), (4, 4), (4, 3), (8, 2), (2, 4)])
@pytest.mark.parametrize("nu", [1, 2])
@pytest.mark.parametrize("variant, one_pass", [(0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (1, 1), (2, 1), (3, 1)])
def test_fused_vcycle_3d_bitwise(ops, nc, levels, nu, variant, one_pass):
    """3D levels above n = 16 run the z-pipelined level passes (forced through the tuning
    interface; ragged tiles and z-chunks at n = 96, 80, 160), and levels up to n = 16 with
    everything below them the one-workgroup bottom kernel (the whole V-cycle for n = 16 on
    coarsest meshes of 2, 4 and 8 cells per side): the same bits as the unfused kernel
    sequence, for V(1,1) (one pass per side) and V(2,2) (3 + 2 half sweeps in two passes per
    side, or 5 in one), with all four tile variants."""
    import ctypes as C
    from paper_1502_04657_amd import _ffi, lib
    saved = _ffi.fmg_tuning()
    assert lib().fmg_get_tuning(C.byref(saved)) == 0
    t = _ffi.fmg_tuning()
    t.vpass3d_variant, t.vpass3d_min_n, t.vpass3d_one_pass = variant, 16, one_pass
    assert lib().fmg_set_tuning(C.byref(t)) == 0
    n = nc << (levels - 1)
    x0 = W.random_interior(3, n, seed=31)
    f = W.random_interior(3, n, seed=32)
    prob = W.Problem(3, nc, levels - 1)
    opts = W.Options(nu_pre=nu, nu_post=nu)
    try:
        got = ops.vcycle(prob, opts, dev_level(3, n, x0), dev_level(3, n, f))
        lib().fmg_set_fused_vcycle(0)
        unf = ops.vcycle(prob, opts, dev_level(3, n, x0), dev_level(3, n, f))
    finally:
        lib().fmg_set_fused_vcycle(1)
        assert lib().fmg_set_tuning(C.byref(saved)) == 0
    assert bool(torch.isfinite(got).all())
    assert torch.equal(got, unf)


@pytest.mark.parametrize("nc, levels", [(4, 6), (6, 5), (5, 5), (3, 5), (7, 3)])
@pytest.mark.parametrize("nu", [1, 2])
def test_tiled_small_levels_3d_bitwise(ops, nc, levels, nu):
    """3D levels between the one-workgroup bottom and the z-pipelined passes run the half
    sweeps of a side in LDS tiles of 8^3 nodes (3 + 2 per launch; here every level above 16,
    the z-pipelined passes being moved to n >= 4096): the same bits as the unfused kernel
    sequence, with ragged tiles at n = 96, 80, 48, 40, 28, 24, 20."""
    import ctypes as C
    from paper_1502_04657_amd import _ffi, lib
    saved = _ffi.fmg_tuning()
    assert lib().fmg_get_tuning(C.byref(saved)) == 0
    t = _ffi.fmg_tuning()
    assert lib().fmg_get_tuning(C.byref(t)) == 0
    t.vpass3d_min_n, t.vtile3d = 4096, 1
    assert lib().fmg_set_tuning(C.byref(t)) == 0
    n = nc << (levels - 1)
    x0 = W.random_interior(3, n, seed=41)
    f = W.random_interior(3, n, seed=42)
    prob = W.Problem(3, nc, levels - 1)
    opts = W.Options(nu_pre=nu, nu_post=nu)
    try:
        got = ops.vcycle(prob, opts, dev_level(3, n, x0), dev_level(3, n, f))
        lib().fmg_set_fused_vcycle(0)
        unf = ops.vcycle(prob, opts, dev_level(3, n, x0), dev_level(3, n, f))
    finally:
        lib().fmg_set_fused_vcycle(1)
        assert lib().fmg_set_tuning(C.byref(saved)) == 0
    assert bool(torch.isfinite(got).all())
    assert torch.equal(got, unf)


RHS_CASES = [W.Problem(2, 4, 2, (1.5, 0.5, 0.0), 0.25, 7.0), W.Problem(2, 12, 3, (1.0, 2.0, 0.0), 0.0, 100.0),
             W.Problem(3, 2, 2, (1.0, 0.5, 2.0), 0.3, 10.0), W.Problem(3, 3, 2, (1.0, 1.0, 1.0), 0.0, 1.0)]


@pytest.mark.parametrize("prob", RHS_CASES)
def test_rhs_and_forms(ops, prob):
    from oracle import fem
    h = oracle_hierarchy(prob)
    l = h.L - 1
    n, dim = prob.n_fine, prob.dim
    u = W.smooth_interior(dim, n, seed=11) + 0.05 * W.random_interior(dim, n, seed=12)
    lam = 23.5
    ref = h.rhs(l, lam, u)
    b = ops.rhs(prob, n, lam, dev_level(dim, n, u))
    assert rel_err(host_compact(dim, n, b), ref) < 1e-12
    kk, mw, mm, q4 = ops.forms(prob, n, dev_level(dim, n, u))
    assert kk == pytest.approx(float(u @ (h.K[l] @ u)), rel=1e-12)
    assert mw == pytest.approx(float(u @ (h.MW[l] @ u)), rel=1e-12)
    assert mm == pytest.approx(float(u @ (h.M[l] @ u)), rel=1e-12)
    assert q4 == pytest.approx(fem.integral_of(h.meshes[l], u, 4), rel=1e-12)


AUG_CASES = [W.Problem(2, 4, 3, (1.5, 0.5, 0.0), 0.25, 7.0), W.Problem(2, 8, 1, (1.0, 1.0, 0.0), 0.0, 100.0),
             W.Problem(2, 16, 2, (0.7, 1.9, 0.0), 0.0, 1000.0), W.Problem(3, 2, 2, (1.0, 0.5, 2.0), 0.3, 10.0),
             W.Problem(3, 4, 1, (1.0, 1.0, 1.0), 0.0, 1.0),
             # 3D coarsest h = 1/6: 25 x 25 blocks, arena in LDS, moments in global memory
             W.Problem(3, 6, 1, (1.0, 0.8, 1.2), 0.0, 30.0)]


def _oracle_aug(h, l, ut, x):
    from oracle import fem
    Z = sp.hstack([h.Pi[l], sp.csr_matrix(ut[:, None])]).tocsr()
    A = (Z.T @ ((h.K[l] + h.MW[l]) @ Z)).toarray()
    B = (Z.T @ (h.M[l] @ Z)).toarray()
    S = (Z.T @ (fem.density_mass(h.meshes[l], Z @ x) @ Z)).toarray()
    return A, B, S


def _unique(arr, order):
    import itertools
    V = arr.shape[-1]
    idx = list(itertools.combinations_with_replacement(range(V), order))
    return np.stack([arr[(slice(None),) + t] for t in idx], axis=-1)


@pytest.mark.parametrize("prob", AUG_CASES + [W.Problem(3, 2, 3, (0.6, 1.4, 1.1), 0.2, 5.0),
                                              W.Problem(2, 2, 5, (1.2, 0.8, 0.0), 0.1, 5.0)])
def test_moments_match_oracle_per_coarse_simplex(ops, prob):
    from oracle import fem
    h = oracle_hierarchy(prob)
    l = h.L - 1
    n, dim = prob.n_fine, prob.dim
    ut = W.smooth_interior(dim, n, seed=13) + 0.02 * W.random_interior(dim, n, seed=14)
    ref = fem.coarse_simplex_moments(h.meshes[0], h.meshes[l], ut, h.W)
    mom = ops.moments(prob, n, dev_level(dim, n, ut)).cpu().numpy()
    ne = 2 if dim == 2 else 6
    ncell = prob.n_coarse ** dim
    # library order: element = cell * ne + type; oracle order: type * ncell + cell
    perm = np.array([t * ncell + c for c in range(ncell) for t in range(ne)])
    V = dim + 1
    cols = [("T3", _unique(ref["T3"], 3)), ("T2", _unique(ref["T2"], 2)), ("T1", ref["T1"]), ("T0", ref["T0"][:, None]),
            ("B1", ref["B1"]), ("B2", ref["B2"][:, None]), ("AW1", ref["AW1"]), ("AW2", ref["AW2"][:, None]),
            ("KG", ref["KG"]), ("Q", ref["Q"][:, None])]
    off = 0
    for name, arr in cols:
        k = arr.shape[1]
        got = mom[:, off:off + k]
        want = arr[perm]
        assert rel_err(got, want) < 1e-12, name
        off += k
    assert off == mom.shape[1]


@pytest.mark.parametrize("prob, chunk", [(W.Problem(3, 2, 3, (0.6, 1.4, 1.1), 0.2, 5.0), 16),
                                         (W.Problem(3, 2, 3, (0.6, 1.4, 1.1), 0.2, 5.0), 7),
                                         (W.Problem(2, 2, 5, (1.2, 0.8, 0.0), 0.1, 5.0), 16)])
def test_moments_split_into_many_blocks(ops, prob, chunk):
    """The moment pass with the cells of every coarse simplex split into blocks of at most
    `chunk` cells (3D n = 16 over 2^3 coarse cells: 56 interior and 64 tie cells per coarse
    tetrahedron in 4 or 8 and 4 or 10 blocks, a short last tie block for chunk 7; 2D n = 64:
    496 and 32 cells in 31 and 2 blocks): the oracle's moments to 1e-12, as with the default
    blocks, and the default result to rounding."""
    from oracle import fem
    h = oracle_hierarchy(prob)
    l = h.L - 1
    n, dim = prob.n_fine, prob.dim
    ut = W.smooth_interior(dim, n, seed=15) + 0.02 * W.random_interior(dim, n, seed=16)
    ref = fem.coarse_simplex_moments(h.meshes[0], h.meshes[l], ut, h.W)
    got = ops.moments(prob, n, dev_level(dim, n, ut), chunk_cells=chunk).cpu().numpy()
    base = ops.moments(prob, n, dev_level(dim, n, ut)).cpu().numpy()
    ne = 2 if dim == 2 else 6
    ncell = prob.n_coarse ** dim
    perm = np.array([t * ncell + c for c in range(ncell) for t in range(ne)])
    cols = [("T3", _unique(ref["T3"], 3)), ("T2", _unique(ref["T2"], 2)), ("T1", ref["T1"]), ("T0", ref["T0"][:, None]),
            ("B1", ref["B1"]), ("B2", ref["B2"][:, None]), ("AW1", ref["AW1"]), ("AW2", ref["AW2"][:, None]),
            ("KG", ref["KG"]), ("Q", ref["Q"][:, None])]
    off = 0
    for name, arr in cols:
        k = arr.shape[1]
        assert rel_err(got[:, off:off + k], arr[perm]) < 1e-12, name
        assert rel_err(got[:, off:off + k], base[:, off:off + k]) < 1e-13, name
        off += k
    assert off == got.shape[1]


@pytest.mark.parametrize("prob", AUG_CASES)
@pytest.mark.parametrize("variant", ["coarse_only", "u_tilde_only", "full"])
def test_moments_build_the_augmented_matrices(ops, prob, variant):
    h = oracle_hierarchy(prob)
    l = h.L - 1
    n, dim = prob.n_fine, prob.dim
    ut = W.smooth_interior(dim, n, seed=13) + 0.02 * W.random_interior(dim, n, seed=14)
    N1 = h.Pi[l].shape[1] + 1
    x = np.random.default_rng(15).standard_normal(N1)
    if variant == "coarse_only":
        x[-1] = 0.0
    elif variant == "u_tilde_only":
        x[:-1] = 0.0
    A, B, S = _oracle_aug(h, l, ut, x)
    mom = ops.moments(prob, n, dev_level(dim, n, ut))
    Ag, Bg, Sg = (t.cpu().numpy() for t in ops.augmented_matrices(prob, mom.reshape(-1), to_dev(x)))
    assert rel_err(Ag, A) < 1e-12
    assert rel_err(Bg, B) < 1e-12
    assert rel_err(Sg, S) < 1e-12


@pytest.mark.parametrize("prob", AUG_CASES)
def test_augmented_newton_matches_oracle(ops, prob):
    from oracle import fmg as ofmg
    h = oracle_hierarchy(prob)
    l = h.L - 1
    n, dim = prob.n_fine, prob.dim
    # a realistic u~: one correction-step MG applied to the prolongated coarse ground state
    lam0, u0, _ = ofmg.coarse_step(h)
    u = h.Pi[l] @ u0
    b = h.rhs(l, lam0, u)
    ut = h.mg.mg(l, b, u, 1, 2, 2)
    mu, unew, _, xo = ofmg.augmented_solve(h, l, ut)
    mom = ops.moments(prob, n, dev_level(dim, n, ut))
    lam, c, xc, iters, ground = ops.augmented_solve(prob, W.Options(), mom.reshape(-1))
    assert ground
    assert lam == pytest.approx(mu, rel=1e-12)
    sgn = 1.0 if h.hat(l) @ unew >= 0 else -1.0
    assert c == pytest.approx(sgn * xo[-1], rel=1e-9)
    xg = host_compact(dim, prob.n_coarse, xc)
    assert rel_err(xg, sgn * xo[:-1]) < 1e-9
    # u = c u~ + Pi x_H formed on the device
    ug = ops.form_u(dim, prob.n_coarse, n, c, xc, dev_level(dim, n, ut))
    ref = sgn * unew
    assert rel_err(host_compact(dim, n, ug), ref) < 1e-9


@pytest.mark.parametrize("prob", [W.Problem(2, 8, 0, (1.0, 1.0, 0.0), 0.0, 1.0),
                                  W.Problem(2, 16, 0, (1.0, 1.0, 0.0), 0.0, 100.0),
                                  W.Problem(2, 16, 0, (0.6, 1.7, 0.0), 0.0, 1000.0),
                                  W.Problem(2, 8, 0, (0.0, 0.0, 0.0), 0.0, 0.0),
                                  W.Problem(3, 4, 0, (1.0, 1.0, 1.0), 0.0, 10.0),
                                  W.Problem(3, 8, 0, (1.0, 1.0, 1.0), 0.0, 100.0)])
def test_coarse_nonlinear_ground_state(ops, prob):
    from oracle import fmg as ofmg
    h = oracle_hierarchy(prob)
    mu, x, _ = ofmg.coarse_step(h)
    lam, xc, iters, ground = ops.coarse_nonlinear(prob, W.Options())
    assert ground
    assert lam == pytest.approx(mu, rel=1e-12)
    assert rel_err(host_compact(prob.dim, prob.n_coarse, xc), x) < 1e-9
