"""The seeded workload generators produce the shapes the batched and serving workloads
specify (sizes, coarsest meshes, parameter ranges); they hold no arithmetic of the method."""
import math

import workloads as W


def test_batch_instances():
    probs = W.batch_instances(64, 0)
    assert len(probs) == 64
    assert {p.n_coarse << p.n_refine for p in probs} <= {256, 512, 1024}
    for p in probs:
        assert p.dim == 2 and p.n_coarse == 16
        assert 0.1 <= p.zeta <= 1000.0
        assert all(0.5 <= a <= 2.0 for a in p.w_quad[:2]) and p.w_quad[2] == 0.0
    assert W.batch_instances(64, 0) == probs   # seeded


def test_serving_requests():
    reqs = W.serving_requests(400, 1)
    two = [p for p in reqs if p.dim == 2]
    three = [p for p in reqs if p.dim == 3]
    assert 0.6 < len(two) / len(reqs) < 0.8
    assert {p.n_coarse << p.n_refine for p in two} == {128, 256, 512, 1024, 2048}
    assert all(p.n_coarse == 16 for p in two)
    assert {p.n_coarse << p.n_refine for p in three} == {64, 128, 192}
    for p in three:
        # the coarsest mesh follows the zeta rule: nested, 4 <= n_c <= 16, and the smallest
        # admissible one with zeta H^2 <= ZETA_H2_MAX when one exists
        n = p.n_coarse << p.n_refine
        cands = [c for c in range(4, 17) if n % c == 0 and ((n // c) & (n // c - 1)) == 0 and n // c >= 2]
        ok = [c for c in cands if p.zeta / c ** 2 <= W.ZETA_H2_MAX]
        assert p.n_coarse == (ok[0] if ok else cands[-1])
    assert W.coarse_cells_3d(192, 10.0) == 6 and W.coarse_cells_3d(192, 300.0) == 12
    assert W.coarse_cells_3d(64, 10.0) == 4 and W.coarse_cells_3d(128, 150.0) == 8
    assert W.coarse_cells_3d(64, 1000.0) == 16
    for p in reqs:
        assert 0.1 <= p.zeta <= 1000.0
        assert all(0.5 <= a <= 2.0 for a in p.w_quad[: p.dim])
        assert math.log2(p.n_coarse << p.n_refine) > 0
