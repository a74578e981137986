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
    sizes = {(p.n_coarse, p.n_coarse << p.n_refine) for p in three}
    assert sizes == {(8, 64), (8, 128), (6, 192)}
    for p in reqs:
        assert 0.1 <= p.zeta <= 1000.0
        assert all(0.5 <= a <= 2.0 for a in p.w_quad[: p.dim])
        assert math.log2(p.n_coarse << p.n_refine) > 0
