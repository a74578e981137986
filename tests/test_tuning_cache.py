"""The tuning cache (paper_1502_04657_amd.tuning): a stored choice is applied without
timing, a missing one is measured and stored (GPU), and a choice applied through the cache
changes no bit of a V-cycle (GPU)."""
import json

import pytest

import workloads as W


def test_cached_choice_is_applied_without_timing(tmp_path, monkeypatch):
    from paper_1502_04657_amd import _ffi, tuning
    calls = []
    monkeypatch.setattr(tuning, "_key", lambda dim, n, p: f"dev|dim={dim}|n={n}|{p}")
    monkeypatch.setattr(tuning, "apply", lambda c: calls.append(("apply", c)))
    lib = _ffi.load()
    monkeypatch.setattr(lib, "fmg_autotune_vcycle", lambda *a: calls.append(("tune",)) or -1, raising=False)
    cache = tmp_path / "t.json"
    cache.write_text(json.dumps({"dev|dim=3|n=256|fp64": {"vpass3d_variant": 2, "vpass3d_min_n": 64}}))
    got = tuning.autotune(3, 256, "fp64", cache=str(cache))
    assert got == {"vpass3d_variant": 2, "vpass3d_min_n": 64}
    assert calls == [("apply", got)]


@pytest.mark.gpu
def test_autotune_2d_returns_valid_choices():
    pytest.importorskip("torch")
    from paper_1502_04657_amd import tuning
    saved = tuning.get()
    try:
        for prec in ("fp64", "mixed"):
            c = tuning.autotune(2, 256, prec, cache=None, apply_result=False)
            assert 64 <= c["vpass2d_wide_min_n"] <= 256 and c["vbottom2d_max_n"] in (-1, 16, 32, 64)
            assert tuning.get() == saved       # the autotuner leaves the tuning as it was
    finally:
        tuning.apply(saved)


@pytest.mark.gpu
def test_autotune_stores_and_keeps_bits(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_1502_04657_amd import ops, tuning
    saved = tuning.get()
    cache = tmp_path / "t.json"
    try:
        choice = tuning.autotune(3, 64, "fp64", cache=str(cache))
        assert choice["vpass3d_variant"] in (0, 1, 2) and choice["vpass3d_min_n"] >= 16
        assert json.loads(cache.read_text())          # stored
        assert tuning.autotune(3, 64, "fp64", cache=str(cache)) == choice   # served from the cache
        prob = W.Problem(3, 4, 4)
        x0 = ops.pack(3, 64, torch.from_numpy(W.random_interior(3, 64, seed=5)).cuda())
        f = ops.pack(3, 64, torch.from_numpy(W.random_interior(3, 64, seed=6)).cuda())
        got = ops.vcycle(prob, W.Options(), x0.clone(), f)
        tuning.apply({"vpass3d_variant": 0, "vpass3d_min_n": 4096})   # no fused level
        ref = ops.vcycle(prob, W.Options(), x0.clone(), f)
        assert torch.equal(got, ref)
    finally:
        tuning.apply(saved)
