"""Autotuner cache logic (CPU) and one tuning pass (GPU)."""
import os

import pytest

dg = pytest.importorskip("paper_1211_0582_amd.dg", reason="libdg.so not built")
from paper_1211_0582_amd import autotune  # noqa: E402


def test_cache_record_lookup_roundtrip(tmp_path):
    path = str(tmp_path / "cache.json")
    cache = autotune.load(path)
    assert cache == {}
    best = autotune.record(cache, "gfx950", "fp32", 4, {"valu": 0.21, "mfma": 0.12})
    assert best == "mfma"
    autotune.record(cache, "gfx950", "fp64", 9, {"valu": 1.0})
    autotune.save(cache, path)
    assert autotune.lookup(4, "fp32", arch="gfx950", path=path) == "mfma"
    assert autotune.lookup(4, dg.DG_FP32, arch="gfx950", path=path) == "mfma"
    assert autotune.lookup(9, "fp64", arch="gfx950", path=path) == "valu"
    assert autotune.lookup(5, "fp32", arch="gfx950", path=path) is None
    assert autotune.lookup(4, "fp32", arch="gfx942", path=path) is None


@pytest.mark.gpu
def test_tuning_pass_picks_a_built_variant(tmp_path):
    import dg_inputs as I
    path = str(tmp_path / "cache.json")
    cache = autotune.tune([2, 4], ["fp32"], dofs=2e5, reps=5, path=path, verbose=True)
    arch = next(iter(cache))
    for N in (2, 4):
        entry = cache[arch]["fp32"][str(N)]
        assert entry["variant"] in entry["ms"] and all(t > 0 for t in entry["ms"].values())
    os.environ["DG_AUTOTUNE_CACHE"] = path
    try:
        VX, EToV = I.kuhn_cube(2, 0.1, 0)
        p = dg.Problem(4, VX, EToV, "fp32", tuned=True)
        assert p.variant == cache[arch]["fp32"]["4"]["variant"]
        p.close()
    finally:
        del os.environ["DG_AUTOTUNE_CACHE"]
