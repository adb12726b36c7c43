"""Autotuner cache logic (CPU) and one tuning pass (GPU)."""
import os

import pytest

dg = pytest.importorskip("paper_1211_0582_amd.dg", reason="libdg.so not built")
from paper_1211_0582_amd import autotune  # noqa: E402


def test_cache_record_lookup_roundtrip(tmp_path):
    path = str(tmp_path / "cache.json")
    cache = autotune.load(path)
    assert cache == {}
    best = autotune.record(cache, "gfx950", "fp32", 4, "large", 82944, {"valu": 0.21, "mfma": 0.12, "mfma_waves": 0.15},
                           {"valu": 0.05, "mfma": 0.03})
    assert best == "mfma"
    autotune.record(cache, "gfx950", "fp32", 4, "small", 384, {"valu": 0.01, "mfma": 0.02}, {})
    autotune.record(cache, "gfx950", "fp64", 9, "large", 48000, {"valu": 1.0}, {})
    autotune.save(cache, path)
    assert autotune.lookup(4, "fp32", 82944, arch="gfx950", path=path) == "mfma"
    assert autotune.lookup(4, dg.DG_FP32, 1000, arch="gfx950", path=path) == "valu"
    assert autotune.lookup(9, "fp64", 10, arch="gfx950", path=path) == "valu"     # falls back to the other bucket
    assert autotune.lookup(5, "fp32", 1000, arch="gfx950", path=path) is None
    assert autotune.lookup(4, "fp32", 1000, arch="gfx942", path=path) is None
    assert autotune.bucket(19999) == "small" and autotune.bucket(20000) == "large"


def test_committed_table_covers_every_order_and_has_a_spread():
    """The gfx950 table committed with the library: an entry per order and
    tuned precision in both buckets, the recorded winner among the timed
    variants, and more than one variant timed where several are built."""
    cache = autotune.load()
    table = cache.get("gfx950", {})
    for prec in ("fp64", "fp32", "f16x3", "bf16x3"):
        for N in range(1, 10):
            if prec == "fp64" and N == 9:
                pass
            entry = table.get(prec, {}).get(str(N), {})
            for b in ("small", "large"):
                assert b in entry, (prec, N, b)
                e = entry[b]
                assert e["variant"] == min(e["step_ms"], key=e["step_ms"].get)
                assert all(t > 0 for t in e["step_ms"].values())
    multi = [len(table[p][str(N)]["large"]["step_ms"]) for p in ("fp64", "fp32") for N in range(2, 8)]
    assert min(multi) >= 3


@pytest.mark.gpu
def test_tuning_pass_picks_a_built_variant(tmp_path):
    import dg_inputs as I
    path = str(tmp_path / "cache.json")
    cache = autotune.tune([2, 4], ["fp32"], buckets=("small",), reps=2, path=path, verbose=True, sizes={"small": 3})
    arch = next(iter(cache))
    for N in (2, 4):
        entry = cache[arch]["fp32"][str(N)]["small"]
        assert entry["variant"] in entry["step_ms"] and all(t > 0 for t in entry["step_ms"].values())
        assert len(entry["step_ms"]) >= 2
    os.environ["DG_AUTOTUNE_CACHE"] = path
    try:
        VX, EToV = I.kuhn_cube(2, 0.1, 0)
        p = dg.Problem(4, VX, EToV, "fp32", tuned=True)
        assert p.variant == cache[arch]["fp32"]["4"]["small"]["variant"]
        p.close()
    finally:
        del os.environ["DG_AUTOTUNE_CACHE"]
