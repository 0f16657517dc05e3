"""Autotuner bookkeeping without a GPU: resolution classes and the cache."""
import json

from paper_2106_08034_amd import autotune


def test_resolution_classes():
    assert autotune.resolution_class(640 * 480) == "<=0.5M"
    assert autotune.resolution_class(1280 * 720) == "<=1.5M"
    assert autotune.resolution_class(1920 * 1080) == "<=4M"
    assert autotune.resolution_class(2560 * 1440) == "<=4M"
    assert autotune.resolution_class(3840 * 2160) == ">4M"


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = autotune.TuneCache(path)
    k = autotune.TuneCache.key("devX", "stream", 8, "f32", 1920 * 1080)
    assert c.get(k) is None
    c.put(k, {"best": [7, 256, 0], "ms": {"128x2/256": 0.23}})
    again = autotune.TuneCache(path)
    assert again.get(k)["best"] == [7, 256, 0]
    assert json.load(open(path))[k]["ms"]["128x2/256"] == 0.23
    # a corrupt file is ignored, not fatal
    open(path, "w").write("{not json")
    assert autotune.TuneCache(path).get(k) is None


def test_candidates_are_valid_launch_shapes():
    for tw, bt in autotune.TILE_CANDIDATES:
        assert bt in (64, 128, 256) and (1 << tw) <= bt
