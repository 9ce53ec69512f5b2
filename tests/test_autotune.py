"""Host logic of the launch-shape autotuner (no GPU): the JSON cache and the
choice rule."""
import json

from paper_2601_16911_amd import autotune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    autotune.store("gfx950|mesh|deg3", {"grid": 8192, "ms": 0.4}, path)
    autotune.store("gfx950|batch|abc", {"grid": 1024, "ms": 2.7}, path)
    data = autotune.load_cache(path)
    assert data["gfx950|mesh|deg3"]["grid"] == 8192
    assert data["gfx950|batch|abc"]["grid"] == 1024
    with open(path) as f:
        assert json.load(f) == data


def test_corrupt_cache_reads_as_empty(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert autotune.load_cache(str(path)) == {}


def test_pick_fastest_first_on_ties():
    assert autotune.pick({1024: 0.5, 2048: 0.4, 4096: 0.4}) == 2048
    assert autotune.pick({0: 1.0}) == 0
