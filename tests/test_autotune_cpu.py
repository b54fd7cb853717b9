"""Host logic of the tile autotuner and the tile-setting call (no GPU)."""
import pytest

from paper_2005_12764_amd import autotune as T
from paper_2005_12764_amd import lb
from paper_2005_12764_amd import workloads as W


def test_pick_takes_the_fastest_runnable_candidate():
    times = {(4, 0): 2.0, (8, 0): None, (8, 16): 1.5, (2, 32): 1.7}
    best, res = T.pick(lambda ty, tz: times[(ty, tz)], list(times))
    assert best == (8, 16, 1.5)
    assert [r["ms"] for r in res] == [2.0, None, 1.5, 1.7]
    with pytest.raises(RuntimeError):
        T.pick(lambda ty, tz: None, [(4, 0)])


def test_box_classes_and_keys():
    assert T.box_class(32 ** 3) == "small"
    assert T.box_class(128 ** 3) == "medium"
    assert T.box_class(256 ** 3) == "large"
    assert T.cache_key("gfx950", W.F16, lb.TILES_BATCH, "small") == "gfx950/f16/batch/small"


def test_cache_roundtrip_and_apply(tmp_path):
    cache = {T.cache_key("gfx950", W.F32, lb.TILES_ONE_READ, "large"): {"ty": 4, "tz": 32, "ms": 1.0}}
    path = str(tmp_path / "tiles.json")
    T.save(cache, path)
    assert T.load(path) == cache
    assert T.load(str(tmp_path / "missing.json")) == {}
    try:
        done = T.apply(T.load(path), "gfx950", W.F32, 256 ** 3)
        assert done == {lb.TILES_ONE_READ: (4, 32)}
        assert T.apply(cache, "gfx950", W.F32, 32 ** 3) == {}
    finally:
        lb.lb_set_tiles(lb.TILES_ONE_READ, W.F32, 0, 0)


def test_set_tiles_validates_its_arguments():
    lb.lb_set_tiles(lb.TILES_COLLIDE, W.F32, 8, 32)
    lb.lb_set_tiles(lb.TILES_COLLIDE, W.F32, 0, 0)
    for args in [(4, W.F32, 4, 0), (lb.TILES_COLLIDE, 7, 4, 0), (lb.TILES_COLLIDE, W.F32, 3, 0),
                 (lb.TILES_ONE_READ, W.F32, 2, 0), (lb.TILES_ONE_READ, W.F32, 1, 0), (lb.TILES_BATCH, W.F16, 16, 0),
                 (lb.TILES_PHASE, W.F16, 8, -1), (lb.TILES_PHASE, W.F16, 8, 5000)]:
        with pytest.raises(lb.LbError):
            lb.lb_set_tiles(*args)
