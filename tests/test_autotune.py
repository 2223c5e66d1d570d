"""Autotuner host logic (CPU): shape classes and the JSON cache."""

import json

import paper_2412_06359_amd as cm
from paper_2412_06359_amd import autotune


def _descs(n, W=346, H=260, refs=(0.0, 1.0), mode=0):
    return [cm.WindowDesc.make(W, H, 200.0, 200.0, (W - 1) / 2, (H - 1) / 2, list(refs), mode)
            for _ in range(n)]


def test_shape_class_buckets():
    a = autotune.shape_class(_descs(64), [40000] * 64)
    b = autotune.shape_class(_descs(60), [41000] * 60)
    assert a == b                                   # same power-of-two buckets
    assert a != autotune.shape_class(_descs(64, refs=(0.0, 0.5, 1.0)), [40000] * 64)
    assert a != autotune.shape_class(_descs(64, W=640, H=480), [40000] * 64)
    assert a != autotune.shape_class(_descs(64, mode=1), [40000] * 64)
    assert "R2" in a and "F1" in a and "nw64" in a


def test_cache_roundtrip_and_hit(tmp_path):
    path = str(tmp_path / "tune.json")
    descs, counts = _descs(8), [1000] * 8
    key = autotune.shape_class(descs, counts)
    autotune.save_cache(path, {key: dict(event_blocks=2048, tile_threads=256, ms=1.0)})
    assert json.load(open(path))[key]["event_blocks"] == 2048
    # a cache hit needs no inputs and no GPU
    assert autotune.tune(descs, counts, cache_path=path) == dict(event_blocks=2048,
                                                                tile_threads=256, tile_w=32,
                                                                tile_h=32)
    autotune.save_cache(path, {key: dict(event_blocks=2048, tile_threads=256, tile_w=64,
                                         tile_h=32, ms=1.0)})
    assert autotune.tune(descs, counts, cache_path=path)["tile_w"] == 64
    # a miss without inputs gives the defaults
    assert autotune.tune(_descs(3), [5] * 3, cache_path=path) == autotune.DEFAULT
    # the deterministic mode is not tuned
    assert autotune.tune(_descs(8, mode=1), counts, cache_path=path) == autotune.DEFAULT


def test_candidates_are_valid_tunings():
    for c in autotune.CANDIDATES:
        assert 256 <= c["event_blocks"] <= 65536 and c["tile_threads"] in (256, 512)
        assert (c["tile_w"], c["tile_h"]) == (32, 32)
    assert autotune.DEFAULT in autotune.CANDIDATES
    assert set(autotune.TILE_SIZES) == {(32, 32), (64, 32), (32, 16), (16, 16)}
