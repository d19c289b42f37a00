"""Host logic of the heterogeneous crossbar batches (no GPU): how a class's
configuration is resolved from the tuning cache, the committed cache's validity,
and the C ABI's host-side argument checks."""
import ctypes
import json
import os

import pytest

from paper_2410_19993_amd import _lib
from paper_2410_19993_amd import tiles as tl


def test_resolve_takes_valid_cache_entries_and_defaults_otherwise():
    cache = {"devices": {"GPU A": {"streams": 6, "classes": {
        "32x32x256": {"method": "one_wg", "block": 64, "split": 2},
        "32x128x256": {"method": "one_wg", "block": 64, "split": 1},      # n > 64 untransposed: invalid
        "64x64x256": {"method": "pipeline", "block": 0, "split": 1}}}}}
    classes = [(32, 32, 5, 256), (32, 128, 5, 256), (64, 64, 5, 256), (64, 64, 5, 128)]
    cfgs, streams, src = tl.resolve(classes, cache, "GPU A")
    assert streams == 6
    assert cfgs[0] == tl.TileConfig("one_wg", 64, 2) and src[0] == "cache"
    assert cfgs[1] == tl.default_config(32, 128) and src[1] == "default"
    assert cfgs[2] == tl.TileConfig("pipeline") and src[2] == "cache"
    assert cfgs[3] == tl.default_config(64, 64) and src[3] == "default"       # other B
    cfgs, streams, src = tl.resolve(classes, cache, "GPU B")                   # other device
    assert streams == tl.DEFAULT_STREAMS and src == ["default"] * 4


def test_config_validity():
    assert tl.TileConfig("one_wg", 0, 1).valid_for(8, 64)
    assert not tl.TileConfig("one_wg", 32, 1).valid_for(8, 40)
    assert not tl.TileConfig("one_wg", 0, 5).valid_for(8, 8)
    assert not tl.TileConfig("one_wg", 0, 1).valid_for(8, 65)
    assert tl.TileConfig("pipeline").valid_for(8, 512) and not tl.TileConfig("pipeline").valid_for(8, 513)
    # transposed: the reciprocal problem has m columns and n unit inputs
    assert tl.TileConfig("one_wg", 32, 1, True).valid_for(32, 256)
    assert not tl.TileConfig("one_wg", 0, 1, True).valid_for(128, 256)
    assert tl.TileConfig("pipeline", 0, 1, True).valid_for(128, 256)
    assert not tl.TileConfig("pipeline", 0, 1, True).valid_for(32, 300)      # 300 unit inputs
    assert all(c.valid_for(20, 48) for c in tl.candidates(20, 48))
    assert tl.candidates(200, 200) == [tl.TileConfig("pipeline")]
    assert tl.TileConfig("pipeline", 0, 1, True) in tl.candidates(128, 256)
    assert tl.default_config(32, 256).transpose and tl.default_config(128, 256).method == "pipeline"
    assert not tl.default_config(256, 128).transpose


def test_committed_cache_is_valid():
    if not os.path.exists(tl.CACHE_PATH):
        pytest.skip("no tuning cache committed yet")
    cache = json.load(open(tl.CACHE_PATH))
    assert cache.get("format") == 1 and cache.get("devices")
    for dev, entry in cache["devices"].items():
        assert 1 <= int(entry["streams"]) <= 8
        for key, rec in entry["classes"].items():
            m, n, B = (int(x) for x in key.split("x"))
            cfg = tl.TileConfig(rec["method"], int(rec["block"]), int(rec["split"]), bool(rec.get("transpose")))
            assert cfg.valid_for(m, n, B), (dev, key, rec)
            assert rec["ms"] == min(rec["candidates"].values())


def test_tiles_create_rejects_bad_arguments():
    L = _lib.lib()
    out = ctypes.c_void_p()
    good = dict(m=8, n=8, count=2, B=16, method=0, block=0, split=1, transpose=0)
    bad = [dict(good, m=0), dict(good, count=0), dict(good, B=257), dict(good, method=2),
           dict(good, n=65), dict(good, split=5), dict(good, block=8), dict(good, block=32, n=40),
           dict(good, method=1, n=513), dict(good, transpose=2),
           dict(good, transpose=1, m=65, n=100),               # reciprocal one-wg: m columns > 64
           dict(good, transpose=1, method=1, m=8, n=300)]      # 300 unit inputs
    for b in bad:
        arr = (_lib.TileClass * 1)(_lib.TileClass(**b))
        assert L.xbar_tiles_create(arr, 1, 1.0, 1.0, 50.0, 50.0, 2, None, ctypes.byref(out)) == _lib.XBAR_ERR_ARG, b
    arr = (_lib.TileClass * 1)(_lib.TileClass(**good))
    assert L.xbar_tiles_create(arr, 1, 0.0, 1.0, 50.0, 50.0, 2, None, ctypes.byref(out)) == _lib.XBAR_ERR_ARG
    assert L.xbar_tiles_create(arr, 1, 1.0, 1.0, 50.0, 50.0, 9, None, ctypes.byref(out)) == _lib.XBAR_ERR_ARG
    assert L.xbar_tiles_create(arr, 0, 1.0, 1.0, 50.0, 50.0, 2, None, ctypes.byref(out)) == _lib.XBAR_ERR_ARG
    assert L.xbar_tiles_run(None, None, None, None) == _lib.XBAR_ERR_ARG
    assert L.xbar_tiles_destroy(None) == _lib.XBAR_OK
