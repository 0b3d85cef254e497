"""Host logic of the autotuner: cache keys and the JSON cache (no GPU)."""
import json

import numpy as np

from paper_1609_09685_amd import autotune


def test_geometry_key_classes():
    k = autotune.geometry_key(9, "fp32", (1, 200, 400), 59200)
    assert k == "D9:fp32:400x200x1:phi0.7"
    # porosity classes of width 0.1; shape and precision separate classes
    assert autotune.geometry_key(9, "fp32", (1, 200, 400), 60000) == "D9:fp32:400x200x1:phi0.8"
    assert autotune.geometry_key(9, "fp64", (1, 200, 400), 59200) != k
    assert autotune.geometry_key(19, "fp32", (2, 200, 400), 118400) != k


def test_cache_hit_needs_no_device(tmp_path, monkeypatch):
    path = tmp_path / "t.json"
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(path))
    mask = np.zeros((20, 64), np.uint8)
    mask[:, :5] = 1
    key = autotune.geometry_key(9, "fp32", (1, 20, 64), int((mask == 0).sum()))
    entry = {"band": 8, "xcd_remap": 1, "ms_per_step": 0.01, "timings": {"8,1": 0.01}}
    path.write_text(json.dumps({key: entry}))
    assert autotune.tune(mask, precision="fp32") == entry


def test_cache_store_roundtrip(tmp_path):
    p = tmp_path / "sub" / "c.json"
    autotune._store(str(p), {"a": {"band": 4}})
    assert autotune._load(str(p)) == {"a": {"band": 4}}
    p.write_text("not json")
    assert autotune._load(str(p)) == {}
