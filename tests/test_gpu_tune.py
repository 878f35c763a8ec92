"""The persisted autotuner on the GPU, through the C ABI: a cache miss times
every compiled tile shape and records the fastest under (architecture,
precision, box count, log2-cells bucket); the next call and a plan created
with the cache path take it from there without timing anything."""
import json

import numpy as np
import pytest
import torch

from gpu_helpers import to_host
from paper_2607_08743_amd import inputs as I
from paper_2607_08743_amd import z4c

pytestmark = pytest.mark.gpu


def test_autotune_miss_then_hit(tmp_path):
    print("case: autotune 32^3 punctures, cache miss then hit", flush=True)
    g, u, dt = I.config_punctures(32)
    boxes = [I.Box(g, u, None, dt)]
    path = tmp_path / "tune.jsonl"
    t1, src1 = z4c.autotune(boxes, tune_cache=str(path))
    assert src1 == "tuned"
    lines = [json.loads(x) for x in path.read_text().splitlines() if x.strip()]
    assert len(lines) == 1
    e = lines[0]
    assert e["arch"].startswith("gfx") and e["precision"] == 0 and e["nbox"] == 1 and e["bucket"] == 15
    assert e["tile"] == list(t1.as_tuple()) and e["ms"] > 0
    t2, src2 = z4c.autotune(boxes, tune_cache=str(path))
    assert src2 == "cache" and t2.as_tuple() == t1.as_tuple()
    # a plan created with the cache path launches the cached shape and steps
    # like a plan given that tile explicitly
    p_cache = z4c.Plan(boxes, tune_cache=str(path))
    tile, src = p_cache.tile()
    assert src == "cache" and tile.as_tuple() == t1.as_tuple()
    p_cache.step(1)
    p_tile = z4c.Plan(boxes, tile=t1)
    p_tile.step(1)
    assert np.array_equal(to_host(p_cache.u[0]), to_host(p_tile.u[0]))
    p_cache.close()
    p_tile.close()
    # another precision is another key: a miss, recorded beside the first entry
    _, src3 = z4c.autotune(boxes, params=z4c.default_params(precision=z4c.MIXED), tune_cache=str(path))
    assert src3 == "tuned"
    assert len([x for x in path.read_text().splitlines() if x.strip()]) == 2
    torch.cuda.empty_cache()


def test_plan_default_on_key_miss(tmp_path):
    print("case: plan with a cache that holds another bucket", flush=True)
    g, u, dt = I.config_punctures(16)
    path = tmp_path / "tune.jsonl"
    path.write_text(json.dumps({"arch": "gfx950", "precision": 0, "nbox": 1, "bucket": 30,
                                "tile": [16, 4, 4, 1, 0], "ms": 1.0}) + "\n")
    p = z4c.Plan([I.Box(g, u, None, dt)], tune_cache=str(path))
    tile, src = p.tile()
    assert src == "default" and tile.as_tuple() == (8, 8, 8, 2, 1)
    p.close()


def test_tile_resources_of_the_benchmark_shapes():
    """z4c_tile_resources reports what the compiler built: the 8x8x8 two-wave
    shapes hold two waves per SIMD (one 512-thread block per compute unit);
    the FP64 form spills a few registers, the mixed form none."""
    print("case: tile resources 8x8x8x2 FP64 and mixed", flush=True)
    t = z4c.Tile(8, 8, 8, 2, 1)
    r64 = z4c.tile_resources(z4c.FP64, t)
    rmx = z4c.tile_resources(z4c.MIXED, t)
    print(r64, rmx)
    assert r64["waves_per_simd"] == 2 and rmx["waves_per_simd"] == 2
    assert 0 < r64["lds_bytes"] <= 163840 and 0 < rmx["lds_bytes"] <= 163840
    assert r64["scratch_bytes_per_lane"] > 0 and rmx["scratch_bytes_per_lane"] == 0
