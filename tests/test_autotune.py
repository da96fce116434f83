"""The schedule autotuner's host logic (no GPU): batch signatures and the
cache path that skips measurement."""
import json

from paper_1902_10078_amd import autotune


def test_shape_key_groups_similar_batches():
    a = autotune.shape_key([1000, 2000], [3, 5], "op", 0)
    b = autotune.shape_key([1010, 1995], [5, 3], "op", 0)
    assert a == b
    assert a != autotune.shape_key([1000, 2000], [3, 5], "op", 1)
    assert a != autotune.shape_key([1000, 2000, 5], [3, 5, 5], "op", 0)
    assert a != autotune.shape_key([1000, 2000], [3, 5], "other", 0)
    gfx = autotune.shape_key([1000, 2000], [3, 5], "op", 0, arch="gfx950")
    assert gfx.startswith("gfx950|") and gfx != autotune.shape_key([1000, 2000], [3, 5], "op", 0, arch="gfx942")


def test_cached_result_is_used_without_measuring(tmp_path):
    ns, ks = [5000, 7000], [5, 5]
    key = autotune.shape_key(ns, ks, "matern52_loss", 0)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({key: {"target_chunks": 32768, "ms": {"32768": 1.0}}}))

    def make_step(t):
        raise AssertionError("no measurement expected")

    res = autotune.tune(ns, ks, make_step, "matern52_loss", 0, cache_path=str(path))
    assert res["target_chunks"] == 32768 and res["cached"]
