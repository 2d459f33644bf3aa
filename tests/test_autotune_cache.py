"""Host logic of the autotuner's JSON cache (no GPU): keys, persistence,
rejection of malformed entries, and the hit/miss paths of tune_cached with a
stand-in graph object."""
import json

import pytest

import paper_2012_10026_amd as rb
from paper_2012_10026_amd import autotune

T = {"block": 256, "per_cu": 2, "lane_row": 16, "bu_grain": 64, "td_chunk": 512, "reset": 0}


def test_scale_bucket():
    assert autotune.scale_bucket(2 ** 26) == 26
    assert autotune.scale_bucket(52_500_000) == 26  # log2 = 25.65
    assert autotune.scale_bucket(3 * 2 ** 20) == 22  # log2 = 21.58
    assert autotune.scale_bucket(1) == 1


def test_tuning_key():
    k = autotune.tuning_key("gfx950:sramecc+:xnack-", "kronecker", 2 ** 24, rb.TUNE_SINGLE)
    assert k == "gfx950/kronecker/s24/single"
    assert autotune.tuning_key("gfx950", "chung-lu", 1000, rb.TUNE_BATCH).endswith("/s10/batch")
    with pytest.raises(ValueError):
        autotune.tuning_key("gfx950", "a/b", 10, rb.TUNE_SINGLE)
    with pytest.raises(ValueError):
        autotune.tuning_key("gfx950", "x", 10, 7)


def test_cache_round_trip_and_malformed_entries(tmp_path):
    path = tmp_path / "sub" / "tuning.json"
    c = rb.TuningCache(str(path))
    assert c.get("k") is None
    c.put("k", T, ms=1.5, default_ms=2.0)
    c2 = rb.TuningCache(str(path))
    assert c2.get("k") == T
    data = json.loads(path.read_text())
    data["entries"]["bad1"] = {"tuning": {"block": 256}}
    data["entries"]["bad2"] = {"tuning": dict(T, block="256")}
    data["entries"]["bad3"] = [1, 2]
    path.write_text(json.dumps(data))
    c3 = rb.TuningCache(str(path))
    assert c3.get("k") == T
    assert c3.get("bad1") is None and c3.get("bad2") is None and c3.get("bad3") is None
    path.write_text(json.dumps({"format": 99, "entries": {"k": {"tuning": T}}}))
    assert rb.TuningCache(str(path)).get("k") is None


def test_summarize():
    d = dict(T, block=1024)
    recs = [dict(d, ms=3.0, mismatches=0), dict(T, ms=2.5, mismatches=0),
            dict(T, ms=2.0, mismatches=0)]
    assert autotune.summarize(recs, T) == (2.0, 3.0)
    assert autotune.summarize([], T) == (None, None)


class FakeGraph:
    n = 2 ** 20

    def __init__(self):
        self.tuned = 0
        self.set = []

    def tune(self, roots, kind, reps, opts):
        self.tuned += 1
        return dict(T), [dict(T, block=1024, ms=2.0, mismatches=0), dict(T, ms=1.0,
                                                                          mismatches=0)]

    def set_tuning(self, t, kind):
        self.set.append((dict(t), kind))


def test_tune_cached_miss_then_hit(tmp_path, monkeypatch):
    monkeypatch.setattr(rb, "device_info", lambda: {"arch": "gfx950:sramecc+:xnack-"})
    cache = rb.TuningCache(str(tmp_path / "t.json"))
    g = FakeGraph()
    t, recs = rb.tune_cached(g, [1, 2], cache, "kronecker")
    assert t == T and recs is not None and g.tuned == 1
    e = cache.entries["gfx950/kronecker/s20/single"]
    assert e["ms"] == 1.0 and e["default_ms"] == 2.0
    g2 = FakeGraph()
    t2, recs2 = rb.tune_cached(g2, [1, 2], rb.TuningCache(str(tmp_path / "t.json")), "kronecker")
    assert t2 == T and recs2 is None and g2.tuned == 0
    assert g2.set == [(T, rb.TUNE_SINGLE)]
    t3, recs3 = rb.tune_cached(g2, [1], cache, "kronecker", retune=True)
    assert recs3 is not None and g2.tuned == 1
