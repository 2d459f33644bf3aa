"""Persistent cache of autotuned search parameters.

The library's autotuner (``rbfs_tune`` / ``rbfs_multi_tune``) times launch
shapes and work splits on sample roots and keeps the fastest setting whose
outputs equal the defaults' bit for bit.  Tuning a large graph takes seconds,
so winners are stored in a JSON file keyed by device architecture, graph
class (the caller's name for the generator or data family), scale bucket
(nearest log2 of the vertex count) and search kind, and reused for graphs that
fall under the same key.
"""
import json
import math
import os
import tempfile

from . import TUNE_BATCH, TUNE_SINGLE, TUNING_FIELDS

KIND_NAMES = {TUNE_SINGLE: "single", TUNE_BATCH: "batch"}
FORMAT = 1


def scale_bucket(n):
    """Nearest integer log2 of the vertex count (at least 1)."""
    return max(1, int(round(math.log2(max(2, int(n))))))


def tuning_key(arch, graph_class, n, kind):
    """Cache key, e.g. 'gfx950/kronecker/s26/single'.  Feature suffixes of
    the architecture name (':sramecc+:xnack-') are dropped."""
    if kind not in KIND_NAMES:
        raise ValueError("unknown tuning kind %r" % (kind,))
    if not graph_class or "/" in graph_class:
        raise ValueError("graph class must be a non-empty name without '/'")
    return "%s/%s/s%d/%s" % (arch.split(":")[0], graph_class, scale_bucket(n), KIND_NAMES[kind])


def _valid_tuning(t):
    return (isinstance(t, dict) and set(t) == set(TUNING_FIELDS) and
            all(isinstance(t[f], int) for f in TUNING_FIELDS))


class TuningCache:
    """JSON file of {key: {"tuning": {...}, "ms": float, "default_ms": float}}.

    A missing file is an empty cache.  Entries that do not have the expected
    fields are ignored.  Writes replace the file atomically."""

    def __init__(self, path):
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            if isinstance(data, dict) and data.get("format") == FORMAT:
                for k, v in data.get("entries", {}).items():
                    if isinstance(v, dict) and _valid_tuning(v.get("tuning")):
                        self.entries[k] = v

    def get(self, key):
        e = self.entries.get(key)
        return dict(e["tuning"]) if e else None

    def put(self, key, tuning, ms=None, default_ms=None):
        tuning = {f: int(tuning[f]) for f in TUNING_FIELDS}
        self.entries[key] = {"tuning": tuning, "ms": ms, "default_ms": default_ms}
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuning-", suffix=".json")
        with os.fdopen(fd, "w") as f:
            json.dump({"format": FORMAT, "entries": self.entries}, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def summarize(records, best):
    """(best ms, default ms) from the tuner's records: the default is the
    first candidate timed; the best is the fastest record equal to `best`."""
    if not records:
        return None, None
    default_ms = records[0]["ms"]
    same = [r["ms"] for r in records if all(r[f] == best[f] for f in TUNING_FIELDS)]
    return (min(same) if same else None), default_ms


def target_size(target):
    """Vertex count that picks the scale bucket: the graph's, or the sum
    over the graphs of a multi-graph batch."""
    return sum(g.n for g in target.graphs) if hasattr(target, "graphs") else target.n


def tune_cached(target, roots, cache, graph_class, kind=TUNE_SINGLE, reps=2, opts=None,
                retune=False):
    """Sets the cached tuning of (device, graph class, scale, kind) on the
    target (a Graph, or a MultiGraph with kind TUNE_BATCH), or tunes it on
    `roots` and stores the winner.  Returns (tuning dict, records or None
    when it came from the cache)."""
    from . import device_info
    multi = hasattr(target, "graphs")
    if multi and kind != TUNE_BATCH:
        raise ValueError("a multi-graph batch is tuned with kind TUNE_BATCH")
    key = tuning_key(device_info()["arch"], graph_class, target_size(target), kind)
    hit = None if retune else cache.get(key)
    if hit is not None:
        if multi:
            target.set_tuning(hit)
        else:
            target.set_tuning(hit, kind)
        return hit, None
    if multi:
        best, records = target.tune(roots, reps=reps)
    else:
        best, records = target.tune(roots, kind=kind, reps=reps, opts=opts)
    best_ms, default_ms = summarize(records, best)
    cache.put(key, best, best_ms, default_ms)
    return best, records
