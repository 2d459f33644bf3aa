"""Host-side helpers of bench.py (no GPU): the algorithmic-bytes model of
the search kernel, the harmonic-mean TEPS, the workload check on the stored
traffic figure, the refusal of more than one GPU, and that the learned
switch is measured on graphs it was neither trained nor validated on, and
that the committed traffic profile belongs to the committed kernel sources."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_alg_bytes_hand_computed(bench):
    # three levels on 100 swept vertices: TD from the root (nf 1, 5 edges),
    # BU (nf 4, 40 entries read), TD (nf 20, 30 edges), nothing after
    st = {"levels": 3, "nf": [1, 4, 20], "dir": [0, 1, 0], "edges": [5, 40, 30],
          "reached": 25}
    td0 = 16 * 1 + 4 * 1 + 4 * 5 + 12 * 4
    bu1 = 8 * (100 - 1 - 4) + 4 * 40 + 3 * ((100 + 7) // 8) + 8 * 20
    td2 = 16 * 20 + 4 * 20 + 4 * 30 + 12 * 0
    assert bench.bfs_alg_bytes(st, 100, original_ids=False) == td0 + bu1 + td2
    assert bench.bfs_alg_bytes(st, 100, original_ids=True) == td0 + bu1 + td2 + 4 * 25


def test_hmean_gteps(bench):
    # 1e9 edges in 1 ms and 2e9 edges in 1 ms: 1000 and 2000 GTEPS
    h = bench.hmean_gteps([1e9, 2e9], [1.0, 1.0])
    assert h == pytest.approx(2 / (1 / 1000 + 1 / 2000))


def test_traffic_only_for_the_profiled_workload(bench):
    assert bench.measured_traffic("kronecker scale 27 seed 1027, 64 roots, alpha 14 beta 24") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_switch_graphs_are_held_out(bench):
    """The learned switch trains on Kronecker scales 18-24 and on Chung-Lu
    graphs, picks its network on other graphs, and is measured on graphs of
    neither set: the Kronecker scale-26 graph (seed 1026), the 52.5M-vertex
    Chung-Lu graph (seed 4000) and the heavy-tailed 300000-vertex graph
    (seed 9)."""
    key = lambda spec: (spec[0].split("-52.5M")[0], spec[1], spec[2])
    train = {key(s) for s in bench.SWITCH_TRAIN_GRAPHS}
    valid = {key(s) for s in bench.SWITCH_VALIDATION_GRAPHS}
    measured = {("kronecker", 26, 1026), ("chung-lu", 50_000_000, 4000),
                ("chung-lu", 300_000, 9)}
    assert len(train) == len(bench.SWITCH_TRAIN_GRAPHS)
    assert not train & valid and not train & measured and not valid & measured
    assert all(18 <= s[1] <= 24 for s in bench.SWITCH_TRAIN_GRAPHS if s[0] == "kronecker")


def test_committed_traffic_profile_matches_the_sources(bench):
    """The committed traffic figure of the search kernel was taken from the
    committed kernel sources (their digest matches), so bench.py reports it."""
    import json
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_bfs_persistent_kernel.json")))
    assert bench.measured_traffic(rec["workload"]) == rec["traffic_bytes_per_launch"]
