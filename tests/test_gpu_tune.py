"""GPU tests of the tunable search parameters and the autotuner: every
setting the tuner may pick (and the extremes of the documented ranges) must
give exactly the oracle's depth and parent arrays; the tuner itself must
time only candidates whose outputs equal the defaults', set its winner, and
work through the JSON cache."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_10026_amd as rb
    return rb


@pytest.fixture(scope="module")
def kron(rb):
    """Scale-14 Kronecker graph: (off, cols, reordered handle, perm, plain
    handle, roots)."""
    off, cols = graphgen.kronecker_csr(14, 16, 77)
    G = rb.Graph(off, cols)
    perm, _ = G.rcm_reorder()
    P = rb.Graph(off, cols)
    roots = graphgen.sample_roots(off, 6, 7)
    return off, cols, G, perm.cpu().numpy(), P, roots


SINGLE_SETTINGS = [
    dict(block=256, per_cu=1, td_chunk=512),
    dict(block=256, per_cu=4, td_chunk=1024),
    dict(block=1024, per_cu=2),
    dict(lane_row=1),
    dict(lane_row=4096),
    dict(bu_grain=1),
    dict(bu_grain=1024),
    dict(td_chunk=256),
    dict(td_chunk=512),
    dict(td_chunk=1024),
    dict(td_chunk=2048),
    dict(block=256, per_cu=2, td_chunk=1024),
    dict(reset=0),
    dict(block=256, per_cu=2, lane_row=8, bu_grain=4, td_chunk=256, reset=0),
    dict(block=1024, per_cu=1, lane_row=256, bu_grain=256, td_chunk=4096, reset=1),
]


def with_changes(rb, kind, **kw):
    t = rb.default_tuning(kind)
    t.update(kw)
    return t


@pytest.mark.parametrize("setting", SINGLE_SETTINGS, ids=lambda s: ",".join(
    "%s=%s" % kv for kv in s.items()))
def test_single_root_settings_are_exact(rb, kron, setting):
    off, cols, G, perm, P, roots = kron
    t = with_changes(rb, rb.TUNE_SINGLE, **setting)
    for H, ell in ((G, perm), (P, None)):
        H.set_tuning(t)
        assert H.get_tuning() == t
        for direction in (rb.DIR_HEURISTIC, rb.DIR_TD_ONLY, rb.DIR_BU_ONLY):
            for r in roots[:3]:
                d, p = H.bfs(r, opts=rb.make_opts(direction))
                d_o, p_o, _ = oracle.bfs(off, cols, r, ell)
                assert np.array_equal(d.cpu().numpy(), d_o), (setting, direction, r)
                assert np.array_equal(p.cpu().numpy(), p_o), (setting, direction, r)
        # searches run back to back keep the internal arrays consistent
        outs = [H.bfs(r) for r in roots]
        for r, (d, p) in zip(roots, outs):
            d_o, p_o, _ = oracle.bfs(off, cols, r, ell)
            assert np.array_equal(d.cpu().numpy(), d_o)
            assert np.array_equal(p.cpu().numpy(), p_o)
        H.check()
        H.set_tuning(rb.default_tuning(rb.TUNE_SINGLE))


BATCH_SETTINGS = [dict(per_cu=2), dict(lane_row=1), dict(lane_row=4096), dict(bu_grain=1),
                  dict(bu_grain=1024), dict(per_cu=2, lane_row=8, bu_grain=4)]


@pytest.mark.parametrize("setting", BATCH_SETTINGS, ids=lambda s: ",".join(
    "%s=%s" % kv for kv in s.items()))
def test_batch_settings_are_exact(rb, kron, setting):
    off, cols, G, perm, P, roots = kron
    t = with_changes(rb, rb.TUNE_BATCH, **setting)
    G.set_tuning(t, rb.TUNE_BATCH)
    assert G.get_tuning(rb.TUNE_BATCH) == t
    roots_b = list(roots) + list(graphgen.sample_roots(off, 40, 8))
    d, p = G.bfs_batch(roots_b)
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for j in (0, 3, 17, len(roots_b) - 1):
        d_o, p_o, _ = oracle.bfs(off, cols, roots_b[j], perm)
        assert np.array_equal(d[j], d_o) and np.array_equal(p[j], p_o), (setting, j)
    G.set_tuning(rb.default_tuning(rb.TUNE_BATCH), rb.TUNE_BATCH)


@pytest.mark.parametrize("bad", [dict(block=512), dict(per_cu=0), dict(per_cu=5),
                                 dict(lane_row=0), dict(bu_grain=2000), dict(td_chunk=128),
                                 dict(td_chunk=3072), dict(td_chunk=8192),
                                 dict(block=256, td_chunk=2048), dict(reset=2)])
def test_invalid_tuning_is_rejected(rb, kron, bad):
    G = kron[2]
    before = G.get_tuning()
    with pytest.raises(rb.RbfsError) as e:
        G.set_tuning(with_changes(rb, rb.TUNE_SINGLE, **bad))
    assert e.value.code == -1
    assert G.get_tuning() == before
    with pytest.raises(rb.RbfsError):
        G.set_tuning(with_changes(rb, rb.TUNE_BATCH, block=256), rb.TUNE_BATCH)


def test_tuner_single_root(rb, kron):
    off, cols, G, perm, P, roots = kron
    best, recs = G.tune(roots[:4], reps=1)
    # the defaults, then every other value of lane_row, bu_grain, td_chunk and
    # reset at least once (launch shapes that cannot be resident are skipped)
    assert len(recs) >= 1 + 4 + 5 + 2 + 1
    assert recs[0] == dict(rb.default_tuning(rb.TUNE_SINGLE), ms=recs[0]["ms"], mismatches=0)
    assert all(r["mismatches"] == 0 and r["ms"] > 0 for r in recs)
    assert G.get_tuning() == best
    for r in roots:
        d, p = G.bfs(r)
        d_o, p_o, _ = oracle.bfs(off, cols, r, perm)
        assert np.array_equal(d.cpu().numpy(), d_o) and np.array_equal(p.cpu().numpy(), p_o)
    G.set_tuning(rb.default_tuning(rb.TUNE_SINGLE))


def test_tuner_internal_output_space_has_no_reset_dimension(rb, kron):
    G = kron[2]
    _, recs = G.tune(kron[5][:2], reps=1, opts=rb.make_opts(output_space=rb.OUT_INTERNAL))
    r0 = rb.default_tuning(rb.TUNE_SINGLE)["reset"]
    assert all(r["reset"] == r0 for r in recs)
    G.set_tuning(rb.default_tuning(rb.TUNE_SINGLE))


def test_tuner_batch(rb, kron):
    off, cols, G, perm, P, roots = kron
    roots_b = list(graphgen.sample_roots(off, 64, 9))
    best, recs = G.tune(roots_b, kind=rb.TUNE_BATCH, reps=1)
    assert all(r["mismatches"] == 0 for r in recs)
    t0 = rb.default_tuning(rb.TUNE_BATCH)
    assert all(r["block"] == 1024 and r["td_chunk"] == t0["td_chunk"] for r in recs)
    assert G.get_tuning(rb.TUNE_BATCH) == best
    d, p = G.bfs_batch(roots_b)
    for j in (0, 63):
        d_o, p_o, _ = oracle.bfs(off, cols, roots_b[j], perm)
        assert np.array_equal(d[j].cpu().numpy(), d_o)
        assert np.array_equal(p[j].cpu().numpy(), p_o)
    G.set_tuning(rb.default_tuning(rb.TUNE_BATCH), rb.TUNE_BATCH)


def test_tuner_multi_graph(rb):
    csrs, Gs, roots = [], [], []
    for g in range(6):
        off, cols = graphgen.kronecker_csr(9 + g % 3, 16, 500 + g)
        G = rb.Graph(off, cols)
        G.rcm_reorder()
        csrs.append((off, cols, G.iperm().cpu().numpy()))
        Gs.append(G)
        roots.append(graphgen.sample_roots(off, 8, 3))
    M = rb.MultiGraph(Gs)
    before = M.bfs(roots)
    before = [(d.cpu().numpy().copy(), p.cpu().numpy().copy()) for d, p in before]
    best, recs = M.tune(roots, reps=1)
    assert all(r["mismatches"] == 0 for r in recs)
    assert M.get_tuning() == best
    after = M.bfs(roots)  # re-captured with the new parameters
    for (d0, p0), (d1, p1) in zip(before, after):
        assert np.array_equal(d0, d1.cpu().numpy()) and np.array_equal(p0, p1.cpu().numpy())
    off, cols, ip = csrs[4]
    perm = np.empty_like(ip)
    perm[ip] = np.arange(ip.shape[0], dtype=ip.dtype)
    for j in (0, 7):
        d_o, p_o, _ = oracle.bfs(off, cols, roots[4][j], perm)
        assert np.array_equal(before[4][0][j], d_o) and np.array_equal(before[4][1][j], p_o)


def test_tune_cached_round_trip(rb, kron, tmp_path):
    G = kron[2]
    cache = rb.TuningCache(str(tmp_path / "tuning.json"))
    t1, recs = rb.tune_cached(G, kron[5][:2], cache, "kronecker", reps=1)
    assert recs is not None and G.get_tuning() == t1
    G.set_tuning(rb.default_tuning(rb.TUNE_SINGLE))
    cache2 = rb.TuningCache(str(tmp_path / "tuning.json"))
    t2, recs2 = rb.tune_cached(G, kron[5][:2], cache2, "kronecker", reps=1)
    assert recs2 is None and t2 == t1 and G.get_tuning() == t1
    G.set_tuning(rb.default_tuning(rb.TUNE_SINGLE))
