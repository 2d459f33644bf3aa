"""GPU parity: RCM permutation and single-root BFS through the C ABI against
the CPU oracle, bit for bit."""
import random

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


def csr_of(n, edges):
    src = np.array([a for a, b in edges], np.int32)
    dst = np.array([b for a, b in edges], np.int32)
    return oracle.canonical_csr(n, src, dst)


def small_graphs():
    """Edge cases: paths, stars, cycles, cliques, many small components with
    equal-degree ties, isolated vertices, random graphs."""
    gs = []
    gs.append(("path", csr_of(6, [(i, i + 1) for i in range(5)])))
    gs.append(("star", csr_of(9, [(0, i) for i in range(1, 9)])))
    gs.append(("cycle", csr_of(10, [(i, (i + 1) % 10) for i in range(10)])))
    gs.append(("clique", csr_of(7, [(a, b) for a in range(7) for b in range(a + 1, 7)])))
    gs.append(("pairs_iso", csr_of(20, [(2 * i, 2 * i + 1) for i in range(7)])))
    gs.append(("mixed", csr_of(7, [(1, 4), (4, 6), (6, 1), (6, 2), (0, 5)])))
    rng = random.Random(5)
    for t in range(6):
        n = rng.randint(20, 300)
        p = rng.choice([0.005, 0.01, 0.03, 0.1])
        edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
        gs.append(("er%d" % t, csr_of(n + rng.randint(0, 5), edges)))
    # long path: many levels
    gs.append(("longpath", csr_of(3000, [(i, i + 1) for i in range(2999)])))
    # a hub larger than a wave and a chunk
    hub = [(0, i) for i in range(1, 5000)] + [(i, i + 1) for i in range(1, 4999, 2)]
    gs.append(("hub", csr_of(5001, hub)))
    return gs


SMALL = small_graphs()


def kron(scale, seed=1016):
    return graphgen.kronecker_csr(scale, 16, seed)


@pytest.mark.parametrize("name,g", SMALL, ids=[s[0] for s in SMALL])
def test_rcm_small(rb, name, g):
    off, cols = g
    G = rb.Graph(off, cols, validate=True)
    perm, ms = G.rcm_reorder()
    perm_o, iperm_o, nplus = oracle.rcm(off, cols)
    assert np.array_equal(perm.cpu().numpy(), perm_o)
    assert np.array_equal(G.iperm().cpu().numpy(), iperm_o)
    assert G.info()["n_plus"] == nplus


@pytest.mark.parametrize("scale,seed", [(8, 1), (12, 2), (16, 1016)])
def test_rcm_kronecker(rb, scale, seed):
    off, cols = kron(scale, seed)
    G = rb.Graph(off, cols)
    perm, ms = G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    assert np.array_equal(perm.cpu().numpy(), perm_o)


def test_rcm_chung_lu(rb):
    off, cols = graphgen.chung_lu_csr(30000, 1500, seed=3, max_deg=3000.0, mean_deg=12.0)
    G = rb.Graph(off, cols)
    perm, _ = G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    assert np.array_equal(perm.cpu().numpy(), perm_o)


MODES = ["heuristic", "td", "bu", "random"]


def opts_for(rb, mode, rng, **kw):
    if mode == "heuristic":
        return rb.make_opts(rb.DIR_HEURISTIC, **kw)
    if mode == "td":
        return rb.make_opts(rb.DIR_TD_ONLY, **kw)
    if mode == "bu":
        return rb.make_opts(rb.DIR_BU_ONLY, **kw)
    sched = [0] + [rng.randint(0, 1) for _ in range(40)]
    return rb.make_opts(rb.DIR_SCHEDULE, schedule=sched, **kw)


def check_bfs(rb, G, off, cols, roots, ell, modes=MODES, seed=0):
    rng = random.Random(seed)
    for root in roots:
        d_o, p_o, _ = oracle.bfs(off, cols, root, ell)
        for mode in modes:
            d, p = G.bfs(root, opts=opts_for(rb, mode, rng))
            assert np.array_equal(d.cpu().numpy(), d_o), (root, mode)
            assert np.array_equal(p.cpu().numpy(), p_o), (root, mode)


@pytest.mark.parametrize("name,g", SMALL, ids=[s[0] for s in SMALL])
def test_bfs_small_unreordered(rb, name, g):
    off, cols = g
    G = rb.Graph(off, cols)
    n = off.shape[0] - 1
    roots = sorted(set([0, n - 1, n // 2]))
    check_bfs(rb, G, off, cols, roots, None)


@pytest.mark.parametrize("name,g", SMALL, ids=[s[0] for s in SMALL])
def test_bfs_small_rcm(rb, name, g):
    off, cols = g
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    n = off.shape[0] - 1
    roots = sorted(set([0, n - 1, n // 2]))
    check_bfs(rb, G, off, cols, roots, perm_o)


@pytest.mark.parametrize("scale", [10, 14, 16])
def test_bfs_kronecker_rcm(rb, scale):
    off, cols = kron(scale)
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    roots = graphgen.sample_roots(off, 8, 7)
    check_bfs(rb, G, off, cols, roots, perm_o, seed=scale)


def test_bfs_kronecker_unreordered(rb):
    off, cols = kron(14, 3)
    G = rb.Graph(off, cols)
    roots = graphgen.sample_roots(off, 4, 7)
    check_bfs(rb, G, off, cols, roots, None)


def test_bfs_internal_output(rb):
    off, cols = kron(12, 4)
    G = rb.Graph(off, cols)
    perm_t, _ = G.rcm_reorder()
    perm = perm_t.cpu().numpy()
    iperm = G.iperm().cpu().numpy()
    root = graphgen.sample_roots(off, 1, 7)[0]
    d_o, p_o, _ = oracle.bfs(off, cols, root, perm)
    d, p = G.bfs(root, opts=rb.make_opts(output_space=rb.OUT_INTERNAL))
    d, p = d.cpu().numpy(), p.cpu().numpy()
    # internal index i holds vertex iperm[i]; parents are internal labels
    assert np.array_equal(d[perm], d_o)
    exp = np.where(p_o >= 0, perm[np.maximum(p_o, 0)], -1)
    assert np.array_equal(p[perm], exp)


def test_isolated_root(rb):
    off, cols = csr_of(8, [(0, 1), (1, 2), (4, 5)])
    for reorder in (False, True):
        G = rb.Graph(off, cols)
        if reorder:
            G.rcm_reorder()
        for root in (3, 6, 7):
            d, p = G.bfs(root)
            d, p = d.cpu().numpy(), p.cpu().numpy()
            exp_d = -np.ones(8, np.int32)
            exp_d[root] = 0
            exp_p = -np.ones(8, np.int32)
            exp_p[root] = root
            assert np.array_equal(d, exp_d) and np.array_equal(p, exp_p)


def test_stats_match_oracle_schedule(rb):
    """Per-level counters and the heuristic directions equal the oracle's
    replay of the alpha/beta rule."""
    off, cols = kron(14, 9)
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    perm_o, _, nplus = oracle.rcm(off, cols)
    for root in graphgen.sample_roots(off, 4, 7):
        for alpha, beta in [(14, 24), (64, 8), (2, 2)]:
            d, p, st = G.bfs(root, opts=rb.make_opts(alpha=alpha, beta=beta), stats=True)
            d_o, _, nlev = oracle.bfs(off, cols, root, perm_o)
            c = oracle.level_counters(off, cols, d_o, perm_o, nplus)
            sched = oracle.heuristic_schedule(c["nf"], c["mf"], c["mu"], nplus, alpha, beta)
            assert st["levels"] == nlev
            assert st["dir"] == sched.tolist()
            assert st["nf"] == c["nf"].tolist()
            assert st["mf"] == c["mf"].tolist()
            assert st["mu"] == c["mu"].tolist()
            assert st["reached"] == int((d_o >= 0).sum())
            assert st["component_edges"] == oracle.component_edges(off, d_o)
            # bottom-up levels read exactly the oracle's count of examined
            # entries over the root's component (after RCM the sweep skips
            # the other components)
            for lv in range(nlev):
                if st["dir"][lv] == 1:
                    assert st["edges"][lv] == c["ebc"][lv]
                else:
                    assert st["edges"][lv] == c["mf"][lv]
    # forced schedules: every bottom-up level after the first walks the
    # vertex list the previous one left; a work range taken twice would
    # show up in the entry counts and in |F|
    for root in graphgen.sample_roots(off, 6, 11):
        d_o, _, nlev = oracle.bfs(off, cols, root, perm_o)
        c = oracle.level_counters(off, cols, d_o, perm_o, nplus)
        for mode in (rb.DIR_TD_ONLY, rb.DIR_BU_ONLY):
            d, p, st = G.bfs(root, opts=rb.make_opts(mode), stats=True)
            assert st["levels"] == nlev and st["nf"] == c["nf"].tolist()
            for lv in range(1, nlev):
                want = c["ebc"][lv] if mode == rb.DIR_BU_ONLY else c["mf"][lv]
                assert st["edges"][lv] == want, (mode, root, lv)
    # without RCM there are no component intervals: the sweep covers every
    # vertex, as in Algorithm 2
    P = rb.Graph(off, cols)
    for root in graphgen.sample_roots(off, 2, 8):
        _, _, st = P.bfs(root, opts=rb.make_opts(rb.DIR_BU_ONLY), stats=True)
        d_o, _, nlev = oracle.bfs(off, cols, root)
        c = oracle.level_counters(off, cols, d_o)
        for lv in range(1, nlev):
            assert st["edges"][lv] == c["ebu"][lv]


def test_repeatable(rb):
    off, cols = kron(15, 5)
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    root = graphgen.sample_roots(off, 1, 7)[0]
    d0, p0 = G.bfs(root)
    d0, p0 = d0.clone(), p0.clone()
    for _ in range(20):
        d, p = G.bfs(root)
        assert torch.equal(d, d0) and torch.equal(p, p0)
    G.check()


def test_graph_create_rejects_bad_csr(rb):
    off = np.array([0, 1, 2], np.int64)
    cols = np.array([1, 1], np.int32)  # self loop at vertex 1
    with pytest.raises(rb.RbfsError):
        rb.Graph(off, cols, validate=True)
    off = np.array([0, 2, 1], np.int64)  # non-monotone
    with pytest.raises(rb.RbfsError):
        rb.Graph(off, np.array([1, 0], np.int32))
    off = np.array([0, 1, 2], np.int64)
    with pytest.raises(rb.RbfsError):
        rb.Graph(off, np.array([5, 0], np.int32))  # column out of range
    off = np.array([0, 1, 1], np.int64)  # asymmetric
    with pytest.raises(rb.RbfsError):
        rb.Graph(off, np.array([1], np.int32), validate=True)


def test_root_out_of_range(rb):
    off, cols = csr_of(4, [(0, 1)])
    G = rb.Graph(off, cols)
    with pytest.raises(rb.RbfsError):
        G.bfs(4)
    with pytest.raises(rb.RbfsError):
        G.bfs(-1)


def test_device_generator_matches_host(rb):
    off_h, cols_h = graphgen.kronecker_csr(14, 16, 33)
    off_d, cols_d = graphgen.kronecker_csr_device(14, 16, 33)
    assert np.array_equal(off_d.cpu().numpy(), off_h)
    assert np.array_equal(cols_d.cpu().numpy(), cols_h)
    off_h, cols_h = graphgen.chung_lu_csr(20000, 1000, seed=4, max_deg=2000.0, mean_deg=10.0)
    off_d, cols_d = graphgen.chung_lu_csr_device(20000, 1000, seed=4, max_deg=2000.0,
                                                 mean_deg=10.0)
    assert np.array_equal(off_d.cpu().numpy(), off_h)
    assert np.array_equal(cols_d.cpu().numpy(), cols_h)


@pytest.mark.parametrize("max_keys", [40000, 150001, 10 ** 6])
def test_device_generator_in_range_passes(rb, max_keys):
    """The device generator cut into passes over source-label ranges (a few
    tens of thousands of keys each, as the largest graphs need on one GPU)
    gives the host generator's CSR."""
    off_h, cols_h = graphgen.kronecker_csr(14, 16, 33)
    info = {}
    off_d, cols_d = graphgen.kronecker_csr_device(14, 16, 33, max_pass_keys=max_keys, info=info)
    assert info["passes"] >= (2 if max_keys < 500000 else 1)
    assert np.array_equal(off_d.cpu().numpy(), off_h)
    assert np.array_equal(cols_d.cpu().numpy(), cols_h)


def test_device_tuple_count_matches_host(rb):
    """The benchmark's Graph500-style edge count: generated tuples with both
    endpoints reached, on the device against the host tuples and the
    oracle's depths."""
    n, src, dst = graphgen.kronecker_tuples(12, 16, 5)
    off, cols = graphgen.csr_from_tuples(n, src, dst)
    for root in graphgen.sample_roots(off, 3, 3):
        d_o, _, _ = oracle.bfs(off, cols, root)
        want = int(np.sum((d_o[src] >= 0) & (d_o[dst] >= 0)))
        got = graphgen.kronecker_tuples_reached_device(12, torch.from_numpy(d_o).cuda(), 16, 5)
        assert got == want
    iso = int(np.flatnonzero(np.diff(off) == 0)[0])
    d_o, _, _ = oracle.bfs(off, cols, iso)
    got = graphgen.kronecker_tuples_reached_device(12, torch.from_numpy(d_o).cuda(), 16, 5)
    assert got == int(np.sum((src == iso) & (dst == iso)))


@pytest.mark.parametrize("reorder", [False, True], ids=["original", "rcm"])
def test_without_load_balance_bit_exact(rb, reorder):
    """The load-balance ablation (OPT_NO_BALANCE: whole rows per wave
    top-down, equal vertex ranges without stealing bottom-up) gives the
    oracle's arrays in every direction mode, and its per-workgroup work
    still adds up to the level counters."""
    off, cols = kron(14, 8)
    G = rb.Graph(off, cols)
    ell = G.rcm_reorder()[0].cpu().numpy() if reorder else None
    rng = random.Random(3)
    for root in graphgen.sample_roots(off, 3, 9):
        d_o, p_o, _ = oracle.bfs(off, cols, root, ell)
        for mode in MODES:
            d, p = G.bfs(root, opts=opts_for(rb, mode, rng, no_balance=True))
            assert np.array_equal(d.cpu().numpy(), d_o), (root, mode)
            assert np.array_equal(p.cpu().numpy(), p_o), (root, mode)
        _, _, st = G.bfs(root, opts=rb.make_opts(no_balance=True, wg_work=True), stats=True)
        W = G.wg_work()
        for d in range(st["levels"]):
            want = st["mf"][d] if st["dir"][d] == 0 else st["edges"][d]
            assert int(W[d].sum()) == want, (root, d)


def test_workgroup_work_adds_up(rb):
    """Per-workgroup work of a search (OPT_WG_WORK): summed over the
    workgroups, every level gives the level's counted work -- its frontier
    edges m_f top-down, the row entries read bottom-up."""
    off, cols = kron(14, 3)
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    for r in graphgen.sample_roots(off, 3, 4):
        for mode in (rb.DIR_HEURISTIC, rb.DIR_TD_ONLY, rb.DIR_BU_ONLY):
            _, _, st = G.bfs(r, opts=rb.make_opts(mode, wg_work=True), stats=True)
            W = G.wg_work()
            assert W.shape[0] == st["levels"]
            for d in range(st["levels"]):
                want = st["mf"][d] if st["dir"][d] == 0 else st["edges"][d]
                assert int(W[d].sum()) == want, (r, mode, d)
                assert (W[d] >= 0).all()
    G.bfs(0)
    with pytest.raises(rb.RbfsError):
        G.wg_work()


@pytest.mark.parametrize("n", [1, 7])
@pytest.mark.parametrize("reorder", [False, True], ids=["original", "rcm"])
def test_edgeless_graph(rb, n, reorder):
    """No edges at all: every vertex is isolated, so the relabelling is the
    identity with an empty V+, and every search reaches its root only."""
    off = np.zeros(n + 1, np.int64)
    cols = np.zeros(0, np.int32)
    G = rb.Graph(off, cols)
    perm_o = oracle.rcm(off, cols)[0]
    if reorder:
        perm, _ = G.rcm_reorder()
        assert np.array_equal(perm.cpu().numpy(), perm_o)
        assert G.info()["n_plus"] == 0
        G0 = rb.Graph(off, cols)
        perm0, _ = G0.rcm_reorder(keep=0)
        assert np.array_equal(perm0.cpu().numpy(), oracle.rcm_partial(off, cols, 0)[0])
    roots = list(range(n))
    for r in roots:
        d_o, p_o, _ = oracle.bfs(off, cols, r, perm_o if reorder else None)
        for dirc in (rb.DIR_HEURISTIC, rb.DIR_TD_ONLY, rb.DIR_BU_ONLY):
            d, p = G.bfs(r, opts=rb.make_opts(dirc))
            assert np.array_equal(d.cpu().numpy(), d_o) and np.array_equal(p.cpu().numpy(), p_o)
            assert G.certify(r, d, p) == 0
    dB, pB = G.bfs_batch(roots)
    for j, r in enumerate(roots):
        d_o, p_o, _ = oracle.bfs(off, cols, r, perm_o if reorder else None)
        assert np.array_equal(dB[j].cpu().numpy(), d_o) and np.array_equal(pB[j].cpu().numpy(), p_o)


def _relabelled_csr(off, cols, perm):
    """Host reference of the relabelled CSR: row k is the row of the vertex
    with new label k, its neighbours renamed by perm, ascending."""
    n = off.shape[0] - 1
    iperm = np.empty(n, np.int64)
    iperm[perm] = np.arange(n)
    deg = np.diff(off)
    noff = np.zeros(n + 1, np.int64)
    noff[1:] = np.cumsum(deg[iperm])
    ncols = np.empty(cols.shape[0], np.int32)
    for k in range(n):
        v = iperm[k]
        ncols[noff[k]:noff[k + 1]] = np.sort(perm[cols[off[v]:off[v + 1]]])
    return noff, ncols


def test_graph_csr_export(rb):
    off, cols = graphgen.kronecker_csr(11, 16, 4711)
    G = rb.Graph(off, cols)
    o0, c0 = G.csr()
    assert np.array_equal(o0.cpu().numpy(), off) and np.array_equal(c0.cpu().numpy(), cols)
    perm_t, _ = G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    o1, c1 = G.csr()
    noff, ncols = _relabelled_csr(off, cols, perm_o)
    assert np.array_equal(o1.cpu().numpy(), noff)
    assert np.array_equal(c1.cpu().numpy(), ncols)
    # a search on the exported graph in its own labels equals the internal output
    r = graphgen.sample_roots(off, 1, 3)[0]
    d, p = G.bfs(r, opts=rb.make_opts(output_space=rb.OUT_INTERNAL))
    d_o, p_o, _ = oracle.bfs(noff, ncols, int(perm_o[r]))
    assert np.array_equal(d.cpu().numpy(), d_o) and np.array_equal(p.cpu().numpy(), p_o)


@pytest.mark.parametrize("stage", [-1, 1], ids=["device", "host-staged"])
@pytest.mark.parametrize("batch", [1, 1000, 50000])
def test_rcm_relabel_in_batches(rb, batch, stage):
    """The relabelled CSR built in batches of new rows (as the largest graphs
    need), with the old columns on the device or staged in host memory,
    equals the host reference, for the full and a partial order, and
    searches on it stay bit-exact."""
    off, cols = graphgen.kronecker_csr(13, 16, 7007)
    perm_o, _, _ = oracle.rcm(off, cols)
    for keep in (None, 3000):
        G = rb.Graph(off, cols)
        G.set_rcm_batch(batch)
        G.set_rcm_staging(stage)
        perm_t, _ = G.rcm_reorder(keep=keep)
        perm = perm_t.cpu().numpy()
        ref = perm_o if keep is None else oracle.rcm_partial(off, cols, keep)[0]
        assert np.array_equal(perm, ref)
        o1, c1 = G.csr()
        noff, ncols = _relabelled_csr(off, cols, perm)
        assert np.array_equal(o1.cpu().numpy(), noff)
        assert np.array_equal(c1.cpu().numpy(), ncols)
        for r in graphgen.sample_roots(off, 2, 11):
            d, p = G.bfs(r)
            d_o, p_o, _ = oracle.bfs(off, cols, r, perm)
            assert np.array_equal(d.cpu().numpy(), d_o)
            assert np.array_equal(p.cpu().numpy(), p_o)


@pytest.mark.parametrize("cap", [1, 64, 5000])
def test_small_subqueues_spill_exactly(rb, cap):
    """Frontier sub-queues of a few entries (every flush spills into the
    shared overflow queue): outputs and level counters stay the oracle's in
    every direction mode, with and without load balancing."""
    off, cols = kron(14, 12)
    rng = random.Random(cap)
    for reorder in (False, True):
        G = rb.Graph(off, cols)
        G.set_queue_cap(cap)
        ell = G.rcm_reorder()[0].cpu().numpy() if reorder else None
        n_sweep = G.info()["n_plus"] if reorder else G.n
        for root in graphgen.sample_roots(off, 2, 21):
            d_o, p_o, _ = oracle.bfs(off, cols, root, ell)
            c = oracle.level_counters(off, cols, d_o, ell=ell, n_sweep=n_sweep)
            for mode in MODES:
                for nb in (False, True):
                    d, p, st = G.bfs(root, opts=opts_for(rb, mode, rng, no_balance=nb),
                                     stats=True)
                    assert np.array_equal(d.cpu().numpy(), d_o), (root, mode, nb)
                    assert np.array_equal(p.cpu().numpy(), p_o), (root, mode, nb)
                    assert st["nf"] == [int(x) for x in c["nf"]]
                    assert st["mf"] == [int(x) for x in c["mf"]]
        G.check()


def components_graph(seed=11):
    """Components of different sizes (a random graph spanning several blocks
    of 4096 original IDs, a path, a star, pairs) and isolated vertices, with
    labels shuffled so that the components interleave in ID space; n is not
    a multiple of 4096."""
    rng = random.Random(seed)
    edges, base = [], 0
    big = 9000
    for u in range(big):
        for _ in range(3):
            v = rng.randrange(big)
            if v != u:
                edges.append((u, v))
    base = big
    edges += [(base + i, base + i + 1) for i in range(59)]
    base += 60
    edges += [(base, base + i) for i in range(1, 25)]
    base += 25
    for i in range(40):
        edges.append((base + 2 * i, base + 2 * i + 1))
    base += 80
    n = base + 333  # isolated tail
    relabel = list(range(n))
    rng.shuffle(relabel)
    return csr_of(n, [(relabel[a], relabel[b]) for a, b in edges]), relabel


def test_output_blocks_across_components(rb):
    # a search must leave no entry of an earlier search's component behind
    # (searches in other components, isolated roots, searches with
    # internal-label outputs in between, both reset modes); n spans several
    # blocks of 4096 IDs with a ragged tail
    (off, cols), relabel = components_graph()
    n = off.shape[0] - 1
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    big, path, star, pair = relabel[5], relabel[9000 + 7], relabel[9060 + 3], relabel[9085]
    iso = [relabel[n - 1], relabel[n - 200]]
    seq = [big, path, iso[0], big, star, pair, iso[1], path, big, big, star]
    internal = rb.make_opts(output_space=rb.OUT_INTERNAL)
    for reset in (0, 1):
        t = rb.default_tuning(rb.TUNE_SINGLE)
        t["reset"] = reset
        G.set_tuning(t)
        for i, root in enumerate(seq):
            if i % 3 == 2:
                G.bfs(seq[(i + 1) % len(seq)], opts=internal)
            d, p = G.bfs(root)
            d_o, p_o, _ = oracle.bfs(off, cols, root, perm_o)
            assert np.array_equal(d.cpu().numpy(), d_o), (reset, i, root)
            assert np.array_equal(p.cpu().numpy(), p_o), (reset, i, root)
    G.set_tuning(rb.default_tuning(rb.TUNE_SINGLE))


def test_searches_in_a_row_across_base_runs(rb):
    # each search lowers the depth-field base instead of re-initialising the
    # packed pairs; a run of bases lasts at most 64 searches, then one search
    # initialises.  150 searches in a row (three runs), roots in different
    # components and isolated ones, both output spaces and both reset modes,
    # each compared with the oracle
    (off, cols), relabel = components_graph(seed=23)
    n = off.shape[0] - 1
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    iperm = G.iperm().cpu().numpy()
    roots = [relabel[5], relabel[9000 + 7], relabel[n - 1], relabel[9060 + 3], relabel[77]]
    expect = {r: oracle.bfs(off, cols, r, perm_o)[:2] for r in roots}
    internal = rb.make_opts(output_space=rb.OUT_INTERNAL)
    for i in range(150):
        if i == 100:
            t = rb.default_tuning(rb.TUNE_SINGLE)
            t["reset"] = 1 - t["reset"]
            G.set_tuning(t)
        r = roots[i % len(roots)]
        d_o, p_o = expect[r]
        if i % 7 == 3:
            d, p = G.bfs(r, opts=internal)
            d, p = d.cpu().numpy(), p.cpu().numpy()
            exp_p = np.where(p_o >= 0, np.argsort(iperm)[np.maximum(p_o, 0)], -1)
            assert np.array_equal(d[np.argsort(iperm)], d_o), i
            assert np.array_equal(p[np.argsort(iperm)], exp_p), i
        else:
            d, p = G.bfs(r)
            assert np.array_equal(d.cpu().numpy(), d_o), i
            assert np.array_equal(p.cpu().numpy(), p_o), i
    G.set_tuning(rb.default_tuning(rb.TUNE_SINGLE))


@pytest.mark.parametrize("name,g", [s for s in SMALL if s[0] in ("path", "mixed", "er3", "hub")] +
                         [("kron14", kron(14, 5))], ids=lambda x: x if isinstance(x, str) else "")
def test_bandwidth(rb, name, g):
    # the largest |u - v| over the edges, before RCM in the input labels and
    # after it in the oracle's RCM labels
    off, cols = g
    n = off.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(off))
    G = rb.Graph(off, cols)
    exp0 = int(np.abs(rows - cols).max()) if cols.size else 0
    assert G.bandwidth() == exp0
    G.rcm_reorder()
    perm_o, _, _ = oracle.rcm(off, cols)
    exp1 = int(np.abs(perm_o[rows].astype(np.int64) - perm_o[cols]).max()) if cols.size else 0
    assert G.bandwidth() == exp1
