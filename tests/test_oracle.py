"""Pins for the CPU oracle (no GPU): worked examples derived by hand from the
paper's algorithms, brute force on tiny graphs, library routines for the
special cases they cover, closed forms, invariants, and planted mistakes the
certificates must reject."""
import itertools
import json
import os
import random

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rcm_worked_examples.json")


def csr_of(n, edges):
    src = [a for a, b in edges]
    dst = [b for a, b in edges]
    return oracle.canonical_csr(n, np.array(src, np.int32), np.array(dst, np.int32))


def random_graph(rng, n, p, isolated=0):
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    return csr_of(n + isolated, edges), edges


# --------------------------------------------------------------------------
# worked examples (Algorithm 3; predecessor map of section 2.1)

with open(GOLDEN) as f:
    CASES = json.load(f)["cases"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_rcm_worked_example(case):
    off, cols = csr_of(case["n"], case["edges"])
    perm, iperm, nplus = oracle.rcm(off, cols)
    assert nplus == case["nplus"]
    assert iperm.tolist() == case["iperm"]
    assert perm.tolist() == case["perm"]
    assert oracle.certify_rcm(off, cols, perm) == 0
    if "bandwidth_after" in case:
        assert oracle.bandwidth(off, cols, perm) == case["bandwidth_after"]
    if "bfs_after_rcm" in case:
        b = case["bfs_after_rcm"]
        depth, parent, _ = oracle.bfs(off, cols, b["root"], perm)
        assert depth.tolist() == b["depth"]
        assert parent.tolist() == b["parent"]
    if "bfs_original_labels" in case:
        b = case["bfs_original_labels"]
        depth, parent, _ = oracle.bfs(off, cols, b["root"], None)
        assert depth.tolist() == b["depth"]
        assert parent.tolist() == b["parent"]


# --------------------------------------------------------------------------
# canonical CSR

def test_canonical_csr_closed_form():
    # duplicates, both orientations and self-loops collapse to one undirected edge
    off, cols = csr_of(4, [(0, 1), (1, 0), (0, 1), (2, 2), (3, 1)])
    assert off.tolist() == [0, 1, 3, 3, 4]
    assert cols.tolist() == [1, 0, 3, 1]


def test_generator_csr_matches_oracle_canonicalisation():
    for scale in (8, 11):
        n, src, dst = graphgen.kronecker_tuples(scale, 16, 5)
        off_g, cols_g = graphgen.csr_from_tuples(n, src, dst)
        off_o, cols_o = oracle.canonical_csr(n, src, dst)
        assert np.array_equal(off_g, off_o)
        assert np.array_equal(cols_g, cols_o)


def test_canonical_csr_properties_kron():
    off, cols = graphgen.kronecker_csr(12, 16, 3)
    n = off.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(off))
    assert not np.any(rows == cols)  # no self-loops
    for v in range(0, n, 97):
        r = cols[off[v]:off[v + 1]]
        assert np.all(np.diff(r) > 0)  # strictly ascending
    fwd = set(zip(rows.tolist(), cols.tolist()))
    assert all((b, a) in fwd for a, b in fwd)  # symmetric


# --------------------------------------------------------------------------
# BFS: brute force (Floyd-Warshall distances + exhaustive max-label parent)

def brute_bfs(n, edges, root, ell):
    INF = 10 ** 9
    dist = [[INF] * n for _ in range(n)]
    for i in range(n):
        dist[i][i] = 0
    for a, b in edges:
        if a != b:
            dist[a][b] = dist[b][a] = 1
    for k in range(n):
        for i in range(n):
            for j in range(n):
                if dist[i][k] + dist[k][j] < dist[i][j]:
                    dist[i][j] = dist[i][k] + dist[k][j]
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    depth = [dist[root][v] if dist[root][v] < INF else -1 for v in range(n)]
    parent = [-1] * n
    for v in range(n):
        if depth[v] > 0:
            cands = [u for u in adj[v] if depth[u] == depth[v] - 1]
            parent[v] = max(cands, key=lambda u: ell[u])
    parent[root] = root
    return depth, parent


@pytest.mark.parametrize("seed", range(40))
def test_bfs_brute_force(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 12)
    iso = rng.randint(0, 2)
    (off, cols), edges = random_graph(rng, n, rng.choice([0.15, 0.3, 0.6]), iso)
    ntot = n + iso
    labels = list(range(ntot))
    rng.shuffle(labels)
    ell = np.array(labels, np.int32)
    for root in range(ntot):
        for e in (None, ell):
            depth, parent, _ = oracle.bfs(off, cols, root, e)
            bd, bp = brute_bfs(ntot, edges, root, list(range(ntot)) if e is None else labels)
            assert depth.tolist() == bd
            assert parent.tolist() == bp
            assert oracle.certify_bfs(off, cols, root, depth, parent, e) == 0


def test_bfs_depth_matches_scipy():
    sp = pytest.importorskip("scipy.sparse")
    csg = pytest.importorskip("scipy.sparse.csgraph")
    off, cols = graphgen.kronecker_csr(11, 16, 9)
    n = off.shape[0] - 1
    A = sp.csr_matrix((np.ones(cols.shape[0]), cols, off), shape=(n, n))
    for root in graphgen.sample_roots(off, 4, 7):
        d_ref = csg.shortest_path(A, unweighted=True, indices=root)
        d_ref = np.where(np.isinf(d_ref), -1, d_ref).astype(np.int64)
        depth, parent, _ = oracle.bfs(off, cols, root)
        assert np.array_equal(depth, d_ref)


def test_isolated_root():
    off, cols = csr_of(5, [(0, 1), (1, 2)])
    depth, parent, nlev = oracle.bfs(off, cols, 4)
    assert depth.tolist() == [-1, -1, -1, -1, 0]
    assert parent.tolist() == [-1, -1, -1, -1, 4]
    assert nlev == 1


# --------------------------------------------------------------------------
# RCM: exhaustive uniqueness of the certificate, invariants

@pytest.mark.parametrize("seed", range(12))
def test_rcm_certificate_unique_by_enumeration(seed):
    """Among all n! labellings of a tiny graph exactly one passes the RCM
    certificate, and it is the oracle's Algorithm 3 result."""
    rng = random.Random(100 + seed)
    n = rng.randint(2, 6)
    iso = rng.randint(0, 1)
    (off, cols), _ = random_graph(rng, n, rng.choice([0.3, 0.5, 0.8]), iso)
    ntot = n + iso
    perm, _, _ = oracle.rcm(off, cols)
    passing = [p for p in itertools.permutations(range(ntot))
               if oracle.certify_rcm(off, cols, np.array(p, np.int32)) == 0]
    assert passing == [tuple(perm.tolist())]


def rcm_components_ok(off, cols, perm, nplus):
    """Each connected component occupies one contiguous label range."""
    n = off.shape[0] - 1
    iperm = np.empty(n, np.int64)
    iperm[perm] = np.arange(n)
    comp = -np.ones(n, np.int64)
    c = 0
    for s in range(n):
        if comp[s] >= 0 or off[s + 1] == off[s]:
            continue
        stack = [s]
        comp[s] = c
        while stack:
            u = stack.pop()
            for w in cols[off[u]:off[u + 1]]:
                if comp[w] < 0:
                    comp[w] = c
                    stack.append(w)
        c += 1
    labs = {}
    for v in range(n):
        if comp[v] >= 0:
            labs.setdefault(comp[v], []).append(perm[v])
    for ls in labs.values():
        if max(ls) - min(ls) + 1 != len(ls):
            return False
    return all(perm[v] < nplus for v in range(n) if off[v + 1] > off[v])


@pytest.mark.parametrize("seed", range(20))
def test_rcm_invariants_random(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(2, 60)
    (off, cols), _ = random_graph(rng, n, rng.choice([0.02, 0.05, 0.1, 0.3]), rng.randint(0, 5))
    perm, iperm, nplus = oracle.rcm(off, cols)
    ntot = off.shape[0] - 1
    assert sorted(perm.tolist()) == list(range(ntot))
    assert np.array_equal(perm[iperm], np.arange(ntot))
    assert nplus == int((np.diff(off) > 0).sum())
    assert rcm_components_ok(off, cols, perm, nplus)
    assert oracle.certify_rcm(off, cols, perm) == 0


def test_rcm_kronecker_structure():
    """Paper statements checked as invariants: the bandwidth falls below |V+|,
    the giant component ends at n+ (section 3.2), and the mean degree rises
    with the RCM label (section 3.3)."""
    off, cols = graphgen.kronecker_csr(14, 16, 21)
    perm, iperm, nplus = oracle.rcm(off, cols)
    assert oracle.certify_rcm(off, cols, perm) == 0
    bw0 = oracle.bandwidth(off, cols)
    bw1 = oracle.bandwidth(off, cols, perm)
    assert bw1 < nplus < bw0 + nplus
    assert bw1 < bw0
    deg = np.diff(off)[iperm[:nplus]]
    q = nplus // 4
    assert deg[:q].mean() < deg[-q:].mean()
    # the vertex with label n+-1 is in the giant component (last CM start reversed)
    roots = graphgen.sample_roots(off, 1, 7)
    depth, _, _ = oracle.bfs(off, cols, roots[0])
    reached = depth >= 0
    assert reached[iperm[nplus - 1]]


def test_rcm_bandwidth_vs_scipy():
    """scipy's RCM uses other tie-breaks and start vertices, so only the
    bandwidth reduction is compared, not the permutation."""
    sp = pytest.importorskip("scipy.sparse")
    csg = pytest.importorskip("scipy.sparse.csgraph")
    off, cols = graphgen.kronecker_csr(12, 16, 4)
    n = off.shape[0] - 1
    A = sp.csr_matrix((np.ones(cols.shape[0]), cols, off), shape=(n, n))
    p_sc = csg.reverse_cuthill_mckee(A, symmetric_mode=True)
    ell_sc = np.empty(n, np.int32)
    ell_sc[p_sc] = np.arange(n)
    perm, _, _ = oracle.rcm(off, cols)
    bw0 = oracle.bandwidth(off, cols)
    assert oracle.bandwidth(off, cols, perm) < bw0
    assert oracle.bandwidth(off, cols, ell_sc) < bw0


# --------------------------------------------------------------------------
# planted mistakes: the certificates must reject them

def test_certify_bfs_rejects_mutations():
    off, cols = graphgen.kronecker_csr(10, 16, 2)
    perm, _, _ = oracle.rcm(off, cols)
    root = graphgen.sample_roots(off, 1, 7)[0]
    depth, parent, _ = oracle.bfs(off, cols, root, perm)
    assert oracle.certify_bfs(off, cols, root, depth, parent, perm) == 0
    # same arrays judged in the wrong label space: some parent is no longer maximal
    assert oracle.certify_bfs(off, cols, root, depth, parent, None) != 0
    rng = np.random.default_rng(0)
    reached = np.nonzero(depth > 0)[0]
    for _ in range(20):
        v = int(rng.choice(reached))
        d2 = depth.copy()
        d2[v] += 1
        assert oracle.certify_bfs(off, cols, root, d2, parent, perm) != 0
        p2 = parent.copy()
        cands = [u for u in cols[off[v]:off[v + 1]] if depth[u] == depth[v] - 1 and u != parent[v]]
        if cands:
            p2[v] = cands[0]
            assert oracle.certify_bfs(off, cols, root, depth, p2, perm) != 0
        p3 = parent.copy()
        p3[v] = -1
        assert oracle.certify_bfs(off, cols, root, depth, p3, perm) != 0


def test_certify_rcm_rejects_mutations():
    off, cols = graphgen.kronecker_csr(10, 16, 2)
    perm, _, nplus = oracle.rcm(off, cols)
    rng = np.random.default_rng(1)
    for _ in range(30):
        i, j = rng.choice(nplus, 2, replace=False)
        p2 = perm.copy()
        a = np.nonzero(perm == i)[0][0]
        b = np.nonzero(perm == j)[0][0]
        p2[a], p2[b] = p2[b], p2[a]
        assert oracle.certify_rcm(off, cols, p2) != 0
    # not reversed (plain Cuthill-McKee order)
    p3 = perm.copy()
    p3[perm < nplus] = nplus - 1 - perm[perm < nplus]
    assert oracle.certify_rcm(off, cols, p3) != 0


# --------------------------------------------------------------------------
# level counters and the direction rule

def test_level_counters_star_closed_form():
    k = 6
    off, cols = csr_of(k + 1, [(0, i) for i in range(1, k + 1)])
    depth, _, _ = oracle.bfs(off, cols, 0)
    c = oracle.level_counters(off, cols, depth)
    assert c["nf"].tolist() == [1, k]
    assert c["mf"].tolist() == [k, k]
    assert c["nu"].tolist() == [k, 0]
    assert c["mu"].tolist() == [k, 0]
    # bottom-up at level 0: every leaf's only neighbour is the centre: 1 edge each
    assert c["ebu"].tolist() == [k, 0]
    # from a leaf, labels identity: level 1 = centre; leaves 2..k scan 1 edge
    depth, _, _ = oracle.bfs(off, cols, 1)
    c = oracle.level_counters(off, cols, depth)
    assert c["nf"].tolist() == [1, 1, k - 1]
    # the centre scans labels k, k-1, .. and meets the root (label 1) last: k
    # edges; leaves 2..k: 1 edge each (no hit)
    assert c["ebu"].tolist() == [k + (k - 1), k - 1, 0]


def test_level_counters_first_hit_index():
    # v=0 with neighbours 1..4; frontier at level 1 is {3, 4} (via root 5)
    edges = [(0, 1), (0, 2), (0, 3), (0, 4), (5, 3), (5, 4), (1, 6), (2, 6)]
    off, cols = csr_of(7, edges)
    depth, _, _ = oracle.bfs(off, cols, 5)
    assert depth[0] == 2 and depth[3] == 1
    c = oracle.level_counters(off, cols, depth)
    # at level 1 vertex 0 scans 4 first (largest label) -> 1 edge; with
    # labels reversed it scans 1, 2, 3 -> 3 edges.  Vertices 1, 2, 6 have no
    # neighbour in F_1.
    base = c["ebu"][1]
    ell = np.array([6, 5, 4, 3, 2, 1, 0], np.int32)
    c2 = oracle.level_counters(off, cols, depth, ell)
    assert c2["ebu"][1] - base == 2


def test_level_counters_invariants_kron():
    off, cols = graphgen.kronecker_csr(11, 16, 8)
    perm, _, nplus = oracle.rcm(off, cols)
    root = graphgen.sample_roots(off, 1, 7)[0]
    depth, _, nlev = oracle.bfs(off, cols, root, perm)
    c = oracle.level_counters(off, cols, depth, perm, nplus)
    assert c["nf"].sum() == (depth >= 0).sum()
    assert c["mf"].sum() == np.diff(off)[depth >= 0].sum()
    for d in range(1, nlev):
        assert c["nu"][d] == c["nu"][d - 1] - c["nf"][d]
        assert c["mu"][d] == c["mu"][d - 1] - c["mf"][d]
    assert np.all(c["ebu"] <= c["mu"])
    assert np.all(c["ebc"] <= c["ebu"])
    assert c["mu"][0] == cols.shape[0] - c["mf"][0]


def test_level_counters_component_scope():
    # two components: a path 0-1-2 (root 0) and a triangle 3-4-5.  Bottom-up
    # at level d over the whole swept set also reads every triangle row in
    # full (2 entries each, no hit possible); the component-scoped count
    # leaves those out.
    edges = [(0, 1), (1, 2), (3, 4), (4, 5), (3, 5)]
    off, cols = csr_of(6, edges)
    depth, _, nlev = oracle.bfs(off, cols, 0)
    c = oracle.level_counters(off, cols, depth)
    assert nlev == 3
    # level 0: 1 scans 2 then meets 0 (2 entries); 2's only neighbour 1 is not
    # in F_0 (1)
    assert c["ebc"].tolist() == [3, 1, 0]
    assert (c["ebu"] - c["ebc"]).tolist() == [6, 6, 6]


def test_heuristic_schedule_hand_cases():
    # TD until m_f * alpha > m_u, BU until n_f * beta < n and shrinking
    nf = [1, 10, 500, 400, 20, 2]
    mf = [5, 100, 5000, 800, 40, 3]
    mu = [9995, 9895, 4895, 4095, 4055, 4052]
    n = 1000
    assert oracle.heuristic_schedule(nf, mf, mu, n, 14, 24).tolist() == [0, 0, 1, 1, 0, 0]
    # alpha large: switch at level 1 already (100*100 > 9895)
    assert oracle.heuristic_schedule(nf, mf, mu, n, 100, 24).tolist() == [0, 1, 1, 1, 0, 0]
    # beta = 1: level 3 already switches back (400 * 1 < 1000 and 400 < 500)
    assert oracle.heuristic_schedule(nf, mf, mu, n, 14, 1).tolist() == [0, 0, 1, 0, 0, 0]
    # frontier not shrinking keeps bottom-up
    nf2 = [1, 10, 500, 600, 700, 2]
    assert oracle.heuristic_schedule(nf2, mf, mu, 100000, 14, 24).tolist() == [0, 0, 1, 1, 1, 0]


def test_component_edges_closed_form():
    k = 7
    edges = [(a, b) for a in range(k) for b in range(a + 1, k)]
    off, cols = csr_of(k + 3, edges + [(k, k + 1)])
    depth, _, _ = oracle.bfs(off, cols, 0)
    assert oracle.component_edges(off, depth) == k * (k - 1) // 2


# --------------------------------------------------------------------------
# partial RCM (section 4.6), under the reading stated in the fixture file

PARTIAL = os.path.join(os.path.dirname(__file__), "golden", "partial_rcm_worked_examples.json")
with open(PARTIAL) as f:
    PARTIAL_CASES = json.load(f)["cases"]


@pytest.mark.parametrize("case", PARTIAL_CASES, ids=[c["name"] for c in PARTIAL_CASES])
def test_partial_rcm_worked_example(case):
    off, cols = csr_of(case["n"], case["edges"])
    for keep, want in case["iperm_by_keep"].items():
        perm, iperm, nplus = oracle.rcm_partial(off, cols, int(keep))
        assert nplus == case["nplus"]
        assert iperm.tolist() == want, keep
        assert np.array_equal(perm[iperm], np.arange(case["n"]))
    # keep = n+ reproduces the full Algorithm 3 worked result
    full = oracle.rcm(off, cols)[1]
    assert full.tolist() == case["iperm_by_keep"][str(case["nplus"])]


def partial_from_full(off, iperm_full, nplus, keep):
    """The same order built from the full RCM: the reversed Cuthill-McKee
    sequence holds sequence position j at label n+ - 1 - j, so its first
    `keep` positions are the full labels [n+ - keep, n+)."""
    head = list(iperm_full[nplus - keep:nplus])
    rest = sorted(set(int(v) for v in np.flatnonzero(np.diff(off) > 0)) - set(head))
    iso = [int(v) for v in np.flatnonzero(np.diff(off) == 0)]
    return head + rest + iso


@pytest.mark.parametrize("seed", range(12))
def test_partial_rcm_is_a_prefix_of_the_full_sequence(seed):
    rng = random.Random(3000 + seed)
    n = rng.randint(2, 80)
    (off, cols), _ = random_graph(rng, n, rng.choice([0.02, 0.05, 0.1, 0.3]), rng.randint(0, 5))
    _, iperm_full, nplus = oracle.rcm(off, cols)
    for keep in sorted({0, 1, nplus // 3, nplus // 2, nplus - 1, nplus, nplus + 7}):
        keep = max(0, keep)
        perm, iperm, np_ = oracle.rcm_partial(off, cols, keep)
        assert np_ == nplus
        assert iperm.tolist() == partial_from_full(off, iperm_full, nplus, min(keep, nplus))
    # keep = 0: only the isolated vertices move (to the end)
    iperm0 = oracle.rcm_partial(off, cols, 0)[1]
    deg = np.diff(off)
    assert iperm0.tolist() == (np.flatnonzero(deg > 0).tolist() + np.flatnonzero(deg == 0).tolist())


def test_partial_rcm_kronecker_prefix():
    off, cols = graphgen.kronecker_csr(11, 16, 9)
    _, iperm_full, nplus = oracle.rcm(off, cols)
    for p in (0.1, 0.5, 0.9):
        keep = oracle.keep_for_ratio(p, nplus)
        assert keep - 1 < p * nplus <= keep
        iperm = oracle.rcm_partial(off, cols, keep)[1]
        assert iperm.tolist() == partial_from_full(off, iperm_full, nplus, keep)
    assert oracle.keep_for_ratio(1.0, nplus) == nplus
    assert oracle.keep_for_ratio(0.0, nplus) == 0
