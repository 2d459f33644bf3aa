"""GPU parity of the batched searches: the 64-root bit-parallel search
(rbfs_bfs_batch) and the multi-graph search (rbfs_bfs_multi) must give, row
for row, exactly the single-root result of the oracle."""
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


def check_rows(off, cols, roots, ell, depth, parent):
    d = depth.cpu().numpy()
    p = parent.cpu().numpy()
    for j, r in enumerate(roots):
        d_o, p_o, _ = oracle.bfs(off, cols, r, ell)
        assert np.array_equal(d[j], d_o), ("depth", j, r)
        assert np.array_equal(p[j], p_o), ("parent", j, r)


def graph_cases():
    rng = random.Random(11)
    cases = []
    n = 300
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.01]
    cases.append(("er300", csr_of(n + 7, edges)))
    cases.append(("pairs", csr_of(40, [(2 * i, 2 * i + 1) for i in range(15)])))
    cases.append(("path", csr_of(500, [(i, i + 1) for i in range(499)])))
    hub = [(0, i) for i in range(1, 3000)] + [(i, i + 1) for i in range(1, 2999, 3)]
    cases.append(("hub", csr_of(3001, hub)))
    cases.append(("kron12", graphgen.kronecker_csr(12, 16, 5)))
    return cases


CASES = graph_cases()


@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("name,g", CASES, ids=[c[0] for c in CASES])
def test_batch_matches_oracle(rb, name, g, reorder):
    off, cols = g
    n = off.shape[0] - 1
    G = rb.Graph(off, cols)
    ell = None
    if reorder:
        perm, _ = G.rcm_reorder()
        ell = perm.cpu().numpy()
    rng = random.Random(n)
    roots = [rng.randrange(n) for _ in range(64)]  # duplicates and isolated roots allowed
    roots[3] = roots[7]
    for mode in (rb.DIR_HEURISTIC, rb.DIR_TD_ONLY, rb.DIR_BU_ONLY):
        d, p = G.bfs_batch(roots, opts=rb.make_opts(mode))
        check_rows(off, cols, roots, ell, d, p)


def test_batch_sizes(rb):
    off, cols = graphgen.kronecker_csr(13, 16, 8)
    G = rb.Graph(off, cols)
    perm, _ = G.rcm_reorder()
    ell = perm.cpu().numpy()
    for k in (1, 5, 64, 100):
        roots = graphgen.sample_roots(off, k, 7 + k, distinct=False) if k <= 64 else \
            graphgen.sample_roots(off, 64, 7) + graphgen.sample_roots(off, k - 64, 9)
        d, p, st = G.bfs_batch(roots, stats=True)
        assert st["status"] == 0
        check_rows(off, cols, roots, ell, d, p)


def test_batch_equals_single_root(rb):
    off, cols = graphgen.kronecker_csr(15, 16, 3)
    G = rb.Graph(off, cols)
    G.rcm_reorder()
    roots = graphgen.sample_roots(off, 64, 7)
    d, p = G.bfs_batch(roots)
    for j in (0, 17, 63):
        d1, p1 = G.bfs(roots[j])
        assert torch.equal(d[j], d1) and torch.equal(p[j], p1)


def multi_graphs():
    gs = []
    for g in range(7):
        scale = 8 + (g % 5)
        gs.append(graphgen.kronecker_csr(scale, 16, 3000 + g))
    gs.append(csr_of(50, [(2 * i, 2 * i + 1) for i in range(10)]))
    return gs


@pytest.mark.parametrize("reorder", [False, True])
def test_multi_matches_oracle(rb, reorder):
    csrs = multi_graphs()
    Gs = [rb.Graph(o, c) for o, c in csrs]
    ells = []
    for G in Gs:
        if reorder:
            perm, _ = G.rcm_reorder()
            ells.append(perm.cpu().numpy())
        else:
            ells.append(None)
    M = rb.MultiGraph(Gs)
    k = 16
    total = M.out_size(k)
    depth = torch.empty(total, dtype=torch.int32, device="cuda")
    parent = torch.empty(total, dtype=torch.int32, device="cuda")
    for rep in range(3):  # first call captures, later calls replay the captured graph
        roots = []
        for gi, (o, c) in enumerate(csrs):
            rng = random.Random(100 * rep + gi)
            n = o.shape[0] - 1
            roots.append([rng.randrange(n) for _ in range(k)])
        outs = M.bfs(roots, depth=depth, parent=parent)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        for gi, (o, c) in enumerate(csrs):
            check_rows(o, c, roots[gi], ells[gi], outs[gi][0], outs[gi][1])


def test_multi_rejects_mixed_state(rb):
    a = rb.Graph(*graphgen.kronecker_csr(8, 16, 1))
    b = rb.Graph(*graphgen.kronecker_csr(8, 16, 2))
    b.rcm_reorder()
    with pytest.raises(rb.RbfsError):
        rb.MultiGraph([a, b])
