"""Parity at the benchmark sizes, in the launch configuration the benchmark
times.  Scale 22: the whole RCM permutation and every output of sampled
roots bit-exact against the oracle.  Scale 26, scale 24 (64-root batch) and
the 52.5M-vertex Chung-Lu graph: the O(nnz) certificates (the RCM
certificate pins the whole permutation to Algorithm 3; the BFS certificate
pins depth and the largest-label parent of every vertex), plus oracle depth
for a sampled root.  Graphs come from the device generator, which equals the
host generator bit for bit (test_gpu_bfs.py)."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_10026_amd as rb
    return rb


def host(t):
    return t.cpu().numpy()


@pytest.mark.timeout(900)
def test_scale22_bit_exact(rb):
    off_d, cols_d = graphgen.kronecker_csr_device(22, 16, 1022)
    off, cols = host(off_d), host(cols_d)
    roots = graphgen.sample_roots(off, 64, 7)
    G = rb.Graph(off_d, cols_d)
    del off_d, cols_d
    perm_t, _ = G.rcm_reorder()
    perm = host(perm_t)
    perm_o, _, _ = oracle.rcm(off, cols)
    assert np.array_equal(perm, perm_o)
    for r in roots[:6]:
        d, p = G.bfs(r)
        d_o, p_o, _ = oracle.bfs(off, cols, r, perm_o)
        assert np.array_equal(host(d), d_o)
        assert np.array_equal(host(p), p_o)
    dB, pB = G.bfs_batch(roots)
    for j in (0, 31, 63):
        d_o, p_o, _ = oracle.bfs(off, cols, roots[j], perm_o)
        assert np.array_equal(host(dB[j]), d_o)
        assert np.array_equal(host(pB[j]), p_o)


def certify_graph(rb, G, off, cols, roots, n_bfs_cert, n_depth):
    perm_t, rcm_ms = G.rcm_reorder()
    perm = host(perm_t)
    assert oracle.certify_rcm(off, cols, perm) == 0
    for i, r in enumerate(roots[:n_bfs_cert]):
        d, p = G.bfs(r)
        d, p = host(d), host(p)
        assert oracle.certify_bfs(off, cols, r, d, p, perm) == 0
        if i < n_depth:
            d_o, _, _ = oracle.bfs(off, cols, r)  # depth is label independent
            assert np.array_equal(d, d_o)
    return perm


@pytest.mark.timeout(1200)
def test_scale26_certified(rb):
    off_d, cols_d = graphgen.kronecker_csr_device(26, 16, 1026)
    off, cols = host(off_d), host(cols_d)
    roots = graphgen.sample_roots(off, 64, 7)
    G = rb.Graph(off_d, cols_d)
    del off_d, cols_d
    torch.cuda.empty_cache()
    certify_graph(rb, G, off, cols, roots, n_bfs_cert=2, n_depth=1)
    # every root the benchmark times, through the on-device certificate
    # (itself checked against the oracle's in test_gpu_certify.py)
    for r in roots:
        d, p = G.bfs(r)
        assert G.certify(r, d, p) == 0, r


@pytest.mark.timeout(1200)
def test_scale24_batch_certified(rb):
    off_d, cols_d = graphgen.kronecker_csr_device(24, 16, 1024)
    off, cols = host(off_d), host(cols_d)
    roots = graphgen.sample_roots(off, 64, 7)
    G = rb.Graph(off_d, cols_d)
    del off_d, cols_d
    perm_t, _ = G.rcm_reorder()
    perm = host(perm_t)
    assert oracle.certify_rcm(off, cols, perm) == 0
    dB, pB = G.bfs_batch(roots)
    for j in (0, 21, 42, 63):
        d, p = host(dB[j]), host(pB[j])
        assert oracle.certify_bfs(off, cols, roots[j], d, p, perm) == 0
        d1, p1 = G.bfs(roots[j])
        assert np.array_equal(host(d1), d) and np.array_equal(host(p1), p)
    for j in range(64):
        assert G.certify(roots[j], dB[j], pB[j]) == 0, j


@pytest.mark.timeout(1200)
def test_chung_lu_50m_certified(rb):
    off_d, cols_d = graphgen.chung_lu_csr_device(50_000_000, 2_500_000, seed=4000)
    off, cols = host(off_d), host(cols_d)
    roots = graphgen.sample_roots(off, 64, 7)
    G = rb.Graph(off_d, cols_d)
    del off_d, cols_d
    torch.cuda.empty_cache()
    certify_graph(rb, G, off, cols, roots, n_bfs_cert=1, n_depth=1)


@pytest.mark.timeout(900)
def test_multi_graph_batch_32_graphs(rb):
    """32 Kronecker graphs of scales 12..20, 16 roots each, one captured
    launch; sampled graphs checked against the oracle row by row."""
    csrs, Gs, roots, perms = [], [], [], []
    for g in range(32):
        s = 12 + (g % 9)
        off, cols = graphgen.kronecker_csr(s, 16, 3000 + g)
        G = rb.Graph(off, cols)
        perm, _ = G.rcm_reorder()
        csrs.append((off, cols))
        Gs.append(G)
        perms.append(host(perm))
        roots.append(graphgen.sample_roots(off, 16, 7))
    M = rb.MultiGraph(Gs)
    outs = M.bfs(roots)
    for g in (0, 5, 8, 17, 31):
        off, cols = csrs[g]
        d, p = host(outs[g][0]), host(outs[g][1])
        for j in (0, 7, 15):
            d_o, p_o, _ = oracle.bfs(off, cols, roots[g][j], perms[g])
            assert np.array_equal(d[j], d_o) and np.array_equal(p[j], p_o)
