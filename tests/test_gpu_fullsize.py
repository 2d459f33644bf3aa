"""Parity at the benchmark sizes, in the launch configuration the benchmark
times.  Scale 22: the whole RCM permutation and every output of all 64
roots bit-exact against the oracle (single-root, batched, and 16 roots in
learned mode).  Scale 26 and the 52.5M-vertex Chung-Lu graph: the RCM
certificate (which pins the whole permutation to Algorithm 3), every output
of the 64 roots -- plain, learned with a network trained on small Kronecker
graphs (not retrained), and the 64-root batch -- through the on-device
certificate, and a sample of each through the oracle's O(nnz) certificate,
which pins depth and the largest-label parent of every vertex.  Scale 24:
the 64-root batch.  Graphs come from the device generator, which equals the
host generator bit for bit (test_gpu_bfs.py)."""
import numpy as np
import pytest

import graphgen
import oracle
from helpers import pmap, train_kronecker_blob

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_10026_amd as rb
    return rb


def say(msg):
    print("  [fullsize] " + msg, flush=True)


def host(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def kron_blob(rb):
    """Switch network trained on small Kronecker graphs; the full-size tests
    evaluate it without retraining."""
    return train_kronecker_blob(rb)


@pytest.mark.timeout(900)
def test_scale22_bit_exact(rb, kron_blob):
    """Scale 22 (configuration of the plain benchmark, 64 roots): the whole
    permutation, and every output of every root bit-exact against the
    oracle -- single-root searches, the 64-root batch, and learned-switch
    searches of 16 roots."""
    off_d, cols_d = graphgen.kronecker_csr_device(22, 16, 1022)
    off, cols = host(off_d), host(cols_d)
    roots = graphgen.sample_roots(off, 64, 7)
    G = rb.Graph(off_d, cols_d)
    del off_d, cols_d
    perm_t, _ = G.rcm_reorder()
    perm = host(perm_t)
    say("scale 22: oracle RCM")
    perm_o, _, _ = oracle.rcm(off, cols)
    assert np.array_equal(perm, perm_o)
    say("scale 22: oracle BFS of 64 roots")
    ref = pmap(lambda r: oracle.bfs(off, cols, r, perm_o)[:2], roots)
    for r, (d_o, p_o) in zip(roots, ref):
        d, p = G.bfs(r)
        assert np.array_equal(host(d), d_o), r
        assert np.array_equal(host(p), p_o), r
    dB, pB = G.bfs_batch(roots)
    for j, (d_o, p_o) in enumerate(ref):
        assert np.array_equal(host(dB[j]), d_o), j
        assert np.array_equal(host(pB[j]), p_o), j
    rb.switch_load(kron_blob)
    learned = rb.make_opts(rb.DIR_LEARNED)
    for r, (d_o, p_o) in list(zip(roots, ref))[:16]:
        d, p = G.bfs(r, opts=learned)
        assert np.array_equal(host(d), d_o), r
        assert np.array_equal(host(p), p_o), r


def oracle_certified(off, cols, perm, pairs):
    """pairs: (root, depth, parent) on the host; True for each that the
    oracle's O(nnz) certificate accepts (run in parallel)."""
    return pmap(lambda t: oracle.certify_bfs(off, cols, t[0], t[1], t[2], perm), pairs)


def check_full_size(rb, G, off, cols, roots, blob, n_oracle):
    """RCM permutation certified by the oracle; then plain, learned (the
    given blob, no retraining) and 64-root batched searches: n_oracle
    outputs of each through the oracle's certificate (one also against the
    oracle's depth), every output through the on-device certificate."""
    perm_t, rcm_ms = G.rcm_reorder()
    perm = host(perm_t)
    say("RCM certificate (oracle)")
    assert oracle.certify_rcm(off, cols, perm) == 0
    say("plain and learned searches, on-device certificates")
    rb.switch_load(blob)
    learned = rb.make_opts(rb.DIR_LEARNED)
    sample = []
    for i, r in enumerate(roots):
        for opts in (None, learned):
            d, p = G.bfs(r, opts=opts)
            assert G.certify(r, d, p) == 0, (r, opts is not None)
            if i < n_oracle:
                sample.append((r, host(d), host(p)))
    dB, pB = G.bfs_batch(roots)
    for j, r in enumerate(roots):
        assert G.certify(r, dB[j], pB[j]) == 0, j
    step = max(1, len(roots) // n_oracle)
    for j in range(0, len(roots), step)[:n_oracle]:
        sample.append((roots[j], host(dB[j]), host(pB[j])))
    del dB, pB
    say("%d oracle certificates" % len(sample))
    assert oracle_certified(off, cols, perm, sample) == [0] * len(sample)
    say("oracle depth of one root")
    d_o, _, _ = oracle.bfs(off, cols, roots[0])  # depth does not depend on labels
    assert np.array_equal(sample[0][1], d_o)
    return perm


@pytest.mark.timeout(1200)
def test_scale26_certified(rb, kron_blob):
    say("scale 26: generate")
    off_d, cols_d = graphgen.kronecker_csr_device(26, 16, 1026)
    off, cols = host(off_d), host(cols_d)
    roots = graphgen.sample_roots(off, 64, 7)
    G = rb.Graph(off_d, cols_d)
    del off_d, cols_d
    torch.cuda.empty_cache()
    check_full_size(rb, G, off, cols, roots, kron_blob, n_oracle=4)


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
def test_chung_lu_50m_certified(rb, kron_blob):
    """The power-law configuration (52.5M vertices): plain, learned with the
    Kronecker-trained network (no retraining) and 64-root batched."""
    say("chung-lu: generate")
    off_d, cols_d = graphgen.chung_lu_csr_device(50_000_000, 2_500_000, seed=4000)
    off, cols = host(off_d), host(cols_d)
    roots = graphgen.sample_roots(off, 64, 7)
    G = rb.Graph(off_d, cols_d)
    del off_d, cols_d
    torch.cuda.empty_cache()
    check_full_size(rb, G, off, cols, roots, kron_blob, n_oracle=2)


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
