"""Partial RCM (section 4.6) through the C ABI against the oracle: the
permutation bit for bit for several cut-offs, then searches on the partially
relabelled graph (single root in every direction mode, batch rows, the
on-device certificate) against the oracle's search under the same labels."""
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


def graphs():
    rng = random.Random(21)
    gs = [("mixed", csr_of(7, [(1, 4), (4, 6), (6, 1), (6, 2), (0, 5)])),
          ("pairs_iso", csr_of(20, [(2 * i, 2 * i + 1) for i in range(7)])),
          ("longpath", csr_of(3000, [(i, i + 1) for i in range(2999)]))]
    for t in range(3):
        n = rng.randint(50, 400)
        p = rng.choice([0.005, 0.01, 0.03])
        edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
        gs.append(("er%d" % t, csr_of(n + rng.randint(0, 5), edges)))
    gs.append(("kron12", graphgen.kronecker_csr(12, 16, 1016)))
    gs.append(("chunglu", graphgen.chung_lu_csr(20000, 1000, seed=6, max_deg=2000.0,
                                                mean_deg=10.0)))
    return gs


GRAPHS = graphs()
DIRS = ("heuristic", "td", "bu")


def keeps(nplus):
    return sorted({0, 1, nplus // 3, nplus // 2, nplus - 1, nplus})


@pytest.mark.parametrize("name,g", GRAPHS, ids=[x[0] for x in GRAPHS])
def test_partial_permutation_and_searches(rb, name, g):
    off, cols = g
    nplus = int((np.diff(off) > 0).sum())
    roots = graphgen.sample_roots(off, 3, 5)
    for keep in keeps(nplus):
        G = rb.Graph(off, cols)
        perm_t, _ = G.rcm_reorder(keep=keep)
        perm = perm_t.cpu().numpy()
        perm_o, iperm_o, np_o = oracle.rcm_partial(off, cols, keep)
        assert np.array_equal(perm, perm_o), keep
        assert np.array_equal(G.iperm().cpu().numpy(), iperm_o), keep
        info = G.info()
        assert info["n_plus"] == np_o and info["rcm_keep"] == keep and info["reordered"] == 1
        for r in roots:
            d_o, p_o, _ = oracle.bfs(off, cols, r, perm_o)
            for mode in DIRS:
                dirc = {"heuristic": rb.DIR_HEURISTIC, "td": rb.DIR_TD_ONLY,
                        "bu": rb.DIR_BU_ONLY}[mode]
                d, p = G.bfs(r, opts=rb.make_opts(dirc))
                assert np.array_equal(d.cpu().numpy(), d_o), (keep, r, mode)
                assert np.array_equal(p.cpu().numpy(), p_o), (keep, r, mode)
                assert G.certify(r, d, p) == 0
        dB, pB = G.bfs_batch(roots)
        for j, r in enumerate(roots):
            d_o, p_o, _ = oracle.bfs(off, cols, r, perm_o)
            assert np.array_equal(dB[j].cpu().numpy(), d_o)
            assert np.array_equal(pB[j].cpu().numpy(), p_o)


def test_ratio_and_second_call(rb):
    off, cols = GRAPHS[-2][1]
    nplus = int((np.diff(off) > 0).sum())
    G = rb.Graph(off, cols)
    perm_t, ms = G.rcm_reorder(partial=0.25)
    keep = oracle.keep_for_ratio(0.25, nplus)
    assert G.info()["rcm_keep"] == keep
    assert np.array_equal(perm_t.cpu().numpy(), oracle.rcm_partial(off, cols, keep)[0])
    # a second reorder of either kind changes nothing
    perm2, ms2 = G.rcm_reorder()
    assert ms2 == 0.0 and torch.equal(perm2, perm_t)
    perm3, _ = G.rcm_reorder(keep=nplus)
    assert torch.equal(perm3, perm_t)


def test_full_keep_equals_rcm(rb):
    off, cols = GRAPHS[-1][1]
    nplus = int((np.diff(off) > 0).sum())
    G1, G2, G3 = rb.Graph(off, cols), rb.Graph(off, cols), rb.Graph(off, cols)
    p1, _ = G1.rcm_reorder()
    p2, _ = G2.rcm_reorder(keep=nplus + 5)
    p3, _ = G3.rcm_reorder(keep=-1)
    assert torch.equal(p1, p2) and torch.equal(p1, p3)
    assert G1.info()["rcm_keep"] == nplus == G2.info()["rcm_keep"]
