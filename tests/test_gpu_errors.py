"""GPU tests of the library's error paths, each forced from the host so that
every kernel exits normally: the sticky device status that rbfs_graph_check
reports for single-root searches, and the lifetime rule between a
multi-graph handle and its member graphs."""
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


def test_status_of_an_earlier_search_reaches_the_check(rb):
    """A search whose grid barrier is given no time to wait stops with the
    time-out status; the searches after it succeed, and the next check still
    reports that status once."""
    off, cols = graphgen.kronecker_csr(12, 16, 77)
    G = rb.Graph(off, cols)
    perm_t, _ = G.rcm_reorder()
    perm = perm_t.cpu().numpy()
    roots = graphgen.sample_roots(off, 3, 7)
    G.check()  # nothing raised yet
    G.bfs(roots[0], opts=rb.make_opts(zero_wait=True))  # no stats: returns OK
    for r in roots[1:]:
        d, p = G.bfs(r)
        d_o, p_o, _ = oracle.bfs(off, cols, r, perm)
        assert np.array_equal(d.cpu().numpy(), d_o)
        assert np.array_equal(p.cpu().numpy(), p_o)
    with pytest.raises(rb.RbfsError) as ei:
        G.check()
    assert ei.value.code == -4
    G.check()  # reported once
    with pytest.raises(rb.RbfsError):
        G.bfs(roots[0], opts=rb.make_opts(zero_wait=True), stats=True)
    d, p = G.bfs(roots[0])
    d_o, p_o, _ = oracle.bfs(off, cols, roots[0], perm)
    assert np.array_equal(d.cpu().numpy(), d_o) and np.array_equal(p.cpu().numpy(), p_o)


def test_multi_graph_pins_its_members(rb):
    """While a multi-graph handle exists, its members can be neither
    relabelled nor destroyed; afterwards both work."""
    graphs, csr = [], []
    for s in (9, 10):
        off, cols = graphgen.kronecker_csr(s, 16, 500 + s)
        csr.append((off, cols))
        graphs.append(rb.Graph(off, cols))
    M = rb.MultiGraph(graphs)
    roots = [graphgen.sample_roots(off, 2, 3) for off, _ in csr]
    out = M.bfs(roots)
    for (off, cols), (dB, pB), rs in zip(csr, out, roots):
        for j, r in enumerate(rs):
            d_o, p_o, _ = oracle.bfs(off, cols, r)
            assert np.array_equal(dB[j].cpu().numpy(), d_o)
            assert np.array_equal(pB[j].cpu().numpy(), p_o)
    with pytest.raises(rb.RbfsError) as ei:
        graphs[0].rcm_reorder()
    assert ei.value.code == -5
    with pytest.raises(rb.RbfsError) as ei:
        graphs[1].close()
    assert ei.value.code == -5
    out = M.bfs(roots)  # the members are untouched
    for (off, cols), (dB, pB), rs in zip(csr, out, roots):
        d_o, p_o, _ = oracle.bfs(off, cols, rs[0])
        assert np.array_equal(dB[0].cpu().numpy(), d_o)
    M.close()
    perm_t, _ = graphs[0].rcm_reorder()
    off, cols = csr[0]
    d, p = graphs[0].bfs(roots[0][0])
    d_o, p_o, _ = oracle.bfs(off, cols, roots[0][0], perm_t.cpu().numpy())
    assert np.array_equal(p.cpu().numpy(), p_o)
    for g in graphs:
        g.close()
