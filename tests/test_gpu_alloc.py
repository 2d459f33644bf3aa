"""GPU tests of the allocator hook: with torch's caching allocator installed
(the binding's default) the library's device memory is counted by torch and
returned when the handles close; the allocator cannot change while handles
exist; results are the oracle's with either allocator."""
import gc

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


def check_searches(rb, G, off, cols, roots, perm):
    for r in roots:
        d, p = G.bfs(r)
        d_o, p_o, _ = oracle.bfs(off, cols, r, perm)
        assert np.array_equal(d.cpu().numpy(), d_o) and np.array_equal(p.cpu().numpy(), p_o)
    d, p = G.bfs_batch(roots)
    for j, r in enumerate(roots):
        d_o, p_o, _ = oracle.bfs(off, cols, r, perm)
        assert np.array_equal(d[j].cpu().numpy(), d_o) and np.array_equal(p[j].cpu().numpy(), p_o)


@pytest.mark.parametrize("kind", ["torch", "hip"])
def test_allocator_memory_and_results(rb, kind):
    off, cols = graphgen.kronecker_csr(13, 16, 99)
    roots = list(graphgen.sample_roots(off, 4, 5))
    gc.collect()  # handles of earlier tests must be closed before switching
    rb.set_allocator(kind)
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        G = rb.Graph(off, cols)
        perm, _ = G.rcm_reorder()
        perm = perm.cpu().numpy()
        torch.cuda.synchronize()
        after_create = torch.cuda.memory_allocated()
        check_searches(rb, G, off, cols, roots, perm)
        graph_bytes = 8 * (off.shape[0]) + 4 * cols.shape[0]
        if kind == "torch":
            # CSR, perm, iperm and the search workspaces are torch allocations
            assert after_create - base >= graph_bytes
        with pytest.raises(rb.RbfsError) as e:
            rb.set_allocator("hip" if kind == "torch" else "torch")
        assert e.value.code == -5
        M = rb.MultiGraph([G])
        outs = M.bfs([roots])
        d_o, p_o, _ = oracle.bfs(off, cols, roots[0], perm)
        assert np.array_equal(outs[0][0][0].cpu().numpy(), d_o)
        M.close()
        G.close()
        del M, G
        torch.cuda.synchronize()
        # everything the library took is back (outputs of the searches are
        # torch tensors that were freed with their Python objects)
        assert torch.cuda.memory_allocated() <= base + (1 << 20)
    finally:
        rb.set_allocator("torch")
