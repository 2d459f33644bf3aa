"""rbfs_certify_noalloc (static device scratch, no allocation) against
rbfs_certify, called through the C ABI: two calls in a row on each path, the
second on a smaller graph, on correct search results and on copies with
planted mistakes, in both output spaces; plus the size limit."""
import ctypes

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_10026_amd as rb
    return rb


def _cert(rb, name, G, root, d, p, space):
    res = ctypes.c_int32(7)
    rc = getattr(rb.lib(), name)(G.handle, int(root), ctypes.c_void_p(d.data_ptr()),
                                 ctypes.c_void_p(p.data_ptr()), int(space),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                 ctypes.byref(res))
    assert rc == 0, rb.lib().rbfs_last_error().decode()
    return res.value


def _cases(rb, G, off, space, seed):
    """(root, depth, parent) triples: search results and planted mistakes."""
    rng = np.random.default_rng(seed)
    out = []
    for r in graphgen.sample_roots(off, 2, seed):
        d, p = G.bfs(r, opts=rb.make_opts(output_space=space))
        out.append((r, d, p))
        for _ in range(6):
            d2, p2 = d.clone(), p.clone()
            v = int(rng.integers(0, G.n))
            kind = int(rng.integers(0, 3))
            if kind == 0:
                d2[v] += 1
            elif kind == 1:
                p2[v] = int(rng.integers(0, G.n))
            else:
                d2[v] = -1
            out.append((r, d2, p2))
    return out


def test_noalloc_certificate_equals_allocating_one(rb):
    print("no-alloc certificate: scale 17 then scale 12, both output spaces", flush=True)
    graphs = []
    for scale, seed in ((17, 917), (12, 912)):  # second call: smaller input
        off, cols = graphgen.kronecker_csr(scale, 16, seed)
        G = rb.Graph(off, cols)
        G.rcm_reorder()
        graphs.append((G, off))
    assert int(np.diff(graphs[0][1]).max()) > 4096  # long rows take the chunked path
    codes = set()
    for G, off in graphs:
        for space in (rb.OUT_ORIGINAL, rb.OUT_INTERNAL):
            for root, d, p in _cases(rb, G, off, space, 5 + space):
                a = _cert(rb, "rbfs_certify", G, root, d, p, space)
                b = _cert(rb, "rbfs_certify_noalloc", G, root, d, p, space)
                assert a == b
                codes.add(a)
    assert 0 in codes and len(codes) > 1


def test_noalloc_certificate_refuses_oversize_graph(rb):
    n = 17 << 20  # edgeless: the gathered depths alone exceed 64 MiB
    off = np.zeros(n + 1, np.int64)
    G = rb.Graph(off, np.zeros(0, np.int32))
    G.rcm_reorder(want_perm=False)
    d, p = G.bfs(3)
    res = ctypes.c_int32(0)
    rc = rb.lib().rbfs_certify_noalloc(G.handle, 3, ctypes.c_void_p(d.data_ptr()),
                                       ctypes.c_void_p(p.data_ptr()), rb.OUT_ORIGINAL,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                       ctypes.byref(res))
    assert rc == -2
    assert "static buffer" in rb.lib().rbfs_last_error().decode()
    assert _cert(rb, "rbfs_certify", G, 3, d, p, rb.OUT_ORIGINAL) == 0
    di, pi = G.bfs(3, opts=rb.make_opts(output_space=rb.OUT_INTERNAL))
    # internal outputs need no gathered depths: within the limit
    assert _cert(rb, "rbfs_certify_noalloc", G, 3, di, pi, rb.OUT_INTERNAL) == 0
