"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference for RCM relabelling (Algorithm 3,
and the partial RCM of section 4.6) and the BFS result (Algorithms 1-2,
predecessor map with the largest-label parent rule), with per-level
counters, the alpha/beta direction rule and O(nnz) certificates.  Only tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the GPU library never does.

The arithmetic lives in oracle.c (built into liboracle.so with gcc); this
module only marshals numpy arrays.  The fp64 MLP reference for the learned
direction switch is in oracle/mlp.py.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        c = ctypes
        P = c.c_void_p
        L.orc_bandwidth.restype = c.c_int64
        L.orc_bandwidth.argtypes = [c.c_int64, P, P, P]
        L.orc_canonical_csr.restype = c.c_int64
        L.orc_canonical_csr.argtypes = [c.c_int64, c.c_int64, P, P, P, P]
        L.orc_rcm.restype = c.c_int64
        L.orc_rcm.argtypes = [c.c_int64, P, P, P, P]
        L.orc_rcm_partial.restype = c.c_int64
        L.orc_rcm_partial.argtypes = [c.c_int64, P, P, c.c_int64, P, P]
        L.orc_bfs.restype = c.c_int32
        L.orc_bfs.argtypes = [c.c_int64, P, P, c.c_int32, P, P, P]
        L.orc_level_counters.restype = None
        L.orc_level_counters.argtypes = [c.c_int64, P, P, P, c.c_int64, P, c.c_int32,
                                         P, P, P, P, P, P]
        L.orc_heuristic_schedule.restype = None
        L.orc_heuristic_schedule.argtypes = [c.c_int32, P, P, P, c.c_int64, c.c_int64,
                                             c.c_int64, P]
        L.orc_certify_bfs.restype = c.c_int32
        L.orc_certify_bfs.argtypes = [c.c_int64, P, P, c.c_int32, P, P, P]
        L.orc_certify_rcm.restype = c.c_int32
        L.orc_certify_rcm.argtypes = [c.c_int64, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(off, cols):
    off = np.ascontiguousarray(off, np.int64)
    cols = np.ascontiguousarray(cols, np.int32)
    if cols.size == 0:
        cols = np.zeros(1, np.int32)
    return off, cols, off.shape[0] - 1


def _opt_i32(a):
    return None if a is None else np.ascontiguousarray(a, np.int32)


def bandwidth(off, cols, ell=None):
    """Eq. 1 in labelling ell (identity when None)."""
    off, cols, n = _csr(off, cols)
    ell = _opt_i32(ell)
    return int(lib().orc_bandwidth(n, _p(off), _p(cols), _p(ell)))


def canonical_csr(n, src, dst):
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    m = src.shape[0]
    off = np.empty(n + 1, np.int64)
    cols = np.empty(max(1, 2 * m), np.int32)
    nnz = lib().orc_canonical_csr(n, m, _p(src), _p(dst), _p(off), _p(cols))
    return off, cols[:nnz].copy()


def rcm(off, cols):
    """Algorithm 3.  Returns (perm, iperm, nplus): perm[v] = new label of v,
    iperm[k] = vertex with label k, nplus = number of non-isolated vertices."""
    off, cols, n = _csr(off, cols)
    P = np.empty(n, np.int32)
    perm = np.empty(n, np.int32)
    nplus = lib().orc_rcm(n, _p(off), _p(cols), _p(P), _p(perm))
    return perm, P, int(nplus)


def rcm_partial(off, cols, keep):
    """Partial RCM (section 4.6): the first `keep` vertices of Algorithm 3's
    Cuthill-McKee sequence reversed into labels [0, keep), the remaining
    non-isolated vertices after them in increasing id, isolated vertices
    last.  Returns (perm, iperm, nplus)."""
    off, cols, n = _csr(off, cols)
    P = np.empty(n, np.int32)
    perm = np.empty(n, np.int32)
    nplus = lib().orc_rcm_partial(n, _p(off), _p(cols), int(keep), _p(P), _p(perm))
    return perm, P, int(nplus)


def keep_for_ratio(p, nplus):
    """Vertices a p-partial RCM reorders: ceil(p * n+), clamped to [0, n+]."""
    import math
    return max(0, min(nplus, math.ceil(p * nplus)))


def bfs(off, cols, root, ell=None):
    """(depth, parent, nlevels) from root; parent rule: largest ell label."""
    off, cols, n = _csr(off, cols)
    ell = _opt_i32(ell)
    depth = np.empty(n, np.int32)
    parent = np.empty(n, np.int32)
    nlev = lib().orc_bfs(n, _p(off), _p(cols), int(root), _p(ell), _p(depth), _p(parent))
    return depth, parent, int(nlev)


def level_counters(off, cols, depth, ell=None, n_sweep=None):
    """Dict of per-level arrays nf, mf, nu, mu, ebu, ebc (see oracle.c)."""
    off, cols, n = _csr(off, cols)
    ell = _opt_i32(ell)
    depth = np.ascontiguousarray(depth, np.int32)
    nlev = int(depth.max()) + 1 if depth.size else 0
    if n_sweep is None:
        n_sweep = n
    out = {k: np.zeros(max(1, nlev), np.int64) for k in ("nf", "mf", "nu", "mu", "ebu", "ebc")}
    lib().orc_level_counters(n, _p(off), _p(cols), _p(ell), int(n_sweep), _p(depth), nlev,
                             _p(out["nf"]), _p(out["mf"]), _p(out["nu"]), _p(out["mu"]),
                             _p(out["ebu"]), _p(out["ebc"]))
    return {k: v[:nlev] for k, v in out.items()}


def heuristic_schedule(nf, mf, mu, n_sweep, alpha, beta):
    """Direction per level (0 top-down, 1 bottom-up)."""
    nf = np.ascontiguousarray(nf, np.int64)
    mf = np.ascontiguousarray(mf, np.int64)
    mu = np.ascontiguousarray(mu, np.int64)
    nlev = nf.shape[0]
    out = np.zeros(max(1, nlev), np.int8)
    lib().orc_heuristic_schedule(nlev, _p(nf), _p(mf), _p(mu), int(n_sweep), int(alpha),
                                 int(beta), _p(out))
    return out[:nlev]


def certify_bfs(off, cols, root, depth, parent, ell=None):
    off, cols, n = _csr(off, cols)
    ell = _opt_i32(ell)
    depth = np.ascontiguousarray(depth, np.int32)
    parent = np.ascontiguousarray(parent, np.int32)
    return int(lib().orc_certify_bfs(n, _p(off), _p(cols), int(root), _p(ell), _p(depth),
                                     _p(parent)))


def certify_rcm(off, cols, perm):
    off, cols, n = _csr(off, cols)
    perm = np.ascontiguousarray(perm, np.int32)
    return int(lib().orc_certify_rcm(n, _p(off), _p(cols), _p(perm)))


def component_edges(off, depth):
    """TEPS numerator: undirected edges in the reached component,
    half the degree sum over reached vertices."""
    deg = np.diff(np.asarray(off, np.int64))
    return int(deg[np.asarray(depth) >= 0].sum() // 2)
