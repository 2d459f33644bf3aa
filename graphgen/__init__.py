"""Seeded synthetic graph inputs shared by the oracle tests and the GPU path.

This module generates inputs only; it holds no part of the RCM or BFS
arithmetic.  Workloads stand in for the Graph500 Kronecker graphs measured in
the paper (initiator (A, B, C, D) = (0.57, 0.19, 0.19, 0.05), N = 2^scale
vertices, M = edgefactor * N tuples with self-loops, duplicates and isolated
vertices; section 4, "Graph Instances") and, for the real-world social graphs
that are not available here, a Chung-Lu power-law graph with isolated
vertices added.

All draws are counter-based (splitmix64 mix of (seed, stream, counter)), so the
host and device generators give the same tuples and the same canonical CSR.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libgraphgen.so")
_lib = None

KRON_ABC = (0.57, 0.19, 0.19)
STREAM_ROOT = 4
MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _nthreads():
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        c = ctypes
        L.gg_host_draw.restype = c.c_uint64
        L.gg_host_draw.argtypes = [c.c_uint64, c.c_uint64, c.c_uint64]
        L.gg_perm_table.restype = c.c_int
        L.gg_perm_table.argtypes = [c.c_int64, c.c_uint64, c.c_void_p, c.c_int]
        L.gg_kron_tuples.restype = c.c_int
        L.gg_kron_tuples.argtypes = [c.c_int, c.c_uint64, c.c_double, c.c_double, c.c_double,
                                     c.c_int64, c.c_int64, c.c_void_p, c.c_void_p, c.c_int]
        L.gg_cl_cdf.restype = c.c_int
        L.gg_cl_cdf.argtypes = [c.c_int64, c.c_double, c.c_double, c.c_double, c.c_void_p,
                                c.c_void_p]
        L.gg_cl_tuples.restype = c.c_int
        L.gg_cl_tuples.argtypes = [c.c_int64, c.c_int64, c.c_uint64, c.c_void_p, c.c_int64,
                                   c.c_int64, c.c_void_p, c.c_void_p, c.c_int]
        L.gg_csr_from_tuples.restype = c.c_int64
        L.gg_csr_from_tuples.argtypes = [c.c_int64, c.c_int64, c.c_void_p, c.c_void_p,
                                         c.c_void_p, c.c_void_p, c.c_int]
        L.gg_dev_last_error.restype = c.c_char_p
        L.gg_dev_kron_csr.restype = c.c_int64
        L.gg_dev_kron_csr.argtypes = [c.c_int, c.c_int64, c.c_uint64, c.c_double, c.c_double,
                                      c.c_double, c.c_void_p, c.c_void_p, c.c_int64, c.c_void_p]
        L.gg_dev_kron_csr_ranges.restype = c.c_int64
        L.gg_dev_kron_csr_ranges.argtypes = [c.c_int, c.c_int64, c.c_uint64, c.c_double,
                                             c.c_double, c.c_double, c.c_void_p, c.c_void_p,
                                             c.c_int64, c.c_int64, c.c_void_p, c.c_void_p]
        L.gg_dev_kron_count_reached.restype = c.c_int64
        L.gg_dev_kron_count_reached.argtypes = [c.c_int, c.c_int64, c.c_uint64, c.c_double,
                                                c.c_double, c.c_double, c.c_void_p, c.c_void_p]
        L.gg_dev_cl_csr.restype = c.c_int64
        L.gg_dev_cl_csr.argtypes = [c.c_int64, c.c_int64, c.c_int64, c.c_uint64, c.c_void_p,
                                    c.c_void_p, c.c_void_p, c.c_int64, c.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# counter-based draws (pure Python copy, for root sampling and tests)

def mix64(z):
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def draw(seed, stream, ctr):
    key = mix64((seed ^ (stream * 0xD1B54A32D192ED03)) & MASK64)
    return mix64((key + (ctr + 1) * GAMMA) & MASK64)


# ----------------------------------------------------------------------------
# Kronecker

def kronecker_tuples(scale, edgefactor=16, seed=1, abc=KRON_ABC):
    n = 1 << scale
    m = edgefactor * n
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    rc = lib().gg_kron_tuples(scale, seed, abc[0], abc[1], abc[2], 0, m, _ptr(src), _ptr(dst),
                              _nthreads())
    if rc != 0:
        raise ValueError("gg_kron_tuples failed")
    return n, src, dst


def csr_from_tuples(n, src, dst):
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    m = src.shape[0]
    off = np.empty(n + 1, np.int64)
    cols = np.empty(max(1, 2 * m), np.int32)
    nnz = lib().gg_csr_from_tuples(n, m, _ptr(src), _ptr(dst), _ptr(off), _ptr(cols),
                                   _nthreads())
    if nnz < 0:
        raise ValueError("gg_csr_from_tuples failed (%d)" % nnz)
    return off, cols[:nnz].copy()


def kronecker_csr(scale, edgefactor=16, seed=1, abc=KRON_ABC):
    """Canonical undirected CSR (int64 offsets, int32 ascending columns)."""
    n, src, dst = kronecker_tuples(scale, edgefactor, seed, abc)
    return csr_from_tuples(n, src, dst)


def perm_table(n, seed):
    out = np.empty(n, np.int32)
    if lib().gg_perm_table(n, seed, _ptr(out), _nthreads()) != 0:
        raise ValueError("gg_perm_table failed")
    return out


# ----------------------------------------------------------------------------
# Chung-Lu power law with isolated vertices

def chung_lu_cdf(ncore, gamma=2.1, mean_deg=30.0, max_deg=2.0e6):
    cdf = np.empty(ncore, np.float64)
    params = np.zeros(3, np.float64)
    if lib().gg_cl_cdf(ncore, gamma, mean_deg, max_deg, _ptr(cdf), _ptr(params)) != 0:
        raise ValueError("gg_cl_cdf failed")
    return cdf, params


def chung_lu_sizes(ncore, n_iso, mean_deg):
    n_total = ncore + n_iso
    m = int(round(ncore * mean_deg / 2.0))
    return n_total, m


def chung_lu_tuples(ncore, n_iso, seed=1, gamma=2.1, mean_deg=30.0, max_deg=2.0e6, cdf=None):
    if cdf is None:
        cdf, _ = chung_lu_cdf(ncore, gamma, mean_deg, max_deg)
    n_total, m = chung_lu_sizes(ncore, n_iso, mean_deg)
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    rc = lib().gg_cl_tuples(ncore, n_total, seed, _ptr(cdf), 0, m, _ptr(src), _ptr(dst),
                            _nthreads())
    if rc != 0:
        raise ValueError("gg_cl_tuples failed")
    return n_total, src, dst


def chung_lu_csr(ncore, n_iso, seed=1, gamma=2.1, mean_deg=30.0, max_deg=2.0e6):
    n, src, dst = chung_lu_tuples(ncore, n_iso, seed, gamma, mean_deg, max_deg)
    return csr_from_tuples(n, src, dst)


# ----------------------------------------------------------------------------
# device builders (torch tensors on a GPU); same graphs as the host builders

def _torch_stream(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def kronecker_csr_device(scale, edgefactor=16, seed=1, abc=KRON_ABC, device="cuda",
                         max_pass_keys=0, info=None):
    """kronecker_csr on the GPU, built in passes over source-label ranges of
    at most max_pass_keys directed keys each (0: as many as fit, with the
    sort's buffers, in 80 % of the free device memory); info (a dict, optional) receives the number
    of passes."""
    import torch
    n = 1 << scale
    m = edgefactor * n
    off = torch.empty(n + 1, dtype=torch.int64, device=device)
    cols = torch.empty(max(1, 2 * m), dtype=torch.int32, device=device)
    passes = ctypes.c_int64(0)
    nnz = lib().gg_dev_kron_csr_ranges(scale, edgefactor, seed, abc[0], abc[1], abc[2],
                                       off.data_ptr(), cols.data_ptr(), cols.numel(),
                                       int(max_pass_keys), ctypes.byref(passes),
                                       _torch_stream(off.device))
    if nnz < 0:
        raise RuntimeError("gg_dev_kron_csr_ranges: " + lib().gg_dev_last_error().decode())
    if info is not None:
        info["passes"] = passes.value
    return off, cols[:nnz]


def kronecker_tuples_reached_device(scale, depth, edgefactor=16, seed=1, abc=KRON_ABC):
    """Tuples of kronecker_csr(scale, edgefactor, seed) (self-loops and
    duplicates included) whose endpoints both have depth >= 0; depth is a
    device int32 tensor indexed by vertex ID."""
    r = lib().gg_dev_kron_count_reached(scale, edgefactor, seed, abc[0], abc[1], abc[2],
                                        depth.data_ptr(), _torch_stream(depth.device))
    if r < 0:
        raise RuntimeError("gg_dev_kron_count_reached: " + lib().gg_dev_last_error().decode())
    return int(r)


def chung_lu_csr_device(ncore, n_iso, seed=1, gamma=2.1, mean_deg=30.0, max_deg=2.0e6,
                        device="cuda"):
    import torch
    cdf, _ = chung_lu_cdf(ncore, gamma, mean_deg, max_deg)
    n_total, m = chung_lu_sizes(ncore, n_iso, mean_deg)
    off = torch.empty(n_total + 1, dtype=torch.int64, device=device)
    cols = torch.empty(max(1, 2 * m), dtype=torch.int32, device=device)
    nnz = lib().gg_dev_cl_csr(ncore, n_total, m, seed, _ptr(cdf), off.data_ptr(),
                              cols.data_ptr(), cols.numel(), _torch_stream(off.device))
    if nnz < 0:
        raise RuntimeError("gg_dev_cl_csr: " + lib().gg_dev_last_error().decode())
    return off, cols[:nnz]


# ----------------------------------------------------------------------------
# roots

def sample_roots(off, k, seed, distinct=True):
    """k roots drawn uniformly from the vertices of nonzero degree (original
    IDs), by rejection from the counter-based stream STREAM_ROOT."""
    off = np.asarray(off)
    n = off.shape[0] - 1
    deg = np.diff(off)
    if not (deg > 0).any():
        raise ValueError("graph has no edges")
    roots, seen, ctr = [], set(), 0
    while len(roots) < k:
        v = draw(seed, STREAM_ROOT, ctr) % n
        ctr += 1
        if deg[v] == 0 or (distinct and v in seen):
            continue
        seen.add(v)
        roots.append(int(v))
    return roots


def sample_roots_device(off_dev, k, seed, distinct=True):
    """Same roots as sample_roots, reading only the degrees it needs."""
    import torch
    n = off_dev.numel() - 1
    roots, seen, ctr = [], set(), 0
    while len(roots) < k:
        cand = []
        while len(cand) < 256:
            cand.append(draw(seed, STREAM_ROOT, ctr) % n)
            ctr += 1
        idx = torch.tensor(cand, dtype=torch.int64, device=off_dev.device)
        d = (off_dev[idx + 1] - off_dev[idx]).cpu().numpy()
        for v, dv in zip(cand, d):
            if len(roots) == k:
                break
            if dv == 0 or (distinct and v in seen):
                continue
            seen.add(v)
            roots.append(int(v))
    return roots


# ----------------------------------------------------------------------------
# seeded draws for training the direction-switch network (initial weights and
# per-epoch sample orders); passed to both the GPU trainer and its reference

MLP_LAYERS = [((32, 8), 8), ((32,), 8), ((32, 32), 32), ((32,), 32), ((2, 32), 32), ((2,), 32)]


def mlp_init_weights(seed):
    """1410 values, layer by layer (W1, b1, W2, b2, W3, b3), each uniform in
    +-1/sqrt(fan_in) of its layer."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1.0 / np.sqrt(fan), 1.0 / np.sqrt(fan), size=shape).ravel()
             for shape, fan in MLP_LAYERS]
    return np.concatenate(parts)


def epoch_orders(n, epochs, seed):
    """Seeded per-epoch permutations of n samples, shape (epochs, n)."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
