"""Python binding of librbfs (RCM-relabelled direction-optimizing BFS on
MI355X).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  The library must
have been built (``python -m paper_2012_10026_amd._build``); importing the
binding without it raises, there is no fallback.
"""
import atexit
import ctypes
import math
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbfs.so")

RBFS_OK = 0
ERRORS = {-1: "INVAL", -2: "RANGE", -3: "NOMEM", -4: "DEVICE", -5: "STATE", -6: "NODEV",
          -7: "UNSUPPORTED"}
HOST_PTRS = 1
VALIDATE = 2
DIR_HEURISTIC, DIR_TD_ONLY, DIR_BU_ONLY, DIR_SCHEDULE, DIR_LEARNED = 0, 1, 2, 3, 4
OUT_ORIGINAL, OUT_INTERNAL = 0, 1
CERT_ROOT, CERT_REACH, CERT_LEVEL, CERT_ORPHAN, CERT_PARENT, CERT_LARGER, CERT_RANGE = \
    -1, -2, -3, -4, -5, -6, -7
STATS_MAX_LEVELS = 64
MLP_PARAMS = 8 * 32 + 32 + 32 * 32 + 32 + 32 * 2 + 2
SWITCH_BLOB = MLP_PARAMS + 8 + 8 + 1 + 1


class RbfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("alpha", ctypes.c_int32),
                ("beta", ctypes.c_int32), ("output_space", ctypes.c_int32),
                ("schedule", ctypes.c_void_p), ("schedule_len", ctypes.c_int32),
                ("tune_profile", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Stats(ctypes.Structure):
    L = STATS_MAX_LEVELS
    _fields_ = [("levels", ctypes.c_int32), ("status", ctypes.c_int32),
                ("dir", ctypes.c_int8 * L), ("fallback", ctypes.c_int8 * L),
                ("nf", ctypes.c_int64 * L),
                ("mf", ctypes.c_int64 * L), ("mu", ctypes.c_int64 * L),
                ("edges", ctypes.c_int64 * L), ("level_us", ctypes.c_float * L),
                ("reached", ctypes.c_int64),
                ("component_edges", ctypes.c_int64), ("ms_kernel", ctypes.c_float),
                ("ms_total", ctypes.c_float)]

    def as_dict(self):
        n = min(self.levels, STATS_MAX_LEVELS)
        return {"levels": self.levels, "status": self.status,
                "dir": list(self.dir[:n]), "fallback": list(self.fallback[:n]),
                "nf": list(self.nf[:n]), "mf": list(self.mf[:n]),
                "mu": list(self.mu[:n]), "edges": list(self.edges[:n]),
                "level_us": list(self.level_us[:n]),
                "reached": self.reached, "component_edges": self.component_edges,
                "ms_kernel": self.ms_kernel, "ms_total": self.ms_total}


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_plus", ctypes.c_int64),
                ("reordered", ctypes.c_int32), ("device", ctypes.c_int32),
                ("max_degree", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("rcm_keep", ctypes.c_int64)]


TUNE_SINGLE, TUNE_BATCH = 0, 1
TUNING_FIELDS = ("block", "per_cu", "lane_row", "bu_grain", "td_chunk", "reset")


class Tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in TUNING_FIELDS]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in TUNING_FIELDS}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for f in TUNING_FIELDS:
            setattr(t, f, int(d[f]))
        return t


class TuneRecord(ctypes.Structure):
    _fields_ = [("tuning", Tuning), ("ms", ctypes.c_float), ("mismatches", ctypes.c_int32)]


class DeviceInfo(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("compute_units", ctypes.c_int32),
                ("wavefront_size", ctypes.c_int32), ("clock_khz", ctypes.c_int32),
                ("global_mem_bytes", ctypes.c_int64), ("l2_bytes", ctypes.c_int64),
                ("arch", ctypes.c_char * 64)]


# exported symbols with their ctypes signatures; tests check that every one
# declared in include/rbfs.h is listed and exported
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
SIGNATURES = {
    "rbfs_last_error": (ctypes.c_char_p, []),
    "rbfs_device_info": (ctypes.c_int, [_P]),
    "rbfs_graph_create": (ctypes.c_int, [_I64, _I64, _P, _P, ctypes.c_uint32, _P, _P]),
    "rbfs_set_allocator": (ctypes.c_int, [_P, _P, _P]),
    "rbfs_graph_destroy": (ctypes.c_int, [_P]),
    "rbfs_graph_info": (ctypes.c_int, [_P, _P]),
    "rbfs_graph_check": (ctypes.c_int, [_P, _P]),
    "rbfs_graph_timings": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P]),
    "rbfs_graph_wg_work": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P]),
    "rbfs_rcm_reorder": (ctypes.c_int, [_P, _P, _P, _P]),
    "rbfs_rcm_reorder_partial": (ctypes.c_int, [_P, _I64, _P, _P, _P]),
    "rbfs_graph_set_rcm_batch": (ctypes.c_int, [_P, _I64]),
    "rbfs_graph_set_queue_cap": (ctypes.c_int, [_P, _I64]),
    "rbfs_graph_set_rcm_staging": (ctypes.c_int, [_P, _I32]),
    "rbfs_graph_iperm": (ctypes.c_int, [_P, _P, _P]),
    "rbfs_graph_csr": (ctypes.c_int, [_P, _P, _P, _P]),
    "rbfs_graph_bandwidth": (ctypes.c_int, [_P, _P, _P]),
    "rbfs_bfs": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P]),
    "rbfs_bfs_batch": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _P, _P]),
    "rbfs_certify": (ctypes.c_int, [_P, _I32, _P, _P, _I32, _P, _P]),
    "rbfs_certify_noalloc": (ctypes.c_int, [_P, _I32, _P, _P, _I32, _P, _P]),
    "rbfs_multi_create": (ctypes.c_int, [_P, _I32, _P, _P]),
    "rbfs_multi_destroy": (ctypes.c_int, [_P]),
    "rbfs_bfs_multi": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _P, _P]),
    "rbfs_switch_load": (ctypes.c_int, [_P, _I32]),
    "rbfs_collect_level_samples": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _I32, _P, _I32,
                                                  _P, _P]),
    "rbfs_collect_level_timings": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _I32, _P, _I32,
                                                  _P, _P]),
    "rbfs_mlp_train": (ctypes.c_int, [_P, _I32, _P, _P, _I32, _I32, ctypes.c_float, _P, _P,
                                      _P]),
    "rbfs_mlp_forward": (ctypes.c_int, [_P, _P, _I32, _P]),
    "rbfs_mlp_grad": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "rbfs_mlp_backward": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "rbfs_tuning_default": (ctypes.c_int, [_I32, _P]),
    "rbfs_graph_set_tuning": (ctypes.c_int, [_P, _I32, _P, _P]),
    "rbfs_graph_get_tuning": (ctypes.c_int, [_P, _I32, _P]),
    "rbfs_tune": (ctypes.c_int, [_P, _I32, _P, _I32, _I32, _P, _P, _P, _I32, _P, _P]),
    "rbfs_multi_set_tuning": (ctypes.c_int, [_P, _P, _P]),
    "rbfs_multi_get_tuning": (ctypes.c_int, [_P, _P]),
    "rbfs_multi_tune": (ctypes.c_int, [_P, _P, _I32, _I32, _P, _P, _I32, _P, _P]),
}

_lib = None

# Device memory of the library: torch's caching allocator by default (set
# RBFS_ALLOCATOR=hip for hipMalloc/hipFree).  The callbacks run on the thread
# of the library call that needs memory.
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  int(stream) if stream else None)
    except Exception:  # out of memory: the library call returns RBFS_E_NOMEM
        return None


def _torch_free(ptr, stream, ctx):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


_torch_alloc_cb = _ALLOC_FN(_torch_alloc)
_torch_free_cb = _FREE_FN(_torch_free)
_allocator = "hip"
_live_graphs = weakref.WeakSet()
_live_multis = weakref.WeakSet()


def lib():
    """Load librbfs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librbfs.so not built: run python -m paper_2012_10026_amd._build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
        if os.environ.get("RBFS_ALLOCATOR", "torch") != "hip":
            set_allocator("torch")
    return _lib


def set_allocator(kind):
    """'torch': the library's device memory comes from torch's caching
    allocator (counted by torch.cuda.memory_allocated); 'hip': hipMalloc.
    Only while no Graph or MultiGraph is open."""
    global _allocator
    if kind == "torch":
        rc = lib().rbfs_set_allocator(ctypes.cast(_torch_alloc_cb, ctypes.c_void_p),
                                      ctypes.cast(_torch_free_cb, ctypes.c_void_p), None)
    elif kind == "hip":
        rc = lib().rbfs_set_allocator(None, None, None)
    else:
        raise ValueError("allocator must be 'torch' or 'hip'")
    _check(rc)
    _allocator = kind


def allocator():
    return _allocator


@atexit.register
def _close_all():
    # release library memory while torch's allocator is still alive
    for m in list(_live_multis):
        m.close()
    for g in list(_live_graphs):
        g.close()


def _check(rc):
    if rc != RBFS_OK:
        raise RbfsError(rc, lib().rbfs_last_error().decode())


def _stream_ptr(device=None):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def device_info():
    d = DeviceInfo()
    _check(lib().rbfs_device_info(ctypes.byref(d)))
    return {"device": d.device, "compute_units": d.compute_units,
            "wavefront_size": d.wavefront_size, "clock_khz": d.clock_khz,
            "global_mem_bytes": d.global_mem_bytes, "l2_bytes": d.l2_bytes,
            "arch": d.arch.decode()}


OPT_TIMING = 1
OPT_WG_WORK = 2
OPT_ZERO_WAIT = 4
OPT_NO_BALANCE = 8


def default_tuning(kind=TUNE_SINGLE):
    t = Tuning()
    _check(lib().rbfs_tuning_default(kind, ctypes.byref(t)))
    return t.as_dict()


def _as_tuning(t):
    return t if isinstance(t, Tuning) else Tuning.from_dict(t)


def _records(recs, cnt):
    return [dict(r.tuning.as_dict(), ms=float(r.ms), mismatches=int(r.mismatches))
            for r in recs[:cnt]]


def make_opts(direction=DIR_HEURISTIC, alpha=14, beta=24, output_space=OUT_ORIGINAL,
              schedule=None, tune_profile=0, timing=False, wg_work=False, zero_wait=False,
              no_balance=False):
    o = Opts()
    o.flags = ((OPT_TIMING if timing else 0) | (OPT_WG_WORK if wg_work else 0) |
               (OPT_ZERO_WAIT if zero_wait else 0) | (OPT_NO_BALANCE if no_balance else 0))
    o.direction = direction
    o.alpha = alpha
    o.beta = beta
    o.output_space = output_space
    o.tune_profile = tune_profile
    o._sched = None
    if schedule is not None:
        arr = (ctypes.c_int8 * len(schedule))(*[int(x) for x in schedule])
        o._sched = arr  # keep alive
        o.schedule = ctypes.cast(arr, ctypes.c_void_p)
        o.schedule_len = len(schedule)
    return o


class Graph:
    """Handle on a graph resident on the current GPU.

    off, cols: canonical undirected CSR (int64 offsets, int32 columns), as
    torch tensors on the GPU or numpy arrays on the host.
    """

    def __init__(self, off, cols, validate=False):
        import torch
        self._h = ctypes.c_void_p()
        flags = VALIDATE if validate else 0
        if isinstance(off, np.ndarray):
            off = np.ascontiguousarray(off, np.int64)
            cols = np.ascontiguousarray(cols, np.int32)
            flags |= HOST_PTRS
            n = off.shape[0] - 1
            nnz = cols.shape[0]
            p_off = off.ctypes.data_as(ctypes.c_void_p)
            p_cols = cols.ctypes.data_as(ctypes.c_void_p) if nnz else None
            self.device = torch.device("cuda", torch.cuda.current_device())
        else:
            assert off.dtype == torch.int64 and cols.dtype == torch.int32
            off = off.contiguous()
            cols = cols.contiguous()
            n = off.numel() - 1
            nnz = cols.numel()
            p_off = _dptr(off)
            p_cols = _dptr(cols) if nnz else None
            self.device = off.device
        self.n = n
        self.nnz = nnz
        _check(lib().rbfs_graph_create(n, nnz, p_off, p_cols, flags, _stream_ptr(self.device),
                                       ctypes.byref(self._h)))
        _live_graphs.add(self)

    def close(self):
        """Release the graph; raises RbfsError (STATE) while a MultiGraph
        built over it is open."""
        if self._h:
            _check(lib().rbfs_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self):
        i = GraphInfo()
        _check(lib().rbfs_graph_info(self._h, ctypes.byref(i)))
        return {"n": i.n, "nnz": i.nnz, "n_plus": i.n_plus, "reordered": i.reordered,
                "device": i.device, "max_degree": i.max_degree,
                "device_bytes": i.device_bytes, "rcm_keep": i.rcm_keep}

    def rcm_reorder(self, want_perm=True, partial=None, keep=None):
        """Relabel by RCM; returns (perm tensor or None, milliseconds).
        partial=p (a ratio in [0, 1]) or keep=k reorders only the first
        ceil(p * n_plus) (or k) vertices of the Cuthill-McKee sequence."""
        import torch
        perm = torch.empty(self.n, dtype=torch.int32, device=self.device) if want_perm else None
        ms = ctypes.c_float(0.0)
        if partial is not None:
            if keep is not None:
                raise ValueError("give partial or keep, not both")
            keep = math.ceil(float(partial) * self.info()["n_plus"])
        pp = _dptr(perm) if perm is not None else None
        if keep is None:
            _check(lib().rbfs_rcm_reorder(self._h, pp, _stream_ptr(self.device),
                                          ctypes.byref(ms)))
        else:
            _check(lib().rbfs_rcm_reorder_partial(self._h, int(keep), pp,
                                                  _stream_ptr(self.device), ctypes.byref(ms)))
        return perm, ms.value

    def set_rcm_batch(self, max_entries):
        """Relabel in batches of about max_entries adjacency entries (0:
        automatic, by graph size); the permutation and CSR are the same."""
        _check(lib().rbfs_graph_set_rcm_batch(self._h, int(max_entries)))

    def set_rcm_staging(self, mode):
        """Old columns of a batched relabel in host memory: 0 when device
        memory is short (default), 1 always, -1 never."""
        _check(lib().rbfs_graph_set_rcm_staging(self._h, int(mode)))

    def set_queue_cap(self, entries):
        """Entries of each frontier sub-queue of single-root searches (0:
        automatic); the rest goes to a shared overflow queue.  Results do
        not depend on it."""
        _check(lib().rbfs_graph_set_queue_cap(self._h, int(entries)))

    def iperm(self):
        import torch
        out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(lib().rbfs_graph_iperm(self._h, _dptr(out), _stream_ptr(self.device)))
        return out

    def csr(self):
        """The current (after RCM: relabelled) CSR as device tensors
        (int64 offsets, int32 columns)."""
        import torch
        off = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        cols = torch.empty(max(1, self.nnz), dtype=torch.int32, device=self.device)
        _check(lib().rbfs_graph_csr(self._h, _dptr(off), _dptr(cols),
                                    _stream_ptr(self.device)))
        return off, cols[:self.nnz]

    def bandwidth(self):
        """Largest |u - v| over the adjacency entries in the current labels."""
        out = ctypes.c_int64(0)
        _check(lib().rbfs_graph_bandwidth(self._h, ctypes.byref(out), _stream_ptr(self.device)))
        return out.value

    def bfs(self, root, depth=None, parent=None, opts=None, stats=False):
        """Returns (depth, parent[, stats dict]) as int32 device tensors."""
        import torch
        if depth is None:
            depth = torch.empty(self.n, dtype=torch.int32, device=self.device)
        if parent is None:
            parent = torch.empty(self.n, dtype=torch.int32, device=self.device)
        st = Stats() if stats else None
        _check(lib().rbfs_bfs(self._h, int(root), _dptr(depth), _dptr(parent),
                              ctypes.byref(opts) if opts is not None else None,
                              _stream_ptr(self.device),
                              ctypes.byref(st) if st is not None else None))
        if stats:
            return depth, parent, st.as_dict()
        return depth, parent

    def bfs_batch(self, roots, depth=None, parent=None, opts=None, stats=False):
        """k roots at once; returns root-major (k, n) depth and parent."""
        import torch
        k = len(roots)
        r = (ctypes.c_int32 * k)(*[int(x) for x in roots])
        if depth is None:
            depth = torch.empty((k, self.n), dtype=torch.int32, device=self.device)
        if parent is None:
            parent = torch.empty((k, self.n), dtype=torch.int32, device=self.device)
        st = Stats() if stats else None
        _check(lib().rbfs_bfs_batch(self._h, r, k, _dptr(depth), _dptr(parent),
                                    ctypes.byref(opts) if opts is not None else None,
                                    _stream_ptr(self.device),
                                    ctypes.byref(st) if st is not None else None))
        if stats:
            return depth, parent, st.as_dict()
        return depth, parent

    def check(self):
        _check(lib().rbfs_graph_check(self._h, _stream_ptr(self.device)))

    def wg_work(self):
        """Entries each workgroup processed per level in the last search (made
        with OPT_WG_WORK): numpy int64 array of shape (levels, grid)."""
        lv, gr = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().rbfs_graph_wg_work(self._h, None, 0, ctypes.byref(lv), ctypes.byref(gr),
                                        _stream_ptr(self.device)))
        out = np.zeros(lv.value * gr.value, dtype=np.int64)
        if out.size:
            _check(lib().rbfs_graph_wg_work(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                            out.size, ctypes.byref(lv), ctypes.byref(gr),
                                            _stream_ptr(self.device)))
        return out.reshape(lv.value, gr.value)

    def certify(self, root, depth, parent, output_space=OUT_ORIGINAL):
        """Checks (depth, parent) of a search from `root` against the graph on
        the device; returns 0 if it is the search result, else a negative
        rule code (CERT_* constants)."""
        res = ctypes.c_int32(0)
        _check(lib().rbfs_certify(self._h, int(root), _dptr(depth), _dptr(parent),
                                  int(output_space), _stream_ptr(self.device),
                                  ctypes.byref(res)))
        return res.value

    def set_tuning(self, tuning, kind=TUNE_SINGLE):
        t = _as_tuning(tuning)
        _check(lib().rbfs_graph_set_tuning(self._h, kind, ctypes.byref(t),
                                           _stream_ptr(self.device)))

    def get_tuning(self, kind=TUNE_SINGLE):
        t = Tuning()
        _check(lib().rbfs_graph_get_tuning(self._h, kind, ctypes.byref(t)))
        return t.as_dict()

    def tune(self, roots, kind=TUNE_SINGLE, reps=2, opts=None, cap=256):
        """Autotune the launch shape and work split on these roots (original
        IDs, at most 64).  Returns (best tuning dict, list of timed
        candidates); the best is set on the graph."""
        k = len(roots)
        r = (ctypes.c_int32 * k)(*[int(x) for x in roots])
        best = Tuning()
        recs = (TuneRecord * cap)()
        cnt = ctypes.c_int32(0)
        _check(lib().rbfs_tune(self._h, kind, r, k, reps,
                               ctypes.byref(opts) if opts is not None else None,
                               ctypes.byref(best), recs, cap, ctypes.byref(cnt),
                               _stream_ptr(self.device)))
        return best.as_dict(), _records(recs, cnt.value)

    def timings(self, cap=1024):
        """(kernel_ms, total_ms) lists of the calls made with timing=True."""
        k = (ctypes.c_float * cap)()
        t = (ctypes.c_float * cap)()
        cnt = ctypes.c_int32(0)
        _check(lib().rbfs_graph_timings(self._h, k, t, cap, ctypes.byref(cnt),
                                        _stream_ptr(self.device)))
        return list(k[:cnt.value]), list(t[:cnt.value])


class MultiGraph:
    """Several graphs searched together in one launch (disjoint union)."""

    def __init__(self, graphs):
        self.graphs = list(graphs)
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_void_p * len(self.graphs))(*[g.handle.value for g in self.graphs])
        self.device = self.graphs[0].device
        _check(lib().rbfs_multi_create(arr, len(self.graphs), _stream_ptr(self.device),
                                       ctypes.byref(self._h)))
        _live_multis.add(self)

    def close(self):
        if self._h:
            lib().rbfs_multi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def out_size(self, k):
        return sum(k * g.n for g in self.graphs)

    def set_tuning(self, tuning):
        t = _as_tuning(tuning)
        _check(lib().rbfs_multi_set_tuning(self._h, ctypes.byref(t), _stream_ptr(self.device)))

    def get_tuning(self):
        t = Tuning()
        _check(lib().rbfs_multi_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def tune(self, roots, reps=2, cap=256):
        """Autotune the batch parameters; roots as for bfs().  Returns (best
        tuning dict, list of timed candidates); the best is set."""
        k = len(roots[0])
        flat = [int(r) for rs in roots for r in rs]
        r = (ctypes.c_int32 * len(flat))(*flat)
        best = Tuning()
        recs = (TuneRecord * cap)()
        cnt = ctypes.c_int32(0)
        _check(lib().rbfs_multi_tune(self._h, r, k, reps, ctypes.byref(best), recs, cap,
                                     ctypes.byref(cnt), _stream_ptr(self.device)))
        return best.as_dict(), _records(recs, cnt.value)

    def bfs(self, roots, opts=None, stats=False, depth=None, parent=None):
        """roots: list (per graph) of k root lists.  Returns a list of
        (depth, parent) views, each (k, n_g).  Passing the same output
        buffers again replays the captured search."""
        import torch
        k = len(roots[0])
        flat = [int(r) for rs in roots for r in rs]
        r = (ctypes.c_int32 * len(flat))(*flat)
        total = self.out_size(k)
        if depth is None:
            depth = torch.empty(total, dtype=torch.int32, device=self.device)
        if parent is None:
            parent = torch.empty(total, dtype=torch.int32, device=self.device)
        st = Stats() if stats else None
        _check(lib().rbfs_bfs_multi(self._h, r, k, _dptr(depth), _dptr(parent),
                                    ctypes.byref(opts) if opts is not None else None,
                                    _stream_ptr(self.device),
                                    ctypes.byref(st) if st is not None else None))
        out, o = [], 0
        for g in self.graphs:
            sz = k * g.n
            out.append((depth[o:o + sz].view(k, g.n), parent[o:o + sz].view(k, g.n)))
            o += sz
        if stats:
            return out, st.as_dict()
        return out


# ----------------------------------------------------------------------------
# learned direction switch

def _fptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def mlp_forward(w, x):
    w = np.ascontiguousarray(w, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    n = x.shape[0]
    y = np.empty((n, 2), np.float32)
    _check(lib().rbfs_mlp_forward(_fptr(w), _fptr(x), n, _fptr(y)))
    return y


def mlp_grad(w, samples):
    w = np.ascontiguousarray(w, np.float32)
    samples = np.ascontiguousarray(samples, np.float32)
    g = np.empty(MLP_PARAMS, np.float32)
    loss = ctypes.c_float(0.0)
    _check(lib().rbfs_mlp_grad(_fptr(w), _fptr(samples), samples.shape[0], _fptr(g),
                               ctypes.byref(loss)))
    return g, loss.value


def mlp_train(samples, w_init, order, batch=256, lr=1e-3):
    """order: (epochs, n) int32.  Returns (weights, loss curve)."""
    samples = np.ascontiguousarray(samples, np.float32)
    w_init = np.ascontiguousarray(w_init, np.float32)
    order = np.ascontiguousarray(order, np.int32)
    epochs, n = order.shape
    w = np.empty(MLP_PARAMS, np.float32)
    curve = np.empty(epochs, np.float32)
    _check(lib().rbfs_mlp_train(_fptr(samples), n, _fptr(w_init), _fptr(order), epochs, batch,
                                ctypes.c_float(lr), _fptr(w), _fptr(curve),
                                _stream_ptr()))
    return w, curve


def switch_load(blob):
    blob = np.ascontiguousarray(blob, np.float32)
    assert blob.shape == (SWITCH_BLOB,)
    _check(lib().rbfs_switch_load(_fptr(blob), SWITCH_BLOB))


def collect_level_samples(graph, roots, reps=3, alpha=14, beta=24, cap=4096):
    """Rows of 11 floats: features[8], ln us top-down, ln us bottom-up, level."""
    r = (ctypes.c_int32 * len(roots))(*[int(x) for x in roots])
    out = np.empty((cap, 11), np.float32)
    cnt = ctypes.c_int32(0)
    _check(lib().rbfs_collect_level_samples(graph.handle, r, len(roots), reps, alpha, beta,
                                            _fptr(out), cap, ctypes.byref(cnt),
                                            _stream_ptr(graph.device)))
    return out[:cnt.value].copy()


def make_switch_blob(w, features, margin=0.1):
    """Weights plus the training feature range, the largest level and the
    decision margin (ln microseconds; the default is the margin that
    validation picks for labels that run to the end of the search)."""
    features = np.asarray(features, np.float32)
    blob = np.zeros(SWITCH_BLOB, np.float32)
    blob[:MLP_PARAMS] = w
    blob[MLP_PARAMS:MLP_PARAMS + 8] = features[:, :8].min(axis=0)
    blob[MLP_PARAMS + 8:MLP_PARAMS + 16] = features[:, :8].max(axis=0)
    blob[MLP_PARAMS + 16] = features[:, 10].max() if features.shape[1] > 10 else 64
    blob[MLP_PARAMS + 17] = margin
    return blob


from .autotune import TuningCache, tuning_key, tune_cached  # noqa: E402,F401
