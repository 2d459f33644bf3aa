"""Shared helpers of the GPU tests (not collected: no test functions)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import graphgen


def oracle_threads():
    """Host threads for independent oracle calls: the oracle's C functions
    release the GIL (ctypes), so roots run in parallel, each single-threaded.
    At most 16, the host CPU share of a one-GPU machine."""
    return max(1, min(16, os.cpu_count() or 1))


def pmap(fn, items, threads=None):
    with ThreadPoolExecutor(threads or oracle_threads()) as ex:
        return list(ex.map(fn, items))


def train_kronecker_blob(rb, scales=(13, 14, 15), seed=0, epochs=200):
    """A switch blob trained on per-level timings of small Kronecker graphs
    (RCM-relabelled), for tests that evaluate it on other graphs without
    retraining."""
    rows = []
    for i, s in enumerate(scales):
        off, cols = graphgen.kronecker_csr(s, 16, 7100 + 10 * s + i)
        G = rb.Graph(off, cols)
        G.rcm_reorder(want_perm=False)
        rows.append(rb.collect_level_samples(G, graphgen.sample_roots(off, 6, 50 + i), reps=2))
        G.close()
    rows = np.vstack(rows)
    order = graphgen.epoch_orders(rows.shape[0], epochs, 1 + seed)
    w, _ = rb.mlp_train(rows[:, :10], graphgen.mlp_init_weights(seed).astype(np.float32), order,
                        batch=64, lr=3e-3)
    return rb.make_switch_blob(w, rows)
