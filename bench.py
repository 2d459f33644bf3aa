"""Benchmark: GTEPS (harmonic mean over 64 roots) of RCM-relabelled
direction-optimizing BFS on one MI355X, Kronecker scale 26 by default.

One step = 64 single-root searches (plain alpha = 14 / beta = 24 heuristic,
outputs in original IDs), inputs resident in HBM.  RCM is timed once,
separately.  Also measured on the same graph and roots: the learned direction
switch (trained here on per-level timings of scale 18-24 graphs) and the
64-root bit-parallel batch; the learned switch on held-out power-law graphs
(exponent 2.1), where it has headroom over alpha/beta; and the 32-graph
multi-graph batch.  Launch
parameters come from the autotuner's JSON cache (tuned on other roots of the
same graphs; a missing entry is tuned in the run, --retune forces it,
--no-tune uses the built-in defaults).  Prints one JSON line.
"""
import argparse
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DEFAULT_TUNING_CACHE = os.path.join(ROOT, "paper_2012_10026_amd", "tuning", "mi355x.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def bfs_alg_bytes(st, n_sweep, original_ids=True):
    """Algorithmic bytes of one search kernel launch from its per-level
    counters: top-down level: 16 n_f (row offsets) + 4 n_f (queue) +
    4 e_td (columns) + 12 n_new (depth, parent, queue write); bottom-up
    level: 8 n_u (row offsets) + 4 e_bu (columns read up to the first hit) +
    3 * n_sweep / 8 (visited read, next write) + 8 n_new.  With outputs in
    original IDs the kernel also does the iperm gather of the output
    translation: 4 bytes per reached vertex (its parent's original ID)."""
    total = 4 * st["reached"] if original_ids else 0
    reached = 0
    L = st["levels"]
    for d in range(min(L, len(st["nf"]))):
        nf = st["nf"][d]
        reached += nf
        n_new = st["nf"][d + 1] if d + 1 < len(st["nf"]) else 0
        if st["dir"][d] == 0:
            total += 16 * nf + 4 * nf + 4 * st["edges"][d] + 12 * n_new
        else:
            n_u = n_sweep - reached
            total += 8 * n_u + 4 * st["edges"][d] + 3 * ((n_sweep + 7) // 8) + 8 * n_new
    return total


def measured_traffic(workload):
    """Per-launch bytes of the search kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the counters were taken on
    another workload or the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_bfs_persistent_kernel.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha1()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["source_sha1"] or rec["workload"] != workload:
            return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(off_dev, cols_dev, roots, budget_s=30.0):
    """The oracle's BFS (single thread, original labels) on a bounded sample
    of the roots of the same graph."""
    import oracle
    off = off_dev.cpu().numpy()
    cols = cols_dev.cpu().numpy()
    t_all, edges_all, used = 0.0, 0, []
    for r in roots:
        t0 = time.perf_counter()
        depth, _, _ = oracle.bfs(off, cols, r)
        t_all += time.perf_counter() - t0
        edges_all += oracle.component_edges(off, depth)
        used.append(r)
        if t_all > budget_s * 0.5:
            break
    del off, cols
    return {"value": edges_all / t_all / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "oracle BFS (single thread, original labels) from %d of the roots on the "
                      "same graph, %.1f s" % (len(used), t_all)}


def time_roots(G, roots, depth, parent, opts, steps):
    """Per-root event times (ms, median over steps) on the current stream, and
    the wall time of all steps."""
    import torch
    stream = torch.cuda.current_stream()
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in roots] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        for i, r in enumerate(roots):
            evs[s][i][0].record(stream)
            G.bfs(r, depth, parent, opts=opts)
            evs[s][i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_root = [statistics.median(evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(steps))
                for i in range(len(roots))]
    return per_root, wall


def hmean_gteps(m_c, per_root_ms):
    teps = [m / (t * 1e-3) for m, t in zip(m_c, per_root_ms)]
    return len(teps) / sum(1.0 / x for x in teps) / 1e9


def train_switch(rb, graphgen):
    """Per-level both-direction timings on Kronecker graphs of scales 18, 20,
    22, 24 (4 graphs each, 8 roots each), then GPU training; returns the
    switch blob and a summary."""
    import numpy as np
    import torch
    rows = []
    t0 = time.perf_counter()
    for s in (18, 20, 22, 24):
        for j in range(4):
            off, cols = graphgen.kronecker_csr_device(s, 16, 2000 + 10 * s + j)
            roots = graphgen.sample_roots_device(off, 8, 7)
            G = rb.Graph(off, cols)
            del off, cols
            G.rcm_reorder(want_perm=False)
            rows.append(rb.collect_level_samples(G, roots, reps=3))
            G.close()
            torch.cuda.empty_cache()
    rows = np.vstack(rows)
    t_collect = time.perf_counter() - t0
    order = graphgen.epoch_orders(rows.shape[0], 300, 1)
    t0 = time.perf_counter()
    w, curve = rb.mlp_train(rows[:, :10], graphgen.mlp_init_weights(0).astype(np.float32), order,
                            batch=64, lr=3e-3)
    t_train = time.perf_counter() - t0
    log("# switch: %d samples (%.1f s), trained %.2f s, loss %.3f -> %.3f"
        % (rows.shape[0], t_collect, t_train, curve[0], curve[-1]))
    return rb.make_switch_blob(w, rows), {"samples": int(rows.shape[0]),
                                          "train_graphs": "kronecker scales 18,20,22,24 x 4",
                                          "collect_s": t_collect, "train_s": t_train,
                                          "loss_first": float(curve[0]),
                                          "loss_last": float(curve[-1])}


def schedule_costs(rb, G, roots, learned_opts, plain_opts):
    """Measured per-level cost of the alpha/beta and learned schedules and of
    the best per-level choice (from both-direction level timings)."""
    tot = {"alpha_beta_us": 0.0, "learned_us": 0.0, "best_us": 0.0}
    agree_l = agree_h = nlev = 0
    for r in roots:
        rows = rb.collect_level_samples(G, [r], reps=3)
        by = {int(x[10]): x for x in rows}
        _, _, sl = G.bfs(r, opts=learned_opts, stats=True)
        _, _, sh = G.bfs(r, opts=plain_opts, stats=True)
        for lv, x in by.items():
            best = 0 if x[8] <= x[9] else 1
            tot["best_us"] += math.exp(min(x[8], x[9]))
            if lv < len(sl["dir"]):
                tot["learned_us"] += math.exp(x[8 + sl["dir"][lv]])
                agree_l += int(sl["dir"][lv] == best)
            if lv < len(sh["dir"]):
                tot["alpha_beta_us"] += math.exp(x[8 + sh["dir"][lv]])
                agree_h += int(sh["dir"][lv] == best)
            nlev += 1
    tot["learned_regret"] = tot["learned_us"] / tot["best_us"] - 1.0
    tot["alpha_beta_regret"] = tot["alpha_beta_us"] / tot["best_us"] - 1.0
    tot["learned_best_choice_frac"] = agree_l / max(1, nlev)
    tot["alpha_beta_best_choice_frac"] = agree_h / max(1, nlev)
    tot["roots"] = len(roots)
    return tot


def heavy_tail_switch(rb, graphgen, steps, alpha, beta):
    """The learned switch on power-law graphs (Chung-Lu, 300000 vertices,
    exponent 2.1, mean degree 30), where the alpha/beta thresholds stay
    bottom-up too long at the tail: trained on 4 graphs (8 roots each),
    measured on a held-out fifth (8 roots).  Loads its own switch blob."""
    import numpy as np
    import torch

    def graph(seed):
        off, cols = graphgen.chung_lu_csr(300000, 15000, seed=seed, gamma=2.1, mean_deg=30.0,
                                          max_deg=20000.0)
        G = rb.Graph(off, cols)
        G.rcm_reorder(want_perm=False)
        return off, G
    rows = []
    for seed in (1, 2, 3, 4):
        off, G = graph(seed)
        rows.append(rb.collect_level_samples(G, graphgen.sample_roots(off, 8, 100 + seed), reps=3))
        G.close()
    rows = np.vstack(rows)
    order = graphgen.epoch_orders(rows.shape[0], 300, 1)
    w, curve = rb.mlp_train(rows[:, :10], graphgen.mlp_init_weights(0).astype(np.float32), order,
                            batch=64, lr=3e-3)
    rb.switch_load(rb.make_switch_blob(w, rows))
    off, G = graph(9)
    roots = graphgen.sample_roots(off, 8, 5)
    depth = torch.empty(G.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(G.n, dtype=torch.int32, device="cuda")
    learned = rb.make_opts(rb.DIR_LEARNED, alpha=alpha, beta=beta)
    plain = rb.make_opts(alpha=alpha, beta=beta)
    for r in roots:
        G.bfs(r, depth, parent, opts=learned)
        G.bfs(r, depth, parent, opts=plain)
    per_l, _ = time_roots(G, roots, depth, parent, learned, max(steps, 5))
    per_h, _ = time_roots(G, roots, depth, parent, plain, max(steps, 5))
    out = {"graph": "chung-lu n=300000 exponent 2.1 mean degree 30 (held-out seed 9)",
           "train_samples": int(rows.shape[0]),
           "ms_per_root_learned": sum(per_l) / len(per_l),
           "ms_per_root_alpha_beta": sum(per_h) / len(per_h),
           "speedup": sum(per_h) / sum(per_l),
           "schedule_costs_8_roots": schedule_costs(rb, G, roots, learned, plain)}
    G.close()
    torch.cuda.empty_cache()
    log("# learned, heavy tail: %.3f ms against %.3f ms per root (%.2fx)"
        % (out["ms_per_root_learned"], out["ms_per_root_alpha_beta"], out["speedup"]))
    return out


def tuned_leg(rb, target, roots, cache, graph_class, kind, retune, opts=None, reps=2):
    """Autotuned parameters for one leg: from the cache, or tuned now (and
    stored).  Returns a report dict."""
    from paper_2012_10026_amd import autotune
    t_t = time.perf_counter()
    best, recs = rb.tune_cached(target, roots, cache, graph_class, kind=kind, reps=reps,
                                opts=opts, retune=retune)
    key = autotune.tuning_key(rb.device_info()["arch"], graph_class,
                              autotune.target_size(target), kind)
    e = cache.entries.get(key, {})
    rep = {"tuning": best, "key": key, "source": "tuned now" if recs else "cache",
           "default_ms": e.get("default_ms"), "tuned_ms": e.get("ms"),
           "seconds": time.perf_counter() - t_t}
    if recs:
        rep["candidates"] = len(recs)
    log("# tuning %s (%s): %s" % (key, rep["source"], best))
    return rep


def multi_batch(rb, graphgen, steps, cache=None, retune=False):
    """32 Kronecker graphs of scales 12 + (g mod 9), 16 roots each, searched in
    one captured launch, against the 512 single-root searches."""
    import torch
    Gs, roots, troots, m_c = [], [], [], 0
    for g in range(32):
        s = 12 + (g % 9)
        off, cols = graphgen.kronecker_csr_device(s, 16, 3000 + g)
        rs = graphgen.sample_roots_device(off, 16, 7)
        troots.append(graphgen.sample_roots_device(off, 16, 1007))  # autotuner's sample
        G = rb.Graph(off, cols)
        G.rcm_reorder(want_perm=False)
        Gs.append(G)
        roots.append(rs)
    M = rb.MultiGraph(Gs)
    tuned = None
    if cache is not None:
        tuned = tuned_leg(rb, M, troots, cache, "kronecker-multi32", rb.TUNE_BATCH, retune)
    tot = M.out_size(16)
    depth = torch.empty(tot, dtype=torch.int32, device="cuda")
    parent = torch.empty(tot, dtype=torch.int32, device="cuda")
    single_ms = 0.0
    for G, rs in zip(Gs, roots):
        d = torch.empty(G.n, dtype=torch.int32, device="cuda")
        p = torch.empty(G.n, dtype=torch.int32, device="cuda")
        for r in rs:
            _, _, st = G.bfs(r, d, p, stats=True)
            m_c += st["component_edges"]
        per_root, _ = time_roots(G, rs, d, p, rb.make_opts(), steps)
        single_ms += sum(per_root)
    M.bfs(roots, depth=depth, parent=parent)  # capture
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        M.bfs(roots, depth=depth, parent=parent)  # replay
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    log("# multi: 32 graphs x 16 roots: %.2f ms batched vs %.2f ms single-root" % (ms, single_ms))
    return {"value": m_c / (ms * 1e-3) / 1e9, "unit": "GTEPS (aggregate)",
            "ms_per_batch": ms, "single_root_ms_sum": single_ms,
            "single_root_gteps": m_c / (single_ms * 1e-3) / 1e9,
            "vs_single_root": single_ms / ms, "graphs": 32, "roots_per_graph": 16,
            "scales": "12..20", "tuning": tuned}


ABLATION_GRAPHS = {
    "kron22": ("kronecker", 22, 1022),
    "kron24": ("kronecker", 24, 1024),
    "kron26": ("kronecker", 26, 1026),
    "chunglu": ("chung-lu", 50_000_000, 4000),
}


def ablation(rb, graphgen, args):
    """Locality study: the same searches on the graph as generated (random
    labels), after RCM, and after partial RCM (variant "p<ratio>", e.g. p0.25:
    the first ceil(ratio * n+) vertices of the Cuthill-McKee sequence
    reordered, p0 only moving isolated vertices to the end), on Kronecker
    scales 22-26 and the 52.5 M-vertex Chung-Lu graph.  One JSON line per
    (graph, variant)."""
    import torch
    names = args.ablation_graphs.split(",")
    variants = args.ablation_variants.split(",")
    cache = rb.TuningCache(args.tuning_cache)
    arch = rb.device_info()["arch"]
    for name in names:
        kind, size, seed = ABLATION_GRAPHS[name]
        if kind == "kronecker":
            off, cols = graphgen.kronecker_csr_device(size, 16, seed)
        else:
            off, cols = graphgen.chung_lu_csr_device(size, size // 20, seed=seed)
        roots = graphgen.sample_roots_device(off, args.ablation_roots, args.root_seed)
        n = off.numel() - 1
        depth = torch.empty(n, dtype=torch.int32, device="cuda")
        parent = torch.empty(n, dtype=torch.int32, device="cuda")
        for variant in variants:
            G = rb.Graph(off, cols)
            rcm_ms = None
            if variant == "rcm":
                _, rcm_ms = G.rcm_reorder(want_perm=False)
            elif variant.startswith("p"):
                _, rcm_ms = G.rcm_reorder(want_perm=False, partial=float(variant[1:]))
            elif variant != "original":
                raise ValueError("unknown variant %r" % variant)
            reordered = variant != "original"
            t = cache.get(rb.tuning_key(arch, "kronecker", n, rb.TUNE_SINGLE))
            if t is not None:
                G.set_tuning(t)
            plain = rb.make_opts(alpha=args.alpha, beta=args.beta)
            timed = rb.make_opts(alpha=args.alpha, beta=args.beta, timing=True)
            stats = [G.bfs(r, depth, parent, opts=plain, stats=True)[2] for r in roots]
            G.timings()
            per_root_ms, _ = time_roots(G, roots, depth, parent, timed, args.steps)
            kernel_ms, total_ms = G.timings()
            G.check()
            info = G.info()
            # load balance: work per workgroup in the heaviest top-down and
            # bottom-up levels of the first root
            _, _, st0 = G.bfs(roots[0], depth, parent,
                              opts=rb.make_opts(alpha=args.alpha, beta=args.beta, wg_work=True),
                              stats=True)
            W = G.wg_work()
            balance = {}
            for dname, dval in (("td", 0), ("bu", 1)):
                lv = [d for d in range(W.shape[0]) if st0["dir"][d] == dval]
                if not lv:
                    continue
                d = max(lv, key=lambda x: int(W[x].sum()))
                row = W[d].astype(float)
                mean = float(row.mean())
                balance[dname] = {"level": d, "entries": int(row.sum()), "workgroups": len(row),
                                  "max_over_mean": float(row.max() / mean) if mean else None,
                                  "min_over_mean": float(row.min() / mean) if mean else None,
                                  "cov": float(row.std() / mean) if mean else None}
            m_c = [st["component_edges"] for st in stats]
            n_sweep = info["n_plus"] if reordered else n
            alg = sum(bfs_alg_bytes(st, n_sweep, original_ids=reordered)
                      for st in stats) / len(stats)
            k_ms = sum(kernel_ms) / len(kernel_ms)
            print(json.dumps({
                "ablation": name, "variant": variant, "n": n, "nnz": info["nnz"],
                "n_plus": info["n_plus"], "roots": len(roots),
                "gteps": hmean_gteps(m_c, per_root_ms),
                "gteps_search_kernel_only": hmean_gteps(m_c * args.steps, kernel_ms),
                "kernel_ms_avg": k_ms,
                "output_ms_avg": (sum(total_ms) - sum(kernel_ms)) / len(kernel_ms),
                "levels_avg": sum(st["levels"] for st in stats) / len(stats),
                "edges_examined_avg": sum(sum(st["edges"][:st["levels"]]) for st in stats)
                / len(stats),
                "alg_bytes_avg": alg, "achieved_gbs": alg / (k_ms * 1e-3) / 1e9,
                "rcm_ms": rcm_ms, "rcm_keep": info["rcm_keep"], "wg_balance": balance,
                "tuning": G.get_tuning()}), flush=True)
            G.close()
            del G
            # the allocator keeps its blocks between variants, so each RCM's
            # time is that of its kernels rather than of fresh hipMallocs
        del off, cols, roots, depth, parent
        torch.cuda.empty_cache()


def ab_grid(rb, graphgen, args):
    """Grid search of the alpha/beta rule on MI355X: the plain search over
    the scale-26 graph's roots for every (alpha, beta) pair; one JSON line per
    pair (harmonic-mean GTEPS and mean search-kernel time)."""
    import torch
    off, cols = graphgen.kronecker_csr_device(args.scale, args.edgefactor, args.seed)
    roots = graphgen.sample_roots_device(off, args.ablation_roots, args.root_seed)
    G = rb.Graph(off, cols)
    del off, cols
    torch.cuda.empty_cache()
    G.rcm_reorder(want_perm=False)
    cache = rb.TuningCache(args.tuning_cache)
    t = cache.get(rb.tuning_key(rb.device_info()["arch"], "kronecker", G.n, rb.TUNE_SINGLE))
    if t is not None:
        G.set_tuning(t)
    n = G.n
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    m_c = [G.bfs(r, depth, parent, stats=True)[2]["component_edges"] for r in roots]
    for a in [int(x) for x in args.ab_alphas.split(",")]:
        for b in [int(x) for x in args.ab_betas.split(",")]:
            timed = rb.make_opts(alpha=a, beta=b, timing=True)
            G.timings()
            per_root_ms, _ = time_roots(G, roots, depth, parent, timed, args.steps)
            kernel_ms, _ = G.timings()
            print(json.dumps({"alpha": a, "beta": b, "gteps": hmean_gteps(m_c, per_root_ms),
                              "kernel_ms_avg": sum(kernel_ms) / len(kernel_ms),
                              "roots": len(roots)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1026)
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--root-seed", type=int, default=7)
    ap.add_argument("--alpha", type=int, default=14)
    ap.add_argument("--beta", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-certify", action="store_true",
                    help="skip the on-device certificate of every root's output")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the built-in launch parameters instead of autotuned ones")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner even where the cache has an entry, and store it")
    ap.add_argument("--tuning-cache", default=DEFAULT_TUNING_CACHE,
                    help="JSON file of autotuned parameters (read, and written on a miss)")
    ap.add_argument("--tune-roots", type=int, default=8)
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--ablation", action="store_true",
                    help="run the locality study (original labels against RCM) instead")
    ap.add_argument("--ablation-graphs", default="kron22,kron24,kron26,chunglu")
    ap.add_argument("--ablation-variants", default="original,rcm")
    ap.add_argument("--ablation-roots", type=int, default=16)
    ap.add_argument("--rcm-only", action="store_true",
                    help="generate the graph, time its RCM relabelling, print one JSON line")
    ap.add_argument("--ab-grid", action="store_true",
                    help="run the alpha/beta grid search of the plain search instead")
    ap.add_argument("--ab-alphas", default="2,4,8,14,24,48,96")
    ap.add_argument("--ab-betas", default="6,12,24,48,96")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (profiler calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen
    import paper_2012_10026_amd as rb

    torch.cuda.set_device(0)
    if args.ablation:
        ablation(rb, graphgen, args)
        return
    if args.ab_grid:
        ab_grid(rb, graphgen, args)
        return
    if args.rcm_only:
        # the relabelling alone (for kernel traces of its passes)
        off, cols = graphgen.kronecker_csr_device(args.scale, args.edgefactor, args.seed)
        G = rb.Graph(off, cols)
        del off, cols
        torch.cuda.empty_cache()
        _, rcm_ms = G.rcm_reorder(want_perm=False)
        info = G.info()
        print(json.dumps({"rcm_ms": rcm_ms, "scale": args.scale, "n": info["n"],
                          "nnz": info["nnz"], "n_plus": info["n_plus"]}), flush=True)
        return
    dev = rb.device_info()
    t0 = time.perf_counter()
    off, cols = graphgen.kronecker_csr_device(args.scale, args.edgefactor, args.seed)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    roots = graphgen.sample_roots_device(off, args.roots, args.root_seed)
    # the autotuner samples its own roots (another seed) from the same graph
    tune_roots = graphgen.sample_roots_device(off, 64, args.root_seed + 1000)
    log("# generated scale %d: n=%d nnz=%d in %.1fs" % (args.scale, off.numel() - 1,
                                                        cols.numel(), t_gen))
    G = rb.Graph(off, cols)
    keep_host = not args.no_cpu
    if not keep_host:
        del off, cols
        torch.cuda.empty_cache()
    _, rcm_ms = G.rcm_reorder(want_perm=False)
    info = G.info()
    log("# rcm %.1f ms, n_plus=%d" % (rcm_ms, info["n_plus"]))

    n = info["n"]
    nroot = len(roots)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    plain = rb.make_opts(alpha=args.alpha, beta=args.beta)
    timed = rb.make_opts(alpha=args.alpha, beta=args.beta, timing=True)

    tuning = {}
    cache = None if args.no_tune else rb.TuningCache(args.tuning_cache)
    if cache is not None:
        tuning["single"] = tuned_leg(rb, G, tune_roots[:args.tune_roots], cache, "kronecker",
                                     rb.TUNE_SINGLE, args.retune, opts=plain)

    # untimed pass: per-root counters (deterministic) for TEPS and the bytes model
    stats = []
    for r in roots:
        _, _, st = G.bfs(r, depth, parent, opts=plain, stats=True)
        stats.append(st)
    for _ in range(args.warmup):
        for r in roots:
            G.bfs(r, depth, parent, opts=plain)
    G.check()
    G.timings()  # clear

    per_root_ms, t_wall = time_roots(G, roots, depth, parent, timed, args.steps)
    G.check()
    kernel_ms, total_ms = G.timings()

    # outside the timed region: every root's output through the on-device
    # O(nnz) certificate, and the Graph500-style count of generated tuples
    # with both endpoints reached (self-loops and duplicates included)
    certified = None if args.no_certify else 0
    tuples = []
    for i, r in enumerate(roots):
        # a root that the previous search reached has the same component,
        # hence the same tuple count
        same = i > 0 and int(depth[r].item()) >= 0
        G.bfs(r, depth, parent, opts=plain)
        if certified is not None:
            code = G.certify(r, depth, parent)
            if code != 0:
                raise RuntimeError("certificate failed for root %d: code %d" % (r, code))
            certified += 1
        tuples.append(tuples[-1] if same else graphgen.kronecker_tuples_reached_device(
            args.scale, depth, args.edgefactor, args.seed))
    if certified is not None:
        log("# certified %d roots on the device" % certified)

    m_c = [st["component_edges"] for st in stats]
    hmean = hmean_gteps(m_c, per_root_ms)
    ms_per_step = t_wall * 1e3 / args.steps
    n_sweep = info["n_plus"]
    alg = [bfs_alg_bytes(st, n_sweep) for st in stats]
    k_avg_ms = sum(kernel_ms) / max(1, len(kernel_ms))
    bytes_avg = sum(alg[i % nroot] for i in range(len(kernel_ms))) / max(1, len(kernel_ms))
    achieved = bytes_avg / (k_avg_ms * 1e-3) / 1e9
    hmean_internal = hmean_gteps(m_c * args.steps, kernel_ms)

    out = {
        "metric": "GTEPS (harmonic mean, 64 roots) Kronecker scale %d" % args.scale,
        "value": hmean,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "kronecker scale %d edgefactor %d (A,B,C)=(0.57,0.19,0.19) "
                               "seed %d, RCM-relabelled, %d roots, plain heuristic "
                               "alpha=%d beta=%d, outputs in original IDs"
                               % (args.scale, args.edgefactor, args.seed, nroot, args.alpha,
                                  args.beta),
                   "n": n, "nnz": info["nnz"], "n_plus": n_sweep},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(
                         "kronecker scale %d seed %d, %d roots, alpha %d beta %d"
                         % (args.scale, args.seed, nroot, args.alpha, args.beta)),
                     "kernel": "bfs_persistent_kernel", "kernel_avg_ms": k_avg_ms,
                     "alg_bytes_avg": bytes_avg},
        "rcm_ms": rcm_ms,
        "gen_s": t_gen,
        "gteps_search_kernel_only": hmean_internal,
        "gteps_graph500_tuples": hmean_gteps(tuples, per_root_ms),
        "giant_component_root_fraction": sum(1 for m in m_c if m == max(m_c)) / nroot,
        "translate_ms_avg": (sum(total_ms) - sum(kernel_ms)) / max(1, len(kernel_ms)),
        "levels_avg": sum(st["levels"] for st in stats) / nroot,
        "certified_roots": certified,
        "device": dev,
    }

    if not args.no_batch:
        # 64 roots bit-parallel on the same graph, one call
        if cache is not None:
            tuning["batch"] = tuned_leg(rb, G, tune_roots, cache, "kronecker", rb.TUNE_BATCH,
                                        args.retune, reps=1)
            torch.cuda.empty_cache()
        dB = torch.empty((nroot, n), dtype=torch.int32, device="cuda")
        pB = torch.empty((nroot, n), dtype=torch.int32, device="cuda")
        G.bfs_batch(roots, dB, pB)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            G.bfs_batch(roots, dB, pB)
        e1.record()
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / args.steps
        d_last, p_last = G.bfs(roots[-1], depth, parent)
        ok = bool(torch.equal(dB[nroot - 1], d_last) and torch.equal(pB[nroot - 1], p_last))
        out["batched"] = {"value": sum(m_c) / (ms_b * 1e-3) / 1e9,
                          "unit": "GTEPS (aggregate, 64 roots bit-parallel, one launch)",
                          "ms_per_batch": ms_b, "vs_plain": sum(per_root_ms) / ms_b,
                          "last_row_equals_single_root": ok}
        log("# batched: %.2f ms for 64 roots (%.1f GTEPS aggregate)"
            % (ms_b, out["batched"]["value"]))
        del dB, pB
        torch.cuda.empty_cache()
    if not args.no_learned:
        blob, info_sw = train_switch(rb, graphgen)
        rb.switch_load(blob)
        learned = rb.make_opts(rb.DIR_LEARNED, alpha=args.alpha, beta=args.beta)
        for r in roots[:4]:
            G.bfs(r, depth, parent, opts=learned)
        per_root_l, _ = time_roots(G, roots, depth, parent, learned, args.steps)
        gl = hmean_gteps(m_c, per_root_l)
        out["learned"] = {"value": gl, "unit": "GTEPS", "vs_plain": gl / hmean,
                          "training": info_sw,
                          "schedule_costs_8_roots": schedule_costs(rb, G, roots[:8], learned,
                                                                   plain)}
        log("# learned: %.1f GTEPS (plain %.1f)" % (gl, hmean))
        out["learned"]["heavy_tail"] = heavy_tail_switch(rb, graphgen, args.steps, args.alpha,
                                                         args.beta)
    if not args.no_multi:
        out["multi"] = multi_batch(rb, graphgen, args.steps, cache, args.retune)
    if tuning:
        out["tuning"] = tuning
    if args.copy_calibration_gib > 0:
        nb = int(args.copy_calibration_gib * (1 << 30))
        a = torch.ones(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nb
        del a, b
    if keep_host:
        out["cpu_baseline"] = cpu_baseline(off, cols, roots, args.cpu_budget)
        model, ncpu = host_cpu()
        out["cpu_baseline"]["host_cpu"] = model
        out["cpu_baseline"]["host_threads_available"] = ncpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
