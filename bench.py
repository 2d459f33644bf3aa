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


def cpu_baseline(off, cols, off_r, cols_r, perm, roots, gpu_rcm_ms, budget_s=30.0):
    """The oracle timed on the host's cores, on bounded samples of the same
    graph, as three single-threaded tasks run side by side (one host thread
    each): its BFS from the first roots in the original labels (the reported
    value); the same roots' BFS on the RCM-relabelled CSR the library built
    (the CPU side of the locality study); and its RCM (Algorithm 3) of the
    whole graph, next to the GPU's RCM time on the same graph."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    def bfs_leg(o, c, rs):
        t_all, edges_all, used = 0.0, 0, 0
        for r in rs:
            t0 = time.perf_counter()
            depth, _, _ = oracle.bfs(o, c, int(r))
            t_all += time.perf_counter() - t0
            edges_all += oracle.component_edges(o, depth)
            used += 1
            if t_all > budget_s * 0.5:
                break
        return t_all, edges_all, used

    def rcm_leg():
        t0 = time.perf_counter()
        oracle.rcm(off, cols)
        return time.perf_counter() - t0

    with ThreadPoolExecutor(3) as ex:
        f_orig = ex.submit(bfs_leg, off, cols, roots)
        f_rl = ex.submit(bfs_leg, off_r, cols_r, [perm[r] for r in roots])
        f_rcm = ex.submit(rcm_leg)
        t_o, e_o, n_o = f_orig.result()
        t_r, e_r, n_r = f_rl.result()
        t_rcm = f_rcm.result()
    v_o = e_o / t_o / 1e9
    v_r = e_r / t_r / 1e9
    return {"value": v_o, "unit": "GTEPS", "cores": 3, "kind": "oracle",
            "sample": "oracle BFS (single thread, original labels) from the first %d of the "
                      "roots on the same graph, %.1f s; run beside the two tasks below, each "
                      "on its own host thread" % (n_o, t_o),
            "rcm_labels": {"value": v_r, "unit": "GTEPS", "vs_original_labels": v_r / v_o,
                           "sample": "oracle BFS (single thread) from the first %d roots on "
                                     "the RCM-relabelled CSR, %.1f s" % (n_r, t_r)},
            "rcm": {"oracle_s": t_rcm, "gpu_ms": gpu_rcm_ms,
                    "gpu_speedup": t_rcm / (gpu_rcm_ms * 1e-3),
                    "sample": "oracle RCM (Algorithm 3, single thread) of the whole graph"}}


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


def certify_roots(G, roots, depth, parent, opts):
    """Outside the timed region: each root's search again, its output through
    the on-device O(nnz) certificate; raises on a failure.  Returns the count."""
    for r in roots:
        G.bfs(r, depth, parent, opts=opts)
        code = G.certify(r, depth, parent)
        if code != 0:
            raise RuntimeError("certificate failed for root %d: code %d" % (r, code))
    return len(roots)


def certify_rows(G, roots, dB, pB):
    """Every row of a batch's root-major outputs through the on-device
    certificate; raises on a failure.  Returns the count."""
    for j, r in enumerate(roots):
        code = G.certify(r, dB[j], pB[j])
        if code != 0:
            raise RuntimeError("certificate failed for batch row %d: code %d" % (j, code))
    return len(roots)


def hmean_gteps(m_c, per_root_ms):
    teps = [m / (t * 1e-3) for m, t in zip(m_c, per_root_ms)]
    return len(teps) / sum(1.0 / x for x in teps) / 1e9


SWITCH_TRAIN_GRAPHS = (
    # (family, size, seed, roots): Kronecker scales 18-24 (edge factor 16)
    # and Chung-Lu graphs of exponents 2.1 and 2.5; none is a graph the
    # benchmark measures on
    [("kronecker", s, 2000 + 10 * s + j, 32) for s in (18, 20, 22) for j in range(4)] +
    [("kronecker", 24, 2240 + j, 16) for j in range(2)] +
    [("chung-lu", n, 5000 + 10 * j + 21, 40, 2.1)
     for n in (300_000, 1_000_000, 3_000_000) for j in range(4)] +
    [("chung-lu", n, 5000 + 10 * j + 25, 32, 2.5) for n in (300_000, 1_000_000) for j in range(2)] +
    [("chung-lu", 10_000_000, 5100 + j, 16, 2.1) for j in range(2)])
# held-out graphs on which the decision margin is chosen: the training
# families, and one Kronecker scale-26 and one 52.5M-vertex Chung-Lu graph of
# other seeds than the measured ones (the sizes the switch is deployed at)
SWITCH_VALIDATION_GRAPHS = [("kronecker", 24, 2299, 8), ("kronecker", 26, 2626, 8),
                            ("chung-lu", 3_000_000, 5999, 8, 2.1),
                            ("chung-lu", 300_000, 5998, 8, 2.1),
                            ("chung-lu", 1_000_000, 5997, 8, 2.5),
                            ("chung-lu-52.5M", 50_000_000, 4001, 8)]
SWITCH_NETS = 4
SWITCH_MARGINS = (0.05, 0.1, 0.25, 0.5, 1.0, 1e9)


def switch_graph(rb, graphgen, spec):
    if spec[0] == "kronecker":
        _, s, seed, k = spec
        off, cols = graphgen.kronecker_csr_device(s, 16, seed)
    elif spec[0] == "chung-lu-52.5M":
        _, n, seed, k = spec
        off, cols = graphgen.chung_lu_csr_device(n, n // 20, seed=seed)
    else:
        _, n, seed, k, g = spec
        off, cols = graphgen.chung_lu_csr_device(n, n // 20, seed=seed, gamma=g,
                                                 mean_deg=30.0 if g < 2.3 else 10.0,
                                                 max_deg=n / 15.0)
    roots = graphgen.sample_roots_device(off, k, 7)
    G = rb.Graph(off, cols)
    del off, cols
    G.rcm_reorder(want_perm=False)
    return G, roots


def kernel_ms_sum(rb, G, roots, opts, reps=3):
    """Sum over roots of the median search-kernel time."""
    tot = 0.0
    for r in roots:
        tot += statistics.median(G.bfs(r, opts=opts, stats=True)[2]["ms_kernel"]
                                 for _ in range(reps))
    return tot


def train_switch(rb, graphgen):
    """Costs of both directions at every level (rbfs_collect_level_samples:
    the alpha/beta path up to the level, each direction there, the alpha/beta
    rule after it; the time from the level to the end of the search) on
    Kronecker graphs of scales 18-24 and on Chung-Lu graphs, GPU training of
    one network for every graph family (several, from their own initial
    weights and sample orders), and the network and decision margin chosen
    on held-out graphs of the same families and sizes: the pair whose worst
    ratio of learned to alpha/beta search time over them is smallest (a
    margin that never lets the network decide is among the candidates), the
    geometric mean breaking near-ties.  Returns the switch blob and a
    summary."""
    import numpy as np
    import torch
    rows = []
    t0 = time.perf_counter()
    for spec in SWITCH_TRAIN_GRAPHS:
        G, roots = switch_graph(rb, graphgen, spec)
        rows.append(rb.collect_level_samples(G, roots, reps=3, cap=16384))
        G.close()
        torch.cuda.empty_cache()
    rows = np.vstack(rows)
    t_collect = time.perf_counter() - t0
    # several networks (their own initial weights and sample orders), since
    # one trained network sometimes mispredicts a family badly
    t0 = time.perf_counter()
    nets = []
    for j in range(SWITCH_NETS):
        order = graphgen.epoch_orders(rows.shape[0], 200, 1 + j)
        w, curve = rb.mlp_train(rows[:, :10], graphgen.mlp_init_weights(j).astype(np.float32),
                                order, batch=64, lr=3e-3)
        nets.append((w, curve))
    t_train = time.perf_counter() - t0
    # every (network, margin) on the validation graphs; a margin that never
    # lets the network decide is timed once
    t0 = time.perf_counter()
    cands = [(j, m) for j in range(SWITCH_NETS) for m in SWITCH_MARGINS if m < 1e8]
    cands.append((0, max(SWITCH_MARGINS)))
    blobs = {c: rb.make_switch_blob(nets[c[0]][0], rows, margin=c[1]) for c in cands}
    ratios = {c: [] for c in cands}
    for spec in SWITCH_VALIDATION_GRAPHS:
        G, roots = switch_graph(rb, graphgen, spec)
        for r in roots[:2]:
            G.bfs(r)
        # root by root, alpha/beta and every candidate in turn, so that a
        # drift of the clocks over the run weighs on all of them alike
        t_ab, t_c = 0.0, {c: 0.0 for c in cands}
        for r in roots:
            t_ab += kernel_ms_sum(rb, G, [r], rb.make_opts())
            for c in cands:
                rb.switch_load(blobs[c])
                t_c[c] += kernel_ms_sum(rb, G, [r], rb.make_opts(rb.DIR_LEARNED))
        for c in cands:
            ratios[c].append(t_c[c] / t_ab)
        G.close()
        torch.cuda.empty_cache()
    # the smallest worst ratio; candidates within 1.5 % of it (timing noise)
    # are ranked by their geometric mean ratio
    best_worst = min(max(ratios[c]) for c in cands)
    pick = min((c for c in cands if max(ratios[c]) <= best_worst + 0.015),
               key=lambda c: sum(math.log(x) for x in ratios[c]))
    w, curve = nets[pick[0]]
    margin = pick[1]
    t_val = time.perf_counter() - t0
    log("# switch: %d samples (%.1f s), %d networks trained %.2f s, loss %.3f -> %.3f; network "
        "%d, margin %g (worst learned/alpha-beta time on validation %.3f)"
        % (rows.shape[0], t_collect, SWITCH_NETS, t_train, curve[0], curve[-1], pick[0], margin,
           max(ratios[pick])))
    return rb.make_switch_blob(w, rows, margin=margin), {
        "samples": int(rows.shape[0]),
        "train_graphs": "kronecker scales 18,20,22 x 4 (32 roots each), 24 x 2 (16 roots); "
                        "chung-lu n = 0.3M, 1M, 3M x 4, exponent 2.1, mean degree 30 (40 roots "
                        "each), 10M x 2 (16 roots); n = 0.3M, 1M x 2, exponent 2.5, mean degree "
                        "10 (32 roots)",
        "collect_s": t_collect, "train_s": t_train, "validate_s": t_val, "epochs": 200,
        "networks": SWITCH_NETS, "network": pick[0],
        "loss_first": float(curve[0]), "loss_last": float(curve[-1]),
        "margin": margin,
        "validation_learned_over_alpha_beta_time": {
            ("net%d margin %g" % c): [round(x, 4) for x in ratios[c]] for c in cands},
        "validation_graphs": "kronecker 24 seed 2299, kronecker 26 seed 2626; chung-lu 3M and "
                             "0.3M exponent 2.1; chung-lu 1M exponent 2.5; chung-lu 52.5M seed "
                             "4001 (8 roots each)"}


def schedule_costs(rb, G, roots, learned_opts, plain_opts, reps=3):
    """Per root, search-kernel times (median of reps) of three schedules run
    end to end: alpha/beta, learned, and the per-level best (at each level
    the direction with the smaller measured cost from there to the end, the
    alpha/beta path before it and the alpha/beta rule after it, from
    rbfs_collect_level_samples), run with DIR_SCHEDULE."""
    tot = {"alpha_beta_ms": 0.0, "learned_ms": 0.0, "best_schedule_ms": 0.0}
    agree_l = agree_h = nlev = 0
    for r in roots:
        rows = rb.collect_level_samples(G, [r], reps=3)
        best = {}
        for x in rows:  # the first row of a level follows the alpha/beta path
            best.setdefault(int(x[10]), 0 if x[8] <= x[9] else 1)
        sched = [0] + [best.get(lv, 0) for lv in range(1, max(best, default=0) + 1)]

        def t_of(opts):
            st = None
            ts = []
            for _ in range(reps):
                _, _, st = G.bfs(r, opts=opts, stats=True)
                ts.append(st["ms_kernel"])
            return statistics.median(ts), st
        t_h, sh = t_of(plain_opts)
        t_l, sl = t_of(learned_opts)
        t_b, _ = t_of(rb.make_opts(rb.DIR_SCHEDULE, alpha=plain_opts.alpha,
                                   beta=plain_opts.beta, schedule=sched))
        tot["alpha_beta_ms"] += t_h
        tot["learned_ms"] += t_l
        tot["best_schedule_ms"] += t_b
        for lv in range(1, len(sched)):
            agree_l += int(lv < len(sl["dir"]) and sl["dir"][lv] == sched[lv])
            agree_h += int(lv < len(sh["dir"]) and sh["dir"][lv] == sched[lv])
            nlev += 1
    tot["learned_vs_alpha_beta"] = tot["alpha_beta_ms"] / tot["learned_ms"]
    tot["best_schedule_vs_alpha_beta"] = tot["alpha_beta_ms"] / tot["best_schedule_ms"]
    tot["learned_agrees_with_best_frac"] = agree_l / max(1, nlev)
    tot["alpha_beta_agrees_with_best_frac"] = agree_h / max(1, nlev)
    tot["roots"] = len(roots)
    return tot


def heavy_tail_switch(rb, graphgen, steps, alpha, beta):
    """The learned switch (the network loaded, not retrained) on a power-law
    graph (Chung-Lu, 300000 vertices, exponent 2.1, mean degree 30) where
    the alpha/beta thresholds stay bottom-up too long at the tail, against
    the alpha/beta rule; outputs certified."""
    import torch
    off, cols = graphgen.chung_lu_csr(300000, 15000, seed=9, gamma=2.1, mean_deg=30.0,
                                      max_deg=20000.0)
    G = rb.Graph(off, cols)
    G.rcm_reorder(want_perm=False)
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
    certified = (certify_roots(G, roots, depth, parent, learned) +
                 certify_roots(G, roots, depth, parent, plain))
    out = {"graph": "chung-lu n=300000 exponent 2.1 mean degree 30 (seed 9, not trained on)",
           "certified_outputs": certified,
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
    outs = M.bfs(roots, depth=depth, parent=parent)
    rows_ok = sum(certify_rows(G, rs, dB, pB) for G, rs, (dB, pB) in zip(Gs, roots, outs))
    log("# multi: 32 graphs x 16 roots: %.2f ms batched vs %.2f ms single-root" % (ms, single_ms))
    return {"value": m_c / (ms * 1e-3) / 1e9, "unit": "GTEPS (aggregate)",
            "ms_per_batch": ms, "single_root_ms_sum": single_ms,
            "single_root_gteps": m_c / (single_ms * 1e-3) / 1e9,
            "vs_single_root": single_ms / ms, "graphs": 32, "roots_per_graph": 16,
            "scales": "12..20", "certified_rows": rows_ok, "tuning": tuned}


def chung_lu_leg(rb, graphgen, args, cache, blob):
    """The power-law configuration: Chung-Lu, 50 M vertices with exponent 2.1,
    mean degree 30 and largest expected degree 2 M, plus 2.5 M isolated
    vertices (dropped to the end by RCM); 64 roots.  Plain heuristic search,
    the learned switch with the network trained on Kronecker graphs (no
    retraining), and the 64-root batch, each timed as on the Kronecker graph
    and every output certified on the device."""
    import torch
    t0 = time.perf_counter()
    off, cols = graphgen.chung_lu_csr_device(50_000_000, 2_500_000, seed=4000)
    roots = graphgen.sample_roots_device(off, args.roots, args.root_seed)
    G = rb.Graph(off, cols)
    del off, cols
    torch.cuda.empty_cache()
    t_gen = time.perf_counter() - t0
    _, rcm_ms = G.rcm_reorder(want_perm=False)
    info = G.info()
    n = info["n"]
    if cache is not None:
        # no Chung-Lu entry: the Kronecker setting of the same size bucket
        for kind in (rb.TUNE_SINGLE, rb.TUNE_BATCH):
            t = cache.get(rb.tuning_key(rb.device_info()["arch"], "kronecker", n, kind))
            if t is not None:
                G.set_tuning(t, kind)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    plain = rb.make_opts(alpha=args.alpha, beta=args.beta)
    stats = [G.bfs(r, depth, parent, opts=plain, stats=True)[2] for r in roots]
    m_c = [st["component_edges"] for st in stats]
    for r in roots:
        G.bfs(r, depth, parent, opts=plain)
    per_p, _ = time_roots(G, roots, depth, parent, plain, args.steps)
    G.check()
    gp = hmean_gteps(m_c, per_p)
    out = {"graph": "chung-lu n=%d (50M power-law, exponent 2.1, mean degree 30, max expected "
                    "degree 2M, + 2.5M isolated) seed 4000" % n,
           "nnz": info["nnz"], "n_plus": info["n_plus"], "gen_s": t_gen, "rcm_ms": rcm_ms,
           "roots": len(roots),
           "giant_component_root_fraction": sum(1 for m in m_c if m == max(m_c)) / len(m_c),
           "plain": {"value": gp, "unit": "GTEPS",
                     "certified_roots": certify_roots(G, roots, depth, parent, plain)}}
    log("# chung-lu: rcm %.1f ms, plain %.1f GTEPS" % (rcm_ms, gp))
    if blob is not None:
        rb.switch_load(blob)
        learned = rb.make_opts(rb.DIR_LEARNED, alpha=args.alpha, beta=args.beta)
        for r in roots[:4]:
            G.bfs(r, depth, parent, opts=learned)
        per_l, _ = time_roots(G, roots, depth, parent, learned, args.steps)
        gl = hmean_gteps(m_c, per_l)
        out["learned"] = {"value": gl, "unit": "GTEPS", "vs_plain": gl / gp,
                          "network": "the one trained in this run (Kronecker scales 18-24 and Chung-Lu graphs of 0.3-10M vertices), not retrained for this graph",
                          "certified_roots": certify_roots(G, roots, depth, parent, learned)}
        log("# chung-lu: learned %.1f GTEPS (%.3fx plain)" % (gl, gl / gp))
    if not args.no_batch:
        del depth, parent
        dB = torch.empty((len(roots), n), dtype=torch.int32, device="cuda")
        pB = torch.empty((len(roots), n), dtype=torch.int32, device="cuda")
        G.bfs_batch(roots, dB, pB)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            G.bfs_batch(roots, dB, pB)
        e1.record()
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / args.steps
        out["batched"] = {"value": sum(m_c) / (ms_b * 1e-3) / 1e9,
                          "unit": "GTEPS (aggregate, 64 roots bit-parallel, one launch)",
                          "ms_per_batch": ms_b, "vs_plain": sum(per_p) / ms_b,
                          "certified_rows": certify_rows(G, roots, dB, pB)}
        log("# chung-lu: batched %.2f ms (%.1f GTEPS aggregate)" % (ms_b, out["batched"]["value"]))
        del dB, pB
    G.close()
    torch.cuda.empty_cache()
    return out


ABLATION_GRAPHS = dict(
    [("kron%d" % s, ("kronecker", s, 1000 + s)) for s in range(21, 27)] +
    [("chunglu", ("chung-lu", 50_000_000, 4000))])


def ablation(rb, graphgen, args):
    """Ablation and locality study (section 4.3 ablation, section 4.4): the
    same searches on the graph as generated (random labels), after RCM, and
    after partial RCM (variant "p<ratio>", e.g. p0.25: the first
    ceil(ratio * n+) vertices of the Cuthill-McKee sequence reordered, p0
    only moving isolated vertices to the end), each with the load-balanced
    kernels or, with the suffix "-nolb", without load balancing (whole rows
    per wave top-down, equal vertex ranges without stealing bottom-up), on
    Kronecker scales 21-26 and the 52.5 M-vertex Chung-Lu graph.  One JSON
    line per (graph, variant), with the vertices each bottom-up level sweeps
    (the unvisited part of its sweep range: the graph before RCM, the root's
    component after it), the analogue of the shrinking partitions of
    section 3.4."""
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
            nolb = variant.endswith("-nolb")
            base = variant[:-len("-nolb")] if nolb else variant
            if base == "rcm":
                _, rcm_ms = G.rcm_reorder(want_perm=False)
            elif base.startswith("p"):
                _, rcm_ms = G.rcm_reorder(want_perm=False, partial=float(base[1:]))
            elif base != "original":
                raise ValueError("unknown variant %r" % variant)
            reordered = base != "original"
            t = cache.get(rb.tuning_key(arch, "kronecker", n, rb.TUNE_SINGLE))
            if t is not None:
                G.set_tuning(t)
            plain = rb.make_opts(alpha=args.alpha, beta=args.beta, no_balance=nolb)
            timed = rb.make_opts(alpha=args.alpha, beta=args.beta, timing=True, no_balance=nolb)
            stats = [G.bfs(r, depth, parent, opts=plain, stats=True)[2] for r in roots]
            G.timings()
            per_root_ms, _ = time_roots(G, roots, depth, parent, timed, args.steps)
            kernel_ms, total_ms = G.timings()
            G.check()
            info = G.info()
            # load balance: work per workgroup in the heaviest top-down and
            # bottom-up levels of the first root
            _, _, st0 = G.bfs(roots[0], depth, parent,
                              opts=rb.make_opts(alpha=args.alpha, beta=args.beta, wg_work=True,
                                                no_balance=nolb),
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
            # vertices each bottom-up level of the first root sweeps: the
            # unvisited part of the whole graph before RCM (every word is
            # swept), of the root's component after it (the sweep covers the
            # component; later levels walk the list the last one left)
            scope = st0["reached"] if (reordered and base == "rcm") else n_sweep
            seen, bu_swept = 0, []
            for d in range(st0["levels"]):
                if st0["dir"][d] == 1:
                    bu_swept.append({"level": d, "vertices": scope - seen,
                                     "entries": st0["edges"][d]})
                seen += st0["nf"][d]
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
                "bu_swept_root0": bu_swept, "load_balance": not nolb,
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
    ap.add_argument("--no-chunglu", action="store_true",
                    help="skip the 52.5M-vertex Chung-Lu leg (plain, learned, batched)")
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
    ap.add_argument("--ablation-graphs",
                    default="kron21,kron22,kron23,kron24,kron25,kron26,chunglu")
    ap.add_argument("--ablation-variants", default="original-nolb,p0-nolb,rcm-nolb,rcm",
                    help="original, p<ratio> (partial RCM), rcm; suffix -nolb: without "
                         "load balancing")
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
    keep_host = not args.no_cpu
    csr_bytes = off.numel() * 8 + cols.numel() * 4
    if 2 * csr_bytes > 0.85 * dev["global_mem_bytes"]:
        # the device cannot hold the generator's CSR and the library's copy
        # at once (scale 30): the CSR goes through host memory
        if keep_host:
            raise SystemExit("this scale needs --no-cpu (the CSR is staged in host memory)")
        t1 = time.perf_counter()
        off_h, cols_h = off.cpu().numpy(), cols.cpu().numpy()
        del off, cols
        torch.cuda.empty_cache()
        G = rb.Graph(off_h, cols_h)
        del off_h, cols_h
        log("# graph created from host memory in %.1f s" % (time.perf_counter() - t1))
    else:
        G = rb.Graph(off, cols)
        if not keep_host:
            del off, cols
            torch.cuda.empty_cache()
    bw_orig = G.bandwidth()
    perm_t, rcm_ms = G.rcm_reorder(want_perm=keep_host)
    info = G.info()
    bw_rcm = G.bandwidth()
    log("# rcm %.1f ms, n_plus=%d, bandwidth %d -> %d" % (rcm_ms, info["n_plus"], bw_orig, bw_rcm))

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
        "bandwidth": {"original_labels": bw_orig, "rcm_labels": bw_rcm},
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
        rows_ok = certify_rows(G, roots, dB, pB)
        out["batched"] = {"value": sum(m_c) / (ms_b * 1e-3) / 1e9,
                          "unit": "GTEPS (aggregate, 64 roots bit-parallel, one launch)",
                          "ms_per_batch": ms_b, "vs_plain": sum(per_root_ms) / ms_b,
                          "certified_rows": rows_ok}
        log("# batched: %.2f ms for 64 roots (%.1f GTEPS aggregate)"
            % (ms_b, out["batched"]["value"]))
        del dB, pB
        torch.cuda.empty_cache()
    blob = None
    if not args.no_learned:
        blob, info_sw = train_switch(rb, graphgen)
        rb.switch_load(blob)
        learned = rb.make_opts(rb.DIR_LEARNED, alpha=args.alpha, beta=args.beta)
        for r in roots[:4]:
            G.bfs(r, depth, parent, opts=learned)
        per_root_l, _ = time_roots(G, roots, depth, parent, learned, args.steps)
        gl = hmean_gteps(m_c, per_root_l)
        out["learned"] = {"value": gl, "unit": "GTEPS", "vs_plain": gl / hmean,
                          "certified_roots": certify_roots(G, roots, depth, parent, learned),
                          "training": info_sw,
                          "schedule_costs_8_roots": schedule_costs(rb, G, roots[:8], learned,
                                                                   plain)}
        log("# learned: %.1f GTEPS (plain %.1f)" % (gl, hmean))
        out["learned"]["heavy_tail"] = heavy_tail_switch(rb, graphgen, args.steps, args.alpha,
                                                         args.beta)
    if not args.no_multi:
        out["multi"] = multi_batch(rb, graphgen, args.steps, cache, args.retune)
    if not args.no_chunglu:
        out["chung_lu"] = chung_lu_leg(rb, graphgen, args, cache, blob)
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
        log("# cpu baseline (oracle)")
        off_r, cols_r = G.csr()
        out["cpu_baseline"] = cpu_baseline(off.cpu().numpy(), cols.cpu().numpy(),
                                           off_r.cpu().numpy(), cols_r.cpu().numpy(),
                                           perm_t.cpu().numpy(), roots, rcm_ms, args.cpu_budget)
        del off_r, cols_r
        model, ncpu = host_cpu()
        out["cpu_baseline"]["host_cpu"] = model
        out["cpu_baseline"]["host_threads_available"] = ncpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
