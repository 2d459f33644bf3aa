"""fp64 reference of the direction-switch network -- TEST INFRASTRUCTURE ONLY.

Not in the paper (the paper tunes the alpha/beta switch of Algorithm 2 by grid
search, "Parameter Tuning"); this is the plain definition of the network the
learned switch uses:

    h1 = ReLU(W1 x + b1)  (8 -> 32)
    h2 = ReLU(W2 h1 + b2) (32 -> 32)
    y  = W3 h2 + b3       (32 -> 2)

loss of a batch B: (1/|B|) sum_s 1/2 ||y_s - t_s||^2, gradients by the chain
rule written out by hand, Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias
correction.  Parameters are one flat vector in the order W1 (32x8, row =
output unit), b1, W2 (32x32), b2, W3 (2x32), b3: 1410 values.
"""
import numpy as np

NIN, NHID, NOUT = 8, 32, 2
SIZES = [("W1", (NHID, NIN)), ("b1", (NHID,)), ("W2", (NHID, NHID)), ("b2", (NHID,)),
         ("W3", (NOUT, NHID)), ("b3", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(w):
    w = np.asarray(w, np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = w[o:o + k].reshape(shape)
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SIZES])


def forward(w, X):
    p = unpack(w)
    X = np.asarray(X, np.float64)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (X, a1, h1, a2, h2)


def loss_and_grad(w, samples):
    """Mean over the rows of 1/2 ||y - t||^2 and its gradient (flat)."""
    samples = np.asarray(samples, np.float64)
    X, T = samples[:, :NIN], samples[:, NIN:NIN + NOUT]
    B = X.shape[0]
    p = unpack(w)
    y, (X, a1, h1, a2, h2) = forward(w, X)
    err = y - T
    loss = 0.5 * np.sum(err * err) / B
    dy = err / B                      # dL/dy
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)


def train(samples, w0, order, batch=256, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam over the given per-epoch sample order; returns (w, loss curve)."""
    samples = np.asarray(samples, np.float64)
    w = np.asarray(w0, np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    t = 0
    curve = []
    order = np.asarray(order)
    n = samples.shape[0]
    for ep in range(order.shape[0]):
        total = 0.0
        for b0 in range(0, n, batch):
            idx = order[ep, b0:b0 + batch]
            loss, g = loss_and_grad(w, samples[idx])
            total += loss * len(idx)
            t += 1
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            w = w - lr * mh / (np.sqrt(vh) + eps)
        curve.append(total / n)
    return w, np.array(curve)


# ---------------------------------------------------------------------------
# The learned direction decision, taken before level d >= 1 (which expands
# the frontier F_d), written from the definition the library documents for
# its switch: the network's inputs are eight per-level features, its two
# outputs are predicted ln(microseconds) of level d run top-down (0) or
# bottom-up (1); the network decides only when the inputs lie inside the
# widened training range and its two predictions differ by at least the
# margin (ln microseconds, the blob's last value); otherwise the alpha/beta
# rule of Algorithm 2 (section 2.1,
# "Parameter Tuning"; integer form) decides.  The switch blob holds the 1410
# network parameters, then fmin[8], fmax[8], the largest training level and
# the margin.

OOD_WIDEN = 0.1           # the training range is widened by 10 % of its width
BLOB = NPARAMS + NIN + NIN + 2  # ... + largest training level + margin
FALLBACK_NONE, FALLBACK_OOD, FALLBACK_MARGIN = 0, 1, 2
_U32 = 2.0 ** -24         # unit roundoff of fp32
# Bound on the absolute error of one fp32 feature: each is at most a few
# correctly rounded fp32 operations (int -> float, log2, divide) on values of
# magnitude <= 2, so it is within a few times 2^-24 * 2 of the exact value;
# 1e-5 is a generous cover.
FEATURE_ERR = 1e-5


def features(nf, mf, mu, nu, nf_prev, level, cur_dir, n_sweep, nnz):
    """The eight inputs, exactly (fp64):
    f0 = log2(1+n_f)/log2(n), f1 = log2(1+m_f)/log2(nnz),
    f2 = log2(1+m_u)/log2(nnz), f3 = n_u/n,
    f4 = clamp(log2((1+m_f)/(1+m_u))/16, -2, 2), f5 = level/32,
    f6 = current direction (that of level d-1),
    f7 = clamp(log2((1+n_f)/(1+n_f_prev))/8, -2, 2);
    n = swept vertex count and nnz the adjacency entries, each at least 2 in
    the logarithms (n at least 1 in f3)."""
    lgn = np.log2(max(n_sweep, 2))
    lge = np.log2(max(nnz, 2))
    f = np.empty(NIN)
    f[0] = np.log2(1.0 + nf) / lgn
    f[1] = np.log2(1.0 + mf) / lge
    f[2] = np.log2(1.0 + mu) / lge
    f[3] = nu / max(n_sweep, 1)
    f[4] = min(max(np.log2((1.0 + mf) / (1.0 + mu)) / 16.0, -2.0), 2.0)
    f[5] = level / 32.0
    f[6] = float(cur_dir)
    f[7] = min(max(np.log2((1.0 + nf) / (1.0 + nf_prev)) / 8.0, -2.0), 2.0)
    return f


def ood(blob, f, level, slack=0.0):
    """True when level exceeds the largest training level or a feature lies
    outside [lo - w/10, hi + w/10], w = hi - lo (strict comparisons).  With
    slack > 0 the boundaries move outwards by slack (a feature counts as
    inside when it is inside within slack)."""
    blob = np.asarray(blob, np.float64)
    if level > blob[NPARAMS + 2 * NIN]:
        return True
    lo = blob[NPARAMS:NPARAMS + NIN]
    hi = blob[NPARAMS + NIN:NPARAMS + 2 * NIN]
    pad = OOD_WIDEN * (hi - lo)
    return bool(np.any(f < lo - pad - slack) or np.any(f > hi + pad + slack))


def heuristic_next(cur_dir, nf, mf, mu, nf_prev, n_sweep, alpha, beta):
    """Integer alpha/beta rule from the current direction: top-down ->
    bottom-up when m_f * alpha > m_u; bottom-up -> top-down when
    n_f * beta < n and n_f < n_f(previous level); else keep."""
    if cur_dir == 0:
        return 1 if mf * alpha > mu else 0
    return 0 if (nf * beta < n_sweep and nf < nf_prev) else 1


def _forward_bound(w, f, f_err):
    """Outputs y (fp64) and a bound on |y_fp32 - y| for a forward pass in
    fp32 whose inputs are within f_err of f: each layer's dot product of
    length k plus bias has rounding error at most gamma_{k+1} times the sum
    of the magnitudes of its terms (Higham, Accuracy and Stability of
    Numerical Algorithms, 3.1), input errors pass through the weights'
    magnitudes, and ReLU does not increase an error."""
    p = unpack(w)
    gam = lambda k: k * _U32 / (1 - k * _U32)  # noqa: E731
    a1 = p["W1"] @ f + p["b1"]
    h1 = np.maximum(a1, 0.0)
    e1 = np.abs(p["W1"]) @ np.full(NIN, f_err) + gam(NIN + 1) * (
        np.abs(p["W1"]) @ np.abs(f) + np.abs(p["b1"]))
    a2 = p["W2"] @ h1 + p["b2"]
    h2 = np.maximum(a2, 0.0)
    e2 = np.abs(p["W2"]) @ e1 + gam(NHID + 1) * (
        np.abs(p["W2"]) @ (np.abs(h1) + e1) + np.abs(p["b2"]))
    y = p["W3"] @ h2 + p["b3"]
    ey = np.abs(p["W3"]) @ e2 + gam(NHID + 1) * (
        np.abs(p["W3"]) @ (np.abs(h2) + e2) + np.abs(p["b3"]))
    return y, ey


def decide(blob, cur_dir, nf, mf, mu, nu, nf_prev, level, n_sweep, nnz, alpha, beta):
    """Direction of level `level` and how it was taken.

    Returns (direction, fallback, outcomes): fallback 0 = the network decided,
    1 = out of range, 2 = predictions within the margin (the alpha/beta rule
    decided in both cases).  The decision itself is taken in exact
    arithmetic.  `outcomes` is the set of (direction, fallback) pairs that an
    fp32 evaluation may reach: one pair when the exact values are farther
    from every threshold (range boundaries, margin) than the fp32 error
    bounds, more when a threshold lies within them."""
    blob = np.asarray(blob, np.float64)
    w = blob[:NPARAMS]
    margin = blob[BLOB - 1]
    f = features(nf, mf, mu, nu, nf_prev, level, cur_dir, n_sweep, nnz)
    rule = heuristic_next(cur_dir, nf, mf, mu, nf_prev, n_sweep, alpha, beta)
    lo = blob[NPARAMS:NPARAMS + NIN]
    hi = blob[NPARAMS + NIN:NPARAMS + 2 * NIN]
    # fp32 boundaries lo - 0.1f*(hi - lo) differ from the exact ones by a few
    # roundings of values of the size of |lo| + |hi|
    bnd_err = 4 * _U32 * (np.abs(lo) + np.abs(hi)).max(initial=0.0)
    slack = FEATURE_ERR + bnd_err

    def net_outcome(gap):
        if gap >= margin:
            return (1, 0)
        if -gap >= margin:
            return (0, 0)
        return (rule, FALLBACK_MARGIN)

    y, ey = _forward_bound(w, f, FEATURE_ERR)
    gap = y[0] - y[1]  # > 0: top-down predicted slower than bottom-up
    # the kernel forms y0 - y1 (and y1 - y0) in fp32: one more rounding
    gap_err = ey[0] + ey[1] + 2 * _U32 * (abs(y[0]) + abs(y[1]) + ey[0] + ey[1])
    net_exact = net_outcome(gap)
    net_any = {net_exact, net_outcome(gap - gap_err), net_outcome(gap + gap_err)}

    surely_out = ood(blob, f, level, slack=slack)      # outside the widened box
    maybe_out = ood(blob, f, level, slack=-slack)      # outside the shrunk box
    exact = (rule, FALLBACK_OOD) if ood(blob, f, level) else net_exact
    if surely_out:
        outcomes = {(rule, FALLBACK_OOD)}
    elif not maybe_out:
        outcomes = set(net_any)
    else:
        outcomes = {(rule, FALLBACK_OOD)} | net_any
    outcomes.add(exact)
    return exact[0], exact[1], outcomes


def learned_schedule(blob, nf, mf, mu, nu, n_sweep, nnz, alpha, beta, taken=None):
    """Replays the learned switch over a search whose per-level counters are
    nf[d], mf[d], mu[d], nu[d] (d = 0 .. levels-1, as the oracle's level
    counters give them).  Level 0 is top-down.  Returns (dirs, fallbacks,
    outcome sets).  taken (optional): the directions actually used; where a
    level's outcome set holds more than one pair, the replay continues from
    the direction taken (the features of the next level depend on it)."""
    L = len(nf)
    dirs = [0] * L
    fbs = [0] * L
    outs = [{(0, 0)}] + [None] * (L - 1)
    for d in range(1, L):
        cur = dirs[d - 1]
        dd, fb, oc = decide(blob, cur, int(nf[d]), int(mf[d]), int(mu[d]), int(nu[d]),
                            int(nf[d - 1]), d, n_sweep, nnz, alpha, beta)
        dirs[d], fbs[d], outs[d] = dd, fb, oc
        if taken is not None and len(oc) > 1:
            dirs[d] = int(taken[d])
    return dirs, fbs, outs
