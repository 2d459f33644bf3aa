"""Pins for the fp64 network oracle (no GPU): central finite differences,
closed forms, and a known property of Adam's first step."""
import numpy as np
import pytest

import graphgen

from oracle import mlp


def rand_samples(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, 8))
    T = rng.normal(size=(n, 2))
    return np.hstack([X, T])


@pytest.mark.parametrize("seed", range(4))
def test_gradient_finite_differences(seed):
    w = graphgen.mlp_init_weights(seed)
    S = rand_samples(37, seed + 10)
    loss, g = mlp.loss_and_grad(w, S)
    h = 1e-6
    rng = np.random.default_rng(seed)
    for i in rng.choice(mlp.NPARAMS, 60, replace=False):
        e = np.zeros_like(w)
        e[i] = h
        num = (mlp.loss_and_grad(w + e, S)[0] - mlp.loss_and_grad(w - e, S)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, i


def test_closed_form_zero_output_layer():
    w = graphgen.mlp_init_weights(3)
    p = mlp.unpack(w)
    p["W3"][:] = 0.0
    w = mlp.pack(p)
    S = rand_samples(16, 4)
    y, _ = mlp.forward(w, S[:, :8])
    assert np.allclose(y, p["b3"])
    loss, g = mlp.loss_and_grad(w, S)
    T = S[:, 8:]
    assert np.isclose(loss, 0.5 * np.mean(np.sum((p["b3"] - T) ** 2, axis=1)))
    gp = mlp.unpack(g)
    assert np.allclose(gp["b3"], np.mean(p["b3"] - T, axis=0))
    assert np.allclose(gp["W1"], 0) and np.allclose(gp["W2"], 0)


def test_linear_regime_matches_least_squares_gradient():
    """With every pre-activation positive the network is linear in x; the
    output-bias gradient is then the mean residual."""
    w = np.full(mlp.NPARAMS, 0.05)
    X = np.random.default_rng(1).uniform(0.1, 1.0, size=(8, 8))
    S = np.hstack([X, np.zeros((8, 2))])
    y, (_, a1, _, a2, _) = mlp.forward(w, X)
    assert (a1 > 0).all() and (a2 > 0).all()
    _, g = mlp.loss_and_grad(w, S)
    assert np.allclose(mlp.unpack(g)["b3"], y.mean(axis=0))


def test_adam_first_step_moves_by_lr_sign():
    w0 = graphgen.mlp_init_weights(5)
    S = rand_samples(64, 6)
    order = np.arange(64)[None, :]
    w1, _ = mlp.train(S, w0, order, batch=64, lr=1e-3)
    _, g = mlp.loss_and_grad(w0, S)
    big = np.abs(g) > 1e-4
    assert np.allclose((w1 - w0)[big], -1e-3 * np.sign(g[big]), rtol=1e-3)


def test_training_reduces_loss_on_learnable_target():
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, size=(512, 8))
    T = np.stack([X[:, 0] * 2 + X[:, 1], 1 - X[:, 2]], axis=1)
    S = np.hstack([X, T])
    order = graphgen.epoch_orders(512, 30, 9)
    w, curve = mlp.train(S, graphgen.mlp_init_weights(1), order, batch=64, lr=3e-3)
    assert curve[-1] < 0.2 * curve[0]


def _bias_only_model(b3):
    """Every weight and hidden bias zero: h1 = h2 = 0, so y = b3 and only b3
    has a nonzero gradient, mean(b3 - t)."""
    w = np.zeros(mlp.NPARAMS)
    w[mlp.NPARAMS - 2:] = b3
    return w


def test_adam_three_steps_closed_form():
    """Adam (Kingma and Ba, Algorithm 1: beta1 0.9, beta2 0.999, eps 1e-8,
    bias-corrected moments) on L = 1/2 (b - 0)^2, whose gradient is b.
    Hand-derived, 40 significant digits, for b0 = 1:
      step 1: g = 1, m = 0.1, v = 0.001, m^ = 1, v^ = 1,
              b1 = 1 - 0.001/(1 + 1e-8) = 0.99900000000999999990...
      step 2: g = b1, m = 0.09 + 0.1 b1, v = 0.000999 + 0.001 b1^2,
              m^ = m/0.19, v^ = v/0.001999 -> b2 = 0.99800002622383660573...
      step 3: likewise -> 0.99700009608014747890...
    and for b0 = -2: -1.99900000000499999997, -1.99800001307735920079,
    -1.99700004790477472725.  A dropped bias correction, a wrong exponent
    or a second moment that stops updating after step 1 moves step 2 by
    more than 1e-4."""
    expect = {1: (0.9990000000099999999, -1.9990000000049999999),
              2: (0.9980000262238366057, -1.9980000130773592008),
              3: (0.9970000960801474789, -1.9970000479047747273)}
    S = np.zeros((4, 10))                      # 4 samples, all targets 0
    w0 = _bias_only_model([1.0, -2.0])
    for steps, (e0, e1) in expect.items():
        order = np.tile(np.arange(4), (steps, 1))  # one full batch per epoch
        w, _ = mlp.train(S, w0, order, batch=4, lr=1e-3)
        assert abs(w[-2] - e0) <= 1e-13 and abs(w[-1] - e1) <= 1e-13, steps
        assert np.all(w[:-2] == 0.0)           # zero gradients leave them alone


# ---- learned direction decision -------------------------------------------

def _blob(b3=(0.0, 0.0), lo=-1.0, hi=1.0, max_level=10, margin=0.25):
    """Switch blob of the bias-only network y = b3 with training range
    [lo, hi] for every feature."""
    blob = np.zeros(mlp.BLOB)
    blob[:mlp.NPARAMS] = _bias_only_model(b3)
    blob[mlp.NPARAMS:mlp.NPARAMS + 8] = lo
    blob[mlp.NPARAMS + 8:mlp.NPARAMS + 16] = hi
    blob[mlp.NPARAMS + 16] = max_level
    blob[mlp.NPARAMS + 17] = margin
    return blob


def test_features_worked_example():
    """n = 256 (log2 8), nnz = 65536 (log2 16); n_f = 15, m_f = 255,
    m_u = 4095, n_u = 64, n_f(prev) = 3, level 3, current direction 1:
    f0 = log2 16 / 8 = 0.5, f1 = log2 256 / 16 = 0.5, f2 = log2 4096 / 16 =
    0.75, f3 = 64/256 = 0.25, f4 = log2(256/4096)/16 = -0.25, f5 = 3/32,
    f6 = 1, f7 = log2(16/4)/8 = 0.25."""
    f = mlp.features(15, 255, 4095, 64, 3, 3, 1, 256, 65536)
    assert np.allclose(f, [0.5, 0.5, 0.75, 0.25, -0.25, 3 / 32, 1.0, 0.25], rtol=0, atol=1e-15)
    # clamps: log2((1+m_f)/(1+m_u))/16 below -2 and log2 ratio of n_f above 2
    f = mlp.features(2 ** 20 - 1, 0, 2 ** 40 - 1, 1, 0, 1, 0, 2 ** 20, 2 ** 20)
    assert f[4] == -2.0 and f[7] == 2.0
    # degenerate sizes: logarithms of at least 2, n_u over at least 1
    f = mlp.features(0, 0, 0, 0, 0, 1, 0, 0, 0)
    assert np.all(np.isfinite(f)) and f[0] == 0.0 and f[3] == 0.0


def test_ood_boundaries():
    """Range [0, 1] widened by 10 % of its width: [-0.1, 1.1], ends inside."""
    blob = _blob(lo=0.0, hi=1.0, max_level=5)
    inside = np.full(8, 0.5)
    assert not mlp.ood(blob, inside, 5)         # level = largest training level
    assert mlp.ood(blob, inside, 6)             # one beyond
    for i in range(8):
        for v, out in ((-0.1, False), (1.1, False), (-0.1 - 1e-9, True), (1.1 + 1e-9, True)):
            f = inside.copy()
            f[i] = v
            assert mlp.ood(blob, f, 1) == out, (i, v)
    # a zero-width range [0.25, 0.25] accepts exactly 0.25
    blob2 = _blob(lo=0.25, hi=0.25)
    assert not mlp.ood(blob2, np.full(8, 0.25), 1)
    assert mlp.ood(blob2, np.full(8, 0.25 + 1e-12), 1)


# counters of one decision, chosen so that every feature lies in [-1, 1]:
# n = 2^16, nnz = 2^20, n_f = 99, m_f = 4000, m_u = 2^19, n_u = 30000,
# n_f(prev) = 50, level 2 -> alpha/beta (14, 24) from top-down says top-down
# (4000 * 14 = 56000 <= 524288), from bottom-up says bottom-up (99 >= 50).
DEC = dict(nf=99, mf=4000, mu=2 ** 19, nu=30000, nf_prev=50, level=2, n_sweep=2 ** 16,
           nnz=2 ** 20, alpha=14, beta=24)


def _decide(blob, cur_dir, **kw):
    a = dict(DEC)
    a.update(kw)
    return mlp.decide(blob, cur_dir, a["nf"], a["mf"], a["mu"], a["nu"], a["nf_prev"],
                      a["level"], a["n_sweep"], a["nnz"], a["alpha"], a["beta"])


def test_decide_network_and_fallbacks():
    f = mlp.features(99, 4000, 2 ** 19, 30000, 50, 2, 0, 2 ** 16, 2 ** 20)
    assert np.all((f >= -1) & (f <= 1))
    # y = (ln us TD, ln us BU)
    d, fb, oc = _decide(_blob(b3=(3.0, 2.0)), 0)      # BU predicted e^1 x cheaper
    assert (d, fb, oc) == (1, 0, {(1, 0)})
    d, fb, oc = _decide(_blob(b3=(2.0, 3.0)), 1)      # TD cheaper
    assert (d, fb, oc) == (0, 0, {(0, 0)})
    # within the margin: the alpha/beta rule decides from the current direction
    assert _decide(_blob(b3=(2.2, 2.0)), 0)[:2] == (0, 2)
    assert _decide(_blob(b3=(2.2, 2.0)), 1)[:2] == (1, 2)
    assert _decide(_blob(b3=(2.0, 2.2)), 0)[:2] == (0, 2)
    # the margin itself belongs to the network (difference >= 0.25); in
    # fp32 the difference may round either way, so both outcomes are allowed
    d, fb, oc = _decide(_blob(b3=(2.25, 2.0)), 0)
    assert (d, fb) == (1, 0) and oc == {(1, 0), (0, 2)}
    # the margin is the blob's: with 0.1 the 0.2 difference decides, with
    # 1.5 a difference of 1 does not
    assert _decide(_blob(b3=(2.2, 2.0), margin=0.1), 0)[:2] == (1, 0)
    assert _decide(_blob(b3=(3.0, 2.0), margin=1.5), 0)[:2] == (0, 2)
    # out of range: level beyond the training maximum, or a feature outside
    assert _decide(_blob(b3=(3.0, 2.0), max_level=1), 0)[:3] == (0, 1, {(0, 1)})
    assert _decide(_blob(b3=(3.0, 2.0), lo=0.9, hi=1.0), 1)[:3] == (1, 1, {(1, 1)})


def test_decide_all_out_of_range_is_the_alpha_beta_schedule():
    """With an empty training range every level falls back, and the replay
    is the alpha/beta schedule, which is pinned by hand cases elsewhere."""
    import graphgen
    import oracle
    off, cols = graphgen.kronecker_csr(12, 16, 3)
    perm, _, nplus = oracle.rcm(off, cols)
    blob = np.zeros(mlp.BLOB)
    blob[mlp.NPARAMS + 16] = 64
    for r in graphgen.sample_roots(off, 4, 7):
        depth, _, _ = oracle.bfs(off, cols, r, perm)
        c = oracle.level_counters(off, cols, depth, perm, nplus)
        dirs, fbs, _ = mlp.learned_schedule(blob, c["nf"], c["mf"], c["mu"], c["nu"], nplus,
                                            int(off[-1]), 14, 24)
        ref = oracle.heuristic_schedule(c["nf"], c["mf"], c["mu"], nplus, 14, 24)
        assert list(dirs) == list(ref)
        assert all(x == 1 for x in fbs[1:])


def test_forward_error_bound_covers_fp32():
    """The bound decide() uses holds for a plain fp32 evaluation of random
    networks at random inputs perturbed within the feature error."""
    import graphgen
    rng = np.random.default_rng(4)
    for seed in range(6):
        w = graphgen.mlp_init_weights(seed) * (1 + seed)
        for _ in range(20):
            f = rng.uniform(-1, 2, 8)
            y, ey = mlp._forward_bound(w, f, mlp.FEATURE_ERR)
            p = {k: v.astype(np.float32) for k, v in mlp.unpack(w).items()}
            x = (f + rng.uniform(-1, 1, 8) * mlp.FEATURE_ERR).astype(np.float32)
            h1 = np.maximum(p["W1"] @ x + p["b1"], np.float32(0))
            h2 = np.maximum(p["W2"] @ h1 + p["b2"], np.float32(0))
            y32 = (p["W3"] @ h2 + p["b3"]).astype(np.float64)
            y64 = mlp.forward(w.astype(np.float32).astype(np.float64), f[None, :])[0][0]
            assert np.all(np.abs(y32 - y64) <= ey + 1e-12)
