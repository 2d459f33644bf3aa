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
