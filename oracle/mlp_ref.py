"""Reference for the learned planner's network -- TEST INFRASTRUCTURE ONLY.

The paper picks its partition with a fixed rule (Section V) and observes that
the best stream count depends on the device (Section VI, Xeon Phi with one
stream instead of two).  The learned planner replaces the rule's choice with a
small regression network that predicts the log run time of a candidate plan
from its features; the plan with the smallest prediction is taken.

Network (FP64 here): x (d) -> tanh(x W1 + b1) (H) -> tanh(. W2 + b2) (H) -> . W3 + b3 (1)
Loss: mean squared error L = (1/n) sum (y - t)^2, optionally plus an L2
penalty (wd/2) * (|W1|^2 + |W2|^2 + |W3|^2) on the weight matrices (biases are
not penalised), whose gradient adds wd * W to each weight matrix's gradient.
Optimiser: Adam (Kingma and Ba, ICLR 2015) with bias correction:
    m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
    theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
Weights are stored row-major: W1 (d x H), W2 (H x H), W3 (H x 1).
"""
import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init(d, H, seed=0):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((d, H)) / np.sqrt(d),
        "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) / np.sqrt(H),
        "b2": np.zeros(H),
        "W3": rng.standard_normal((H, 1)) / np.sqrt(H),
        "b3": np.zeros(1),
    }


def forward(P, X):
    """Returns (y, cache): y has shape (n,)."""
    Z1 = X @ P["W1"] + P["b1"]
    H1 = np.tanh(Z1)
    Z2 = H1 @ P["W2"] + P["b2"]
    H2 = np.tanh(Z2)
    y = (H2 @ P["W3"] + P["b3"])[:, 0]
    return y, (X, H1, H2)


def mse(y, t):
    """(loss, dL/dy)."""
    n = y.shape[0]
    d = y - t
    return float(np.sum(d * d) / n), 2.0 * d / n


def penalty(P, wd):
    """The L2 penalty (wd/2) * sum of the squared weight-matrix entries."""
    return 0.5 * wd * sum(float(np.sum(P[k] * P[k])) for k in ("W1", "W2", "W3"))


def backward(P, cache, dy, wd=0.0):
    """Gradients of the loss w.r.t. every parameter, given dL/dy (shape (n,)),
    plus the gradient wd * W of the L2 penalty on the weight matrices."""
    X, H1, H2 = cache
    g = {}
    dY = dy[:, None]
    g["W3"] = H2.T @ dY
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ P["W3"].T) * (1.0 - H2 * H2)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"].T) * (1.0 - H1 * H1)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    if wd:
        for k in ("W1", "W2", "W3"):
            g[k] = g[k] + wd * P[k]
    return g


def adam_init(P):
    return {"t": 0, "m": {k: np.zeros_like(v) for k, v in P.items()}, "v": {k: np.zeros_like(v) for k, v in P.items()}}


def adam_step(P, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    state["t"] += 1
    t = state["t"]
    for k in PARAM_NAMES:
        m = state["m"][k] = b1 * state["m"][k] + (1.0 - b1) * g[k]
        v = state["v"][k] = b2 * state["v"][k] + (1.0 - b2) * g[k] * g[k]
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P


def train(P, X, t, epochs, lr=1e-3, batch=None, seed=0, wd=0.0):
    """Full-batch (batch=None) or minibatch Adam training; returns the history of
    the objective (loss plus penalty)."""
    st = adam_init(P)
    rng = np.random.default_rng(seed)
    hist = []
    n = X.shape[0]
    for _ in range(epochs):
        if batch is None:
            y, c = forward(P, X)
            L, dy = mse(y, t)
            hist.append(L + penalty(P, wd))
            adam_step(P, backward(P, c, dy, wd), st, lr=lr)
        else:
            perm = rng.permutation(n)
            for s in range(0, n, batch):
                idx = perm[s:s + batch]
                y, c = forward(P, X[idx])
                L, dy = mse(y, t[idx])
                adam_step(P, backward(P, c, dy, wd), st, lr=lr)
            hist.append(mse(forward(P, X)[0], t)[0] + penalty(P, wd))
    return hist
