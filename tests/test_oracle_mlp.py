"""Pins of the MLP reference: gradients against central finite differences,
the forward pass against a scalar network written with math.tanh, Adam's first
step against its closed form, loss reduction on a smooth target, and two-step
training trajectories (full batch and minibatches) written out by hand with
scalar arithmetic for a one-unit network."""
import math

import numpy as np
import pytest

from oracle import mlp_ref


def _data(n, d, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2 % d] - 0.3 * X[:, -1]
    return X, t


def test_gradients_match_finite_differences():
    d, H, n = 6, 9, 13
    P = mlp_ref.init(d, H, seed=1)
    for k in P:
        P[k] = P[k] + 0.1 * np.random.default_rng(2).standard_normal(P[k].shape)
    X, t = _data(n, d, 3)
    y, c = mlp_ref.forward(P, X)
    L, dy = mlp_ref.mse(y, t)
    g = mlp_ref.backward(P, c, dy)
    h = 1e-6
    for k in mlp_ref.PARAM_NAMES:
        flat = P[k].reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            Lp = mlp_ref.mse(mlp_ref.forward(P, X)[0], t)[0]
            flat[idx] = old - h
            Lm = mlp_ref.mse(mlp_ref.forward(P, X)[0], t)[0]
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, an)


def test_forward_against_scalar_network():
    P = {"W1": np.array([[0.7]]), "b1": np.array([-0.2]), "W2": np.array([[1.3]]), "b2": np.array([0.1]),
         "W3": np.array([[-0.8]]), "b3": np.array([0.05])}
    X = np.array([[0.3], [-1.1], [2.0]])
    y, _ = mlp_ref.forward(P, X)
    for x, yy in zip(X[:, 0], y):
        want = -0.8 * math.tanh(1.3 * math.tanh(0.7 * x - 0.2) + 0.1) + 0.05
        assert abs(yy - want) < 1e-15
    # zero weights give the output bias
    Z = {k: np.zeros_like(v) for k, v in mlp_ref.init(4, 5).items()}
    Z["b3"] = np.array([1.25])
    assert np.all(mlp_ref.forward(Z, np.ones((3, 4)))[0] == 1.25)


def test_mse_definition():
    L, dy = mlp_ref.mse(np.array([1.0, 2.0]), np.array([0.0, 4.0]))
    assert L == 2.5 and np.array_equal(dy, np.array([1.0, -2.0]))


def test_adam_first_step_closed_form():
    P = {k: np.ones(3) for k in mlp_ref.PARAM_NAMES}
    g = {k: np.array([0.5, -2.0, 1e-3]) for k in mlp_ref.PARAM_NAMES}
    st = mlp_ref.adam_init(P)
    mlp_ref.adam_step(P, g, st, lr=0.01, eps=1e-8)
    want = 1.0 - 0.01 * g["W1"] / (np.abs(g["W1"]) + 1e-8)
    for k in P:
        assert np.allclose(P[k], want, rtol=0, atol=1e-15)


def test_training_reduces_loss():
    X, t = _data(256, 5, 4)
    P = mlp_ref.init(5, 32, seed=5)
    hist = mlp_ref.train(P, X, t, epochs=300, lr=3e-3)
    assert hist[-1] < 0.2 * hist[0]


def test_weight_decay_gradient_matches_finite_differences():
    # objective = mse + (wd/2)|W|^2 over the weight matrices; biases unpenalised
    d, H, n, wd = 4, 5, 9, 0.37
    P = mlp_ref.init(d, H, seed=11)
    for k in P:
        P[k] = P[k] + 0.2 * np.random.default_rng(12).standard_normal(P[k].shape)
    X, t = _data(n, d, 13)
    y, c = mlp_ref.forward(P, X)
    _, dy = mlp_ref.mse(y, t)
    g = mlp_ref.backward(P, c, dy, wd)

    def objective():
        return mlp_ref.mse(mlp_ref.forward(P, X)[0], t)[0] + mlp_ref.penalty(P, wd)

    h = 1e-6
    for k in mlp_ref.PARAM_NAMES:
        flat = P[k].reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            Lp = objective()
            flat[idx] = old - h
            Lm = objective()
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)
    # the penalty of a hand-made parameter set
    Q = {"W1": np.array([[1.0, 2.0]]), "b1": np.array([5.0, 5.0]), "W2": np.array([[3.0, 0.0], [0.0, 0.0]]),
         "b2": np.zeros(2), "W3": np.array([[0.0], [-1.0]]), "b3": np.array([9.0])}
    assert mlp_ref.penalty(Q, 0.5) == 0.25 * (1 + 4 + 9 + 1)


# ---- training trajectories written out by hand for a one-unit network ------------------

def _scalar_params():
    return {"W1": 0.7, "b1": -0.2, "W2": 1.3, "b2": 0.1, "W3": -0.8, "b3": 0.05}


def _scalar_grad(P, xs, ts, wd):
    """Loss (1/n) sum (y - t)^2 over the given samples and its gradient, by the chain rule
    on scalars, plus wd * w for the three weights."""
    n = len(xs)
    g = {k: 0.0 for k in P}
    L = 0.0
    for x, t in zip(xs, ts):
        h1 = math.tanh(P["W1"] * x + P["b1"])
        h2 = math.tanh(P["W2"] * h1 + P["b2"])
        y = P["W3"] * h2 + P["b3"]
        L += (y - t) ** 2 / n
        dy = 2.0 * (y - t) / n
        g["W3"] += dy * h2
        g["b3"] += dy
        dz2 = dy * P["W3"] * (1.0 - h2 * h2)
        g["W2"] += dz2 * h1
        g["b2"] += dz2
        dz1 = dz2 * P["W2"] * (1.0 - h1 * h1)
        g["W1"] += dz1 * x
        g["b1"] += dz1
    for k in ("W1", "W2", "W3"):
        g[k] += wd * P[k]
    return L, g


def _scalar_adam(P, g, st, lr, b1=0.9, b2=0.999, eps=1e-8):
    st["t"] += 1
    for k in P:
        st["m"][k] = b1 * st["m"][k] + (1.0 - b1) * g[k]
        st["v"][k] = b2 * st["v"][k] + (1.0 - b2) * g[k] ** 2
        mh = st["m"][k] / (1.0 - b1 ** st["t"])
        vh = st["v"][k] / (1.0 - b2 ** st["t"])
        P[k] -= lr * mh / (math.sqrt(vh) + eps)


def _as_arrays(P):
    return {"W1": np.array([[P["W1"]]]), "b1": np.array([P["b1"]]), "W2": np.array([[P["W2"]]]),
            "b2": np.array([P["b2"]]), "W3": np.array([[P["W3"]]]), "b3": np.array([P["b3"]])}


def _close(a, b):
    return abs(a - b) <= 1e-13 * max(1.0, abs(b))


def test_full_batch_training_two_steps_by_hand():
    xs, ts, wd, lr = [0.3, -1.1, 2.0], [0.5, -0.25, 1.0], 0.1, 0.05
    P = _scalar_params()
    st = {"t": 0, "m": {k: 0.0 for k in P}, "v": {k: 0.0 for k in P}}
    want_hist = []
    for _ in range(2):
        L, g = _scalar_grad(P, xs, ts, wd)
        want_hist.append(L + 0.5 * wd * (P["W1"] ** 2 + P["W2"] ** 2 + P["W3"] ** 2))
        _scalar_adam(P, g, st, lr)
    Q = _as_arrays(_scalar_params())
    hist = mlp_ref.train(Q, np.array(xs)[:, None], np.array(ts), epochs=2, lr=lr, wd=wd)
    assert len(hist) == 2 and all(_close(a, b) for a, b in zip(hist, want_hist)), (hist, want_hist)
    for k in P:
        assert _close(float(Q[k].reshape(-1)[0]), P[k]), k


@pytest.mark.parametrize("batch", [1, 2])
def test_minibatch_training_two_epochs_by_hand(batch):
    # the samples are visited in the order of the seeded permutation, one Adam step per
    # minibatch (the last one ragged for batch = 2), and the history holds the whole-data
    # objective after each epoch
    xs, ts, wd, lr, seed = [0.3, -1.1, 2.0], [0.5, -0.25, 1.0], 0.02, 0.05, 7
    P = _scalar_params()
    st = {"t": 0, "m": {k: 0.0 for k in P}, "v": {k: 0.0 for k in P}}
    rng = np.random.default_rng(seed)
    want_hist = []
    for _ in range(2):
        order = [int(i) for i in rng.permutation(len(xs))]
        for s in range(0, len(xs), batch):
            idx = order[s:s + batch]
            _, g = _scalar_grad(P, [xs[i] for i in idx], [ts[i] for i in idx], wd)
            _scalar_adam(P, g, st, lr)
        L, _ = _scalar_grad(P, xs, ts, 0.0)
        want_hist.append(L + 0.5 * wd * (P["W1"] ** 2 + P["W2"] ** 2 + P["W3"] ** 2))
    assert st["t"] == 2 * (-(-len(xs) // batch))
    Q = _as_arrays(_scalar_params())
    hist = mlp_ref.train(Q, np.array(xs)[:, None], np.array(ts), epochs=2, lr=lr, batch=batch, seed=seed, wd=wd)
    assert all(_close(a, b) for a, b in zip(hist, want_hist)), (hist, want_hist)
    for k in P:
        assert _close(float(Q[k].reshape(-1)[0]), P[k]), k
