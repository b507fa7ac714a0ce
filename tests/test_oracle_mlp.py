"""The CPU MLP oracle's gradient against central finite differences of its
own loss in double precision (the backpropagation is checked against the
definition of the derivative), and its parameter layout."""
import numpy as np

from oracle import mlp as M


def test_param_count_and_layout():
    assert M.N_PARAMS == 4481
    theta = np.arange(M.N_PARAMS, dtype=np.float64)
    p = M.unpack(theta)
    assert p["W1"][0, 0] == 0 and p["b1"][0] == 192 and p["W2"][0, 0] == 256
    assert p["b2"][0] == 4352 and p["w3"][0] == 4416 and p["b3"][0] == 4480
    assert np.array_equal(M.pack(p), theta)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = rng.normal(0, 0.3, M.N_PARAMS)
    X = rng.normal(size=(40, 3))
    T = rng.normal(size=40)
    loss, g = M.loss_and_grad(theta, X, T)
    idx = rng.choice(M.N_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, [4480, 4416, 4352, 256, 192, 0]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.N_PARAMS); e[i] = h
        fd = (M.loss_and_grad(theta + e, X, T)[0] - M.loss_and_grad(theta - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_is_the_composition():
    rng = np.random.default_rng(1)
    theta = rng.normal(0, 0.5, M.N_PARAMS)
    p = M.unpack(theta)
    x = rng.normal(size=3)
    h1 = np.maximum(0, [sum(x[k] * p["W1"][k, j] for k in range(3)) + p["b1"][j] for j in range(64)])
    h2 = np.maximum(0, [sum(h1[k] * p["W2"][k, j] for k in range(64)) + p["b2"][j] for j in range(64)])
    y = sum(h2[j] * p["w3"][j] for j in range(64)) + p["b3"][0]
    assert abs(M.forward(theta, x[None, :])[0][0] - y) < 1e-12 * (1 + abs(y))
