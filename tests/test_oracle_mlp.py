"""Pins of the fp64 selector reference: finite differences, closed forms of
special networks, Adam's first step, argmin ties and the zone-map features."""
import numpy as np

from oracle import mlp

K = 8


def rand_theta(rng, k=K, scale=0.3):
    return rng.normal(0.0, scale, size=mlp.n_params(k))


def test_gradient_matches_central_differences(rng):
    x = rng.normal(size=(17, 6))
    y = rng.normal(size=(17, K))
    mask = (rng.random((17, K)) < 0.8).astype(float)
    mask[0, 0] = 1.0
    theta = rand_theta(rng)
    _, g = mlp.backward(theta, x, y, mask, K)
    h = 1e-6
    idx = rng.choice(len(theta), size=200, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp.loss(theta + e, x, y, mask, K) - mlp.loss(theta - e, x, y, mask, K)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])


def test_zero_weights_give_bias_and_mean_gradient(rng):
    theta = np.zeros(mlp.n_params(K))
    b3 = rng.normal(size=K)
    theta[-K:] = b3
    x = rng.normal(size=(9, 6))
    y = rng.normal(size=(9, K))
    out, _ = mlp.forward(theta, x, K)
    assert np.allclose(out, np.broadcast_to(b3, (9, K)), rtol=0, atol=0)
    _, g = mlp.backward(theta, x, y, np.ones((9, K)), K)
    # d/db3_j of mean_{i,j}(b3_j - y_ij)^2 over 9*K entries
    assert np.allclose(g[-K:], 2.0 * (b3 * 9 - y.sum(axis=0)) / (9 * K), rtol=1e-12, atol=1e-15)
    assert np.all(g[:-K] == 0.0)


def test_all_active_relus_reduce_to_a_linear_map(rng):
    """With non-negative weights, biases and inputs every ReLU passes its input,
    so the network is the product W3 W2 W1 applied to x plus the carried biases."""
    W1, b1 = rng.random((64, 6)), rng.random(64)
    W2, b2 = rng.random((64, 64)) * 0.1, rng.random(64)
    W3, b3 = rng.normal(size=(K, 64)), rng.normal(size=K)
    theta = mlp.flatten([W1, b1, W2, b2, W3, b3])
    x = rng.random((5, 6))
    out, _ = mlp.forward(theta, x, K)
    A = W3 @ W2 @ W1
    c = W3 @ (W2 @ b1 + b2) + b3
    assert np.allclose(out, x @ A.T + c, rtol=1e-12)


def test_adam_first_step_moves_by_lr_times_sign(rng):
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, m1, v1 = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(t1 - theta, -1e-3 * np.sign(g), rtol=1e-6)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_argmin_ties_and_validity():
    p = np.array([[3.0, 1.0, 1.0, 2.0], [0.5, 0.5, 0.1, 0.1]])
    assert list(mlp.argmin_strategy(p)) == [1, 2]
    valid = np.array([[True, False, True, True], [True, True, False, False]])
    assert list(mlp.argmin_strategy(p, valid)) == [2, 0]


def test_training_reduces_loss(rng):
    x = rng.random((256, 6))
    W = rng.normal(size=(6, K))
    y = x @ W
    theta = rand_theta(rng, scale=0.2)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, x, y, np.ones_like(y), K)
    for t in range(1, 301):
        _, g = mlp.backward(theta, x, y, np.ones_like(y), K)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=3e-3)
    assert mlp.loss(theta, x, y, np.ones_like(y), K) < 0.1 * l0


def test_features_closed_forms():
    n = 64 * 1024
    # every block holds each of 0..1023 once: the overlap estimate is exact
    zmin, zmax = np.zeros(64), np.full(64, 1023.0)
    f = mlp.features(10, n, 0, zmin, zmax, 100, 356)
    assert np.isclose(f[0], 10 / 32) and np.isclose(f[1], 16 / 24)
    assert np.isclose(f[2], np.log10(256 / 1024) / 6)
    assert f[3] == 1.0 and np.isclose(f[4], 1.0 - 1023 / 1024) and f[5] == 0.0
    # a sorted column of constant blocks: block k holds only value k
    zk = np.arange(64, dtype=float)
    f = mlp.features(6, n, 2, zk, zk, 10, 14)
    assert np.isclose(f[2], np.log10(4 / 64) / 6) and np.isclose(f[3], 4 / 64)
    assert f[4] == 1.0 and f[5] == 1.0
    # empty predicate
    f = mlp.features(6, n, 1, zk, zk, 14, 10)
    assert f[3] == 0.0 and np.isclose(f[2], -1.0) and np.isclose(f[5], 0.5)


def test_choose_with_margin_limits_and_brute_force():
    """margin 0 is the plain argmin; an unreachable margin always keeps the
    heuristic; in between, a brute-force reading of the rule row by row."""
    rng = np.random.default_rng(7)
    pred = rng.normal(size=(200, 8))
    valid = rng.random((200, 8)) < 0.8
    heur = rng.integers(0, 8, size=200)
    valid[np.arange(200), heur] = True
    assert np.array_equal(mlp.choose_with_margin(pred, valid, heur, 0.0), mlp.argmin_strategy(pred, valid))
    assert np.array_equal(mlp.choose_with_margin(pred, valid, heur, 1e9), heur)
    for margin in (0.1, 0.5):
        got = mlp.choose_with_margin(pred, valid, heur, margin)
        for i in range(200):
            vals = [(pred[i, j], j) for j in range(8) if valid[i, j]]
            best_v, best_j = min(vals)
            want = heur[i] if pred[i, heur[i]] - best_v < margin else best_j
            assert got[i] == want, (i, margin)
