"""Pins of the MLP oracle: finite differences, closed forms, Adam's first step."""
import numpy as np

import oracle.mlp as M


def _data(seed, B=12):
    r = np.random.default_rng(seed)
    X = r.standard_normal((B, 16)) * 3 + 1
    labels = np.stack([r.integers(0, k, B) for k in M.HEADS], axis=1)
    return X, X.mean(0), X.std(0) + 0.1, labels


def test_param_count():
    assert M.NPARAM == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 11 + 11 == 5963


def test_gradient_matches_central_differences():
    X, mu, sd, y = _data(1)
    th = M.init_params(3) + 0.01 * np.random.default_rng(4).standard_normal(M.NPARAM)
    loss, g = M.loss_and_grad(th, X, mu, sd, y)
    idx = np.random.default_rng(5).choice(M.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss_and_grad(th + e, X, mu, sd, y)[0] - M.loss_and_grad(th - e, X, mu, sd, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_zero_logits_loss_closed_form():
    X, mu, sd, y = _data(2)
    th = np.zeros(M.NPARAM)
    loss, g = M.loss_and_grad(th, X, mu, sd, y)
    assert np.isclose(loss, np.log(4) + np.log(5) + np.log(2))
    # with zero weights only the output biases get a gradient: mean(softmax) - onehot
    W1, b1, W2, b2, W3, b3 = M.unpack(g)
    assert np.all(W1 == 0) and np.all(W3 == 0) and np.all(b1 == 0)
    onehot = np.concatenate([np.eye(k)[y[:, h]] for h, k in enumerate(M.HEADS)], axis=1)
    ref = np.concatenate([np.full(k, 1.0 / k) for k in M.HEADS]) - onehot.mean(0)
    assert np.allclose(b3, ref)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = M.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    assert np.allclose(th[:3], -1e-3 * np.sign(g[:3]), rtol=1e-4) and th[3] == 0


def test_training_fits_a_learnable_rule():
    r = np.random.default_rng(7)
    X = r.standard_normal((200, 16))
    y = np.stack([(X[:, 0] > 0).astype(int) * 3, (X[:, 1] > 0).astype(int) * 4, (X[:, 2] > 0).astype(int)], axis=1)
    mu, sd = X.mean(0), X.std(0)
    th = M.init_params(11)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = M.loss_and_grad(th, X, mu, sd, y)[0]
    for t in range(1, 301):
        loss, g = M.loss_and_grad(th, X, mu, sd, y)
        th, m, v = M.adam_step(th, g, m, v, t, lr=3e-3)
    assert loss < 0.2 * l0
    assert np.mean(M.predict(th, X, mu, sd) == y) > 0.95
