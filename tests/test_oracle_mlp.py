"""Pins of the pivot-proposer oracle (float64): gradients against central finite
differences, the features against hand-checked values, the loss and Adam against closed
forms."""
import math

import numpy as np

from oracle import mlp


def _problem(seed=0, n=37):
    rng = np.random.default_rng(seed)
    p = mlp.init_weights(rng)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((n, mlp.F))
    y = (rng.random(n) < 0.3).astype(float)
    return p, X, y


def test_backward_matches_central_differences():
    p, X, y = _problem()
    pw = 5.0
    s, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, s, y, pw)
    rng = np.random.default_rng(1)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(p, X)[0], y, pw)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(p, X)[0], y, pw)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_loss_closed_forms():
    y = np.array([1.0, 0.0, 1.0, 0.0])
    # s = 0: every term is w log 2
    assert math.isclose(mlp.loss(np.zeros(4), y, 3.0), (3 + 1 + 3 + 1) / 4 * math.log(2.0),
                        rel_tol=1e-15)
    # a confident correct logit costs ~e^{-|s|}
    assert mlp.loss(np.array([40.0]), np.array([1.0]), 1.0) < 1e-16
    assert math.isclose(mlp.loss(np.array([-40.0]), np.array([1.0]), 1.0), 40.0, rel_tol=1e-12)


def test_features_hand_values():
    n2, r = 10, 2
    B0 = np.zeros((n2, r))
    B0[3, 0] = 2.0
    B0[7, 1] = 1.0
    X = mlp.features(B0, [3, 8])
    nrm2 = 5.0
    # previous pivots and the distance feature
    assert X[3, 0] == 1.0 and X[8, 0] == 1.0 and X[0, 0] == 0.0
    assert math.isclose(X[5, 1], math.exp(-1.0)) and math.isclose(X[0, 1], math.exp(-1.5))
    # leverage: row 3 holds 4/5 of the norm; centre tap o = 0 is feature 4
    assert math.isclose(X[3, 4], math.log1p(n2 * 4.0 / nrm2))
    assert math.isclose(X[5, 2], math.log1p(n2 * 4.0 / nrm2))        # o = -2 from row 5
    assert X[0, 4] == 0.0
    # mean leverage is 1: sum over rows of (e^f - 1) = n2
    assert math.isclose(np.sum(np.expm1(X[:, 4])), n2)
    # jump at row 2 (B0[3] - B0[2]) and at row 3 (B0[4] - B0[3]); none at the last row
    assert math.isclose(X[2, 9], math.log1p(n2 * 4.0 / nrm2))
    assert math.isclose(X[3, 9], math.log1p(n2 * 4.0 / nrm2))
    assert X[9, 9] == 0.0
    # clamping at the edges: o = -2 at row 0 reads row 0
    assert X[0, 2] == X[0, 4]
    assert X[4, 12] == 0.4 and X[0, 14] == 1.0 and np.all(X[:, 15] == 1.0)


def test_adam_first_step_is_signed_lr():
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    mlp.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    assert np.allclose(p["a"], np.array([1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01]), rtol=0,
                       atol=1e-15)


def test_adam_matches_closed_form_over_three_steps():
    """Adam (Kingma and Ba 2015) unrolled: after t steps the moments are the bias-weighted
    sums m_t = (1 - b1) sum_i b1^(t-i) g_i and v_t = (1 - b2) sum_i b2^(t-i) g_i^2, and step t
    moves p by lr m_t / (1 - b1^t) / (sqrt(v_t / (1 - b2^t)) + eps).  Gradients change sign
    and size between steps, so (1 - b2)^t in place of 1 - b2^t fails at t = 2 and 3."""
    b1, b2, lr, eps = 0.9, 0.999, 0.01, 1e-8
    gs = [np.array([1.0, -0.5]), np.array([3.0, 0.25]), np.array([-2.0, 4.0])]
    p = {"a": np.array([0.3, -0.7])}
    m = {"a": np.zeros(2)}
    v = {"a": np.zeros(2)}
    ref = p["a"].copy()
    for t in (1, 2, 3):
        mlp.adam_step(p, {"a": gs[t - 1]}, m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        mt = (1 - b1) * sum(b1 ** (t - i) * gs[i - 1] for i in range(1, t + 1))
        vt = (1 - b2) * sum(b2 ** (t - i) * gs[i - 1] ** 2 for i in range(1, t + 1))
        ref = ref - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        assert np.allclose(p["a"], ref, rtol=0, atol=1e-15), t


def test_adam_constant_gradient_moves_by_lr():
    """With a constant gradient the bias corrections cancel exactly: every step moves each
    parameter by lr against the gradient's sign (eps = 0), whatever t."""
    p = {"a": np.array([1.0, 2.0])}
    g = {"a": np.array([0.3, -7.0])}
    m = {"a": np.zeros(2)}
    v = {"a": np.zeros(2)}
    for t in range(1, 6):
        before = p["a"].copy()
        mlp.adam_step(p, g, m, v, t, lr=0.05, eps=0.0)
        assert np.allclose(p["a"] - before, [-0.05, 0.05], rtol=0, atol=1e-14), t
