"""Pins of the learned-guess oracle (features, network, loss gradient, Adam) on the CPU."""
import math

import numpy as np
import pytest

from oracle import mlp
from oracle.fit import edge_coefficients, gauss_legendre
from oracle.ssq import chord_start, newton_root

RNG = np.random.default_rng(11)


def _params(scale=0.3, rng=RNG):
    return rng.normal(scale=scale, size=mlp.N_PARAMS)


def test_parameter_count():
    assert mlp.N_PARAMS == 64 * 8 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 4866


def test_forward_hand_cases():
    """Zero weights give y = b3; one path through the network gives
    y_0 = w3 tanh(w2 tanh(w1 x_0 + c1) + c2) + c3, computed by hand."""
    p = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)   # views into p
    b3[:] = [0.25, -1.5]
    X = RNG.normal(size=(5, 8))
    _, _, Y = mlp.forward(p, X)
    assert np.all(Y == np.array([0.25, -1.5]))
    W1[3, 0] = 0.7
    b1[3] = -0.2
    W2[10, 3] = 1.3
    b2[10] = 0.1
    W3[0, 10] = -2.0
    x0 = 0.4
    X = np.zeros((1, 8))
    X[0, 0] = x0
    _, _, Y = mlp.forward(p, X)
    expect = -2.0 * math.tanh(1.3 * math.tanh(0.7 * x0 - 0.2) + 0.1) + 0.25
    assert abs(Y[0, 0] - expect) < 1e-15
    assert Y[0, 1] == -1.5


def test_loss_gradient_matches_central_differences():
    p = _params()
    X = RNG.normal(size=(7, 8))
    Yt = RNG.normal(size=(7, 2))
    L, g = mlp.loss_grad(p, X, Yt)
    assert abs(L - mlp.loss(p, X, Yt)) < 1e-14 * max(1.0, L)
    idx = np.concatenate([RNG.choice(mlp.N_PARAMS, 150, replace=False),
                          [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4863, 4864, 4865]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, Yt) - mlp.loss(p - e, X, Yt)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-8 + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_adam_first_step_closed_form():
    """From zero moments, the first bias-corrected step is lr * g / (|g| + eps)."""
    p = _params()
    g = RNG.normal(size=mlp.N_PARAMS)
    p1, m, v = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def _edge_from_curve(fun, pt=16):
    t, _ = gauss_legendre(pt)
    return edge_coefficients(np.stack([fun(ti) for ti in t]))


def test_features_parabola_closed_form():
    """r(t) = (t, c t^2, 0): Legendre coefficients a0 = (0, c/3, 0), a1 = (1, 0, 0),
    a2 = (0, 2c/3, 0); chord from (-1, c, 0) to (1, c, 0): m = (0, c, 0), |d| = 1.  For a
    target above the chord in +y, e2 = +y, so the features are (t_s, 0, 2c/3, 0, 0, 0, 0)."""
    c = 0.3
    coef = _edge_from_curve(lambda t: np.array([t, c * t * t, 0.0]))
    x = np.array([0.2, c + 0.5, 0.0])
    f, ts = mlp.edge_features(coef, x)
    assert abs(ts - complex(0.2, 0.5)) < 1e-14
    expect = np.array([0.2, 0.5, 0.0, 2 * c / 3, 0.0, 0.0, 0.0, 0.0])
    assert np.max(np.abs(f - expect)) < 1e-13
    # the chord start used by the method is the same number
    assert abs(chord_start(coef, x) - ts) < 1e-14


def test_features_invariant_under_similarity():
    coef = _edge_from_curve(lambda t: np.array([t, 0.2 * t * t - 0.1 * t ** 3, 0.05 * t ** 3]))
    x = np.array([0.1, 0.3, 0.2])
    f0, _ = mlp.edge_features(coef, x)
    A = np.linalg.qr(RNG.normal(size=(3, 3)))[0]
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    s, sh = 2.7, np.array([0.3, -1.0, 4.0])
    coef2 = s * coef @ A.T
    coef2[0] += sh
    f1, _ = mlp.edge_features(coef2, s * A @ x + sh)
    assert np.max(np.abs(f1 - f0)) < 1e-12


def test_straight_edge_chord_start_is_the_root():
    """For a straight edge the chord start solves the distance equation exactly, so Newton
    from it stops at once and the target dt = t0 - t_s is zero."""
    coef = np.zeros((16, 3))
    coef[0] = [0.5, -0.3, 0.0]
    coef[1] = [0.8, 0.1, 0.2]
    x = np.array([0.7, 0.4, -0.2])
    _, ts = mlp.edge_features(coef, x)
    assert mlp.root_residual(coef, x, ts) < 1e-14
    t0, its, conv = newton_root(coef, x, ts)
    assert conv and its <= 2 and abs(t0 - ts) < 1e-14
