"""Learned initial guess for the singularity-swap Newton solve: edge features and a small
multilayer perceptron, in float64.

Oracle module (test infrastructure only).

The method itself has no learned part.  The root t0 of sum_c (r_c(t) - x_c)^2 (eq.
complexparameter) is found by Newton from the chord start (Sec. 3.5, Step 5).  The
learned form proposes a better start, t_s + dt, where dt is predicted from features of the
edge and the target.  Plain Newton from t_s stays the fallback, so converged roots and
weights are those of the method.  This module defines:

* the features (8 numbers per (edge, target)): the chord start t_s (real, imaginary part)
  and the quadratic and cubic Legendre coefficients of the edge, divided by the chord
  half-length |d| and expressed in the chord frame (e1 along the chord, e2 toward the
  target's component perpendicular to it, e3 = e1 x e2).  They do not change under
  rotations, translations and uniform scalings of the edge and target together.
* the network 8 -> 64 -> 64 -> 2 with tanh hidden units and a linear output, and the
  mean squared error over a batch, L = (1/n) sum_b sum_o (y_bo - t_bo)^2, with its
  gradient by the chain rule (written out, no autodiff).
* one Adam step (Kingma & Ba, 2015) with bias correction.

Parameter layout (float32 on the device, float64 here), row-major, in this order:
W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2]  (4866 numbers).

Pins: the gradient is checked against central finite differences of the loss, the
forward pass against hand-computed cases, the features against the closed form of a
parabolic edge and against their invariances, and the chord start of a straight edge
against its exact root.
"""
import numpy as np

from .fit import poly_eval

N_IN, N_H, N_OUT = 8, 64, 2
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_OUT * N_H + N_OUT


def unpack(p):
    """Views (W1, b1, W2, b2, W3, b3) of a flat parameter vector."""
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    o = 0
    out = []
    for shape in ((N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (N_OUT, N_H), (N_OUT,)):
        n = int(np.prod(shape))
        out.append(p[o:o + n].reshape(shape))
        o += n
    return out


def forward(p, X):
    """Hidden activations and outputs for inputs X (n, 8)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.tanh(X @ W1.T + b1)
    H2 = np.tanh(H1 @ W2.T + b2)
    Y = H2 @ W3.T + b3
    return H1, H2, Y


def loss(p, X, Yt):
    """Mean over the batch of the squared output error, summed over the two outputs."""
    _, _, Y = forward(p, X)
    return float(np.sum((Y - Yt) ** 2) / X.shape[0])


def loss_grad(p, X, Yt):
    """(loss, gradient) by the chain rule: dL/dY = 2 (Y - Yt) / n; through the output
    layer, the tanh derivative 1 - h^2, the second layer, and the first."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    H1, H2, Y = forward(p, X)
    dY = 2.0 * (Y - Yt) / n                       # (n, 2)
    gW3 = dY.T @ H2
    gb3 = dY.sum(axis=0)
    dH2 = (dY @ W3) * (1.0 - H2 * H2)             # (n, 64)
    gW2 = dH2.T @ H1
    gb2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2) * (1.0 - H1 * H1)
    gW1 = dH1.T @ X
    gb1 = dH1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.sum((Y - Yt) ** 2) / n), g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def edge_features(coef, x):
    """Features of (edge, target) and the chord start t_s.

    coef: Legendre coefficients (ptilde, 3) of the edge (patch-local coordinates);
    x: target (3,).  The chord joins r(-1) and r(1): m = sum of even coefficients,
    d = sum of odd ones (P_k(1) = 1, P_k(-1) = (-1)^k)."""
    coef = np.asarray(coef, dtype=np.float64)
    n = coef.shape[0]
    k = np.arange(n)
    m = coef[k % 2 == 0].sum(axis=0)
    d = coef[k % 2 == 1].sum(axis=0)
    v = np.asarray(x, dtype=np.float64) - m
    dd = float(d @ d)
    ld = np.sqrt(dd)
    cr = np.cross(d, v)
    ts = complex(d @ v / dd, np.linalg.norm(cr) / dd)
    e1 = d / ld
    vp = v - (v @ e1) * e1
    nvp = np.linalg.norm(vp)
    if nvp > 0.0:
        e2 = vp / nvp
    else:
        # target on the chord line: any unit vector perpendicular to the chord
        a = np.array([1.0, 0.0, 0.0]) if abs(e1[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e2 = a - (a @ e1) * e1
        e2 = e2 / np.linalg.norm(e2)
    e3 = np.cross(e1, e2)
    a2 = coef[2] / ld if n > 2 else np.zeros(3)
    a3 = coef[3] / ld if n > 3 else np.zeros(3)
    f = np.array([ts.real, ts.imag, a2 @ e1, a2 @ e2, a2 @ e3, a3 @ e1, a3 @ e2, a3 @ e3])
    return f, ts


def root_residual(coef, x, t):
    """|sum_c (r_c(t) - x_c)^2| at complex t (zero at the root t0)."""
    r, _ = poly_eval(np.asarray(coef), np.array(complex(t)))
    e = r - x
    return abs(np.sum(e * e))
