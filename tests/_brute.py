"""Brute-force reference for the pins: heavily oversampled, graded tensor Gauss-Legendre
quadrature of the defining surface integrals with the patch's fitted densities.

The integrand of each kernel is the definition the method reproduces exactly once the
density is replaced by its harmonic fit (Lemma lem:dlpreduction, Theorem thm:slpreduction,
Sec. 3.6, Sec. 3.7); no line integral, root or recurrence is involved.
"""
import math

import numpy as np

from oracle.fit import gauss_legendre
from oracle.harmonics import H_basis
from oracle.quaternion import qmul, pure

FOUR_PI = 4.0 * math.pi


def _graded_1d(c, nlev, ng=24):
    c = min(max(c, -1.0), 1.0)
    pts = {-1.0, 1.0}
    h = 1.0
    for _ in range(nlev):
        h *= 0.5
        for s in (c - h, c + h):
            if -1 < s < 1:
                pts.add(s)
    if -1 < c < 1:
        pts.add(c)
    pts = sorted(pts)
    g, gw = gauss_legendre(ng)
    U, W = [], []
    for a, b in zip(pts[:-1], pts[1:]):
        U.append(0.5 * (a + b) + 0.5 * (b - a) * g)
        W.append(0.5 * (b - a) * gw)
    return np.concatenate(U), np.concatenate(W)


def brute_weights_dot(fit, pmap, x, nu_t, f, u0, v0, delta):
    """int_P K_eff(x, r) (fitted density of nodal data f)(r) da for K = S, D, S', D'."""
    fr = fit.frame
    xl = fr.point(x)
    nl = fr.vector(nu_t)
    nlev = max(2, int(math.log2(1.0 / max(delta, 1e-7))) + 3)
    U, WU = _graded_1d(u0, nlev)
    V, WV = _graded_1d(v0, nlev)
    uu, vv = np.meshgrid(U, V, indexing="ij")
    ww = np.outer(WU, WV).reshape(-1)
    r, ru, rv = pmap.derivs(uu.reshape(-1), vv.reshape(-1))
    n = np.cross(ru, rv)
    J = np.linalg.norm(n, axis=1)
    n /= J[:, None]
    da = ww * J / fr.s ** 2
    rl = fr.point(r)
    nn = fr.vector(n)
    H, gH = H_basis(fit.p, rl)
    n_p = H.shape[1]
    d = xl[None, :] - rl
    R = np.linalg.norm(d, axis=1)
    gG = d / (FOUR_PI * R[:, None] ** 3)
    G = 1.0 / (FOUR_PI * R)

    def qfield(c):
        cq = c.reshape(4, n_p).T
        out = np.zeros((len(R), 4))
        for i in range(n_p):
            out += qmul(pure(gH[:, :, i]), cq[i][None, :])
        return out

    qD = qfield(fit.M_D @ f)
    D = np.sum(da * (np.sum(gG * nn, 1) * qD[:, 0] + np.sum(np.cross(gG, nn) * qD[:, 1:], 1)))
    dgG = (nl[None, :] / R[:, None] ** 3 - 3 * d * (d @ nl)[:, None] / R[:, None] ** 5) / FOUR_PI
    Dp = np.sum(da * (np.sum(dgG * nn, 1) * qD[:, 0]
                      + np.sum(np.cross(dgG, nn) * qD[:, 1:], 1))) / fr.s
    qS = qfield(fit.M_Sp @ f)
    tot = np.sum(da[:, None] * qmul(qmul(pure(gG), pure(nn)), qS), 0)
    Sp = -qmul(pure(nl), tot)[0]
    cS = fit.M_S @ f
    dco, gco = cS[:n_p], cS[n_p:]
    sig = np.einsum("mkn,mk,n->m", gH, nn, dco)
    rho = H @ dco
    qr = qfield(gco)
    S = np.sum(da * (G * sig - np.sum(gG * nn, 1) * rho + np.sum(gG * nn, 1) * qr[:, 0]
                     + np.sum(np.cross(gG, nn) * qr[:, 1:], 1))) * fr.s
    return {"S": S, "D": D, "Sp": Sp, "Dp": Dp}
