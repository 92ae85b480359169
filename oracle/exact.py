"""The oracle's steps for one far pair carried out with 40 significant digits (mpmath).

Oracle module (test infrastructure only).

For a near pair whose four edges all fall in the far class (the chord root of every edge
lies outside the Bernstein ellipse of radius rho_far, so every edge uses the plain
Gauss-Legendre rule), the method's weights are a finite composition of arithmetic and
square roots on the double-precision inputs: the frame (Step 1), the weighted least-squares
fits (Step 2), the edge interpolants and tables (Step 3), the target harmonics (Step 4), the
edge rule (Step 5, far class), the line integrals (Step 6), the translation (Step 7) and the
rows (Step 8), multiplied with the maps as in the matrix-row remark after the algorithm in
Sec. 4, and the smooth rule subtracted (eq. dlpsplitting).  This module evaluates that same
composition, step by step as the double-precision oracle does, from the same inputs, with 40
digits, so that its result is the exact-arithmetic result of the method for those inputs to
far below the rounding of any FP64 implementation.  The least-squares solutions are unique
(full-rank systems), so they are computed here from the normal equations, whose squared
conditioning (below 1e16 for these fits) still leaves more than 20 digits.

Parity status: pinned by agreement with the double-precision oracle within that oracle's
own rounding spread (tests/test_oracle_pins.py).
"""
import math

import mpmath
import numpy as np

from .ssq import bernstein_radius, rho_far

DPS = 40


def _mp(x):
    return mpmath.mpf(float(x))


def gauss_legendre(n):
    """n-point Gauss-Legendre nodes and weights: the double nodes refined by Newton on P_n."""
    t0, _ = np.polynomial.legendre.leggauss(n)
    ts, ws = [], []
    for x in t0:
        t = _mp(x)
        for _ in range(4):
            p, dp = _legendre_last(n, t)
            t = t - p / dp
        p, dp = _legendre_last(n, t)
        ts.append(t)
        ws.append(2 / ((1 - t * t) * dp * dp))
    return ts, ws


def _legendre_last(n, t):
    """P_n(t) and P_n'(t) by the three-term recurrence."""
    p0, p1 = mpmath.mpf(1), t
    if n == 0:
        return p0, mpmath.mpf(0)
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
    dp = n * (t * p1 - p0) / (t * t - 1)
    return p1, dp


def _legendre_all(n, t):
    """P_k(t) and P_k'(t) for k = 0..n-1."""
    P = [mpmath.mpf(1), t]
    D = [mpmath.mpf(0), mpmath.mpf(1)]
    for k in range(1, n - 1):
        P.append(((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1))
        D.append(D[k - 1] + (2 * k + 1) * P[k])
    return P[:n], D[:n]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _sub(a, b):
    return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]


def _scale(a, s):
    return [a[0] * s, a[1] * s, a[2] * s]


def _unit(a):
    return _scale(a, 1 / mpmath.sqrt(_dot(a, a)))


# ---------------------------------------------------------------- edges and frame (Steps 1, 3)

def edge_coefficients(samples, tw):
    """Legendre coefficients of the interpolant through the GL samples of one edge (the same
    discrete Legendre transform as the double oracle)."""
    t, w = tw
    n = len(t)
    Ps = [_legendre_all(n, ti)[0] for ti in t]
    return [[(2 * k + 1) * sum(w[i] * Ps[i][k] * samples[i][c] for i in range(n)) / 2
             for c in range(3)] for k in range(n)]


def poly_eval(coef, t):
    n = len(coef)
    P, D = _legendre_all(n, t)
    val = [sum(coef[k][c] * P[k] for k in range(n)) for c in range(3)]
    der = [sum(coef[k][c] * D[k] for k in range(n)) for c in range(3)]
    return val, der


class Frame:
    """Origin at the mean corner, z along (c2 - c0) x (c3 - c1) signed by the mean node
    normal, x along the first side, scale = longest side (Step 1; the quad reading)."""

    def __init__(self, edge_samples, node_nrm, tw):
        c = [poly_eval(edge_coefficients(edge_samples[e], tw), mpmath.mpf(-1))[0]
             for e in range(4)]
        self.o = [sum(c[k][a] for k in range(4)) / 4 for a in range(3)]
        ez = _unit(_cross(_sub(c[2], c[0]), _sub(c[3], c[1])))
        mn = [sum(n[a] for n in node_nrm) / len(node_nrm) for a in range(3)]
        if _dot(ez, mn) < 0:
            ez = _scale(ez, -1)
        d = _sub(c[1], c[0])
        ex = _unit(_sub(d, _scale(ez, _dot(d, ez))))
        ey = _cross(ez, ex)
        self.axes = (ex, ey, ez)
        self.s = max(mpmath.sqrt(_dot(_sub(c[(k + 1) % 4], c[k]), _sub(c[(k + 1) % 4], c[k])))
                     for k in range(4))

    def point(self, x):
        d = _sub(x, self.o)
        return [_dot(d, a) / self.s for a in self.axes]

    def vector(self, v):
        return [_dot(v, a) for a in self.axes]


# ---------------------------------------------------------------- harmonics (Sec. 2.3, 3.2)

def solid_harmonics(L, x, y, z):
    """R_l^m (Racah normalisation, no Condon-Shortley phase) as a dict {(l, m): mpc}, by the
    Cartesian recurrence of eq. associatelegendrerecurrence."""
    r2 = x * x + y * y + z * z
    w = mpmath.mpc(x, y)
    R = {(0, 0): mpmath.mpc(1)}
    for l in range(1, L + 1):
        R[(l, l)] = mpmath.sqrt(mpmath.mpf(2 * l - 1) / (2 * l)) * w * R[(l - 1, l - 1)]
        for m in range(0, l):
            prev2 = R.get((l - 2, m), 0) if l >= 2 else 0
            R[(l, m)] = ((2 * l - 1) * z * R[(l - 1, m)]
                         - r2 * mpmath.sqrt((l - 1 + m) * (l - 1 - m)) * prev2) / mpmath.sqrt(l * l - m * m)
    for l in range(1, L + 1):
        for m in range(1, l + 1):
            R[(l, -m)] = (-1) ** m * mpmath.conj(R[(l, m)])
    return R


def _ladder(T, L, which):
    out = {}
    for l in range(0, L + 1):
        for m in range(-l, l + 1):
            v = 0
            if which == 'z':
                if abs(m) <= l - 1:
                    v = mpmath.sqrt((l + m) * (l - m)) * T[(l - 1, m)]
            elif which == '-':
                if l >= 1 and abs(m - 1) <= l - 1:
                    v = mpmath.sqrt((l + m) * (l + m - 1)) * T[(l - 1, m - 1)]
            else:
                if l >= 1 and abs(m + 1) <= l - 1:
                    v = -mpmath.sqrt((l - m) * (l - m - 1)) * T[(l - 1, m + 1)]
            out[(l, m)] = mpmath.mpc(v)
    return out


def _d(T, L, axis):
    """Cartesian partial derivative of a table of solid harmonics (ladder identities)."""
    if axis == 2:
        return _ladder(T, L, 'z')
    p, mi = _ladder(T, L, '+'), _ladder(T, L, '-')
    if axis == 0:
        return {k: (p[k] + mi[k]) / 2 for k in p}
    return {k: mpmath.mpc(0, -1) * (p[k] - mi[k]) / 2 for k in p}


_INV = (2, 0, 1)   # dS/dx_a = (dR/dq_{_INV[a]})(y, z, x)


def S_harmonics(L, pt, order=2):
    """S^{(l,m)}(x, y, z) = R_l^m(y, z, x) (eq. slmdef) with gradient and Hessian."""
    x, y, z = pt
    R = solid_harmonics(L, y, z, x)
    dR = [_d(R, L, a) for a in range(3)]
    g = [dR[_INV[a]] for a in range(3)]
    h = None
    if order >= 2:
        h = [[_d(dR[_INV[a]], L, _INV[b]) for b in range(3)] for a in range(3)]
    return R, g, h


def basis_index(p):
    return [(l, m) for l in range(1, p + 1) for m in range(1, l + 1)]


# ---------------------------------------------------------------- fit (Step 2)

class _Mat:
    """Row-major list-of-lists matrix with [i, j] indexing (results of _lsq_pinv)."""

    def __init__(self, rows):
        self.r = rows

    def __getitem__(self, ij):
        return self.r[ij[0]][ij[1]]


def _lsq_pinv(M, w):
    """(Omega M)^+ Omega, Omega = diag(sqrt(w)), from the normal equations
    (M^T W M) X = M^T W (the unique weighted least-squares solution), by Cholesky."""
    rows, cols = len(M), len(M[0])
    AtW = [[M[i][j] * w[i] for i in range(rows)] for j in range(cols)]
    G = [[mpmath.fsum(AtW[a][i] * M[i][b] for i in range(rows)) for b in range(cols)]
         for a in range(cols)]
    Lc = [[mpmath.mpf(0)] * cols for _ in range(cols)]
    for j in range(cols):
        d = G[j][j] - mpmath.fsum(Lc[j][k] ** 2 for k in range(j))
        Lc[j][j] = mpmath.sqrt(d)
        for i in range(j + 1, cols):
            Lc[i][j] = (G[i][j] - mpmath.fsum(Lc[i][k] * Lc[j][k] for k in range(j))) / Lc[j][j]
    # forward then backward substitution, all right-hand sides (the columns of AtW) at once
    Y = [row[:] for row in AtW]
    for i in range(cols):
        for k in range(i):
            f = Lc[i][k]
            Yk = Y[k]
            Y[i] = [a - f * b for a, b in zip(Y[i], Yk)]
        Y[i] = [a / Lc[i][i] for a in Y[i]]
    for i in reversed(range(cols)):
        for k in range(i + 1, cols):
            f = Lc[k][i]
            Yk = Y[k]
            Y[i] = [a - f * b for a, b in zip(Y[i], Yk)]
        Y[i] = [a / Lc[i][i] for a in Y[i]]
    return _Mat(Y)


class PatchFit:
    """Frame, maps M_D, M_S', M_S and edge data of one patch (Steps 1-3), as the double
    oracle's PatchFit, in 40-digit arithmetic."""

    def __init__(self, q, node_xyz, node_nrm, edge_samples, weighted=True):
        self.q = self.p = q
        pt = edge_samples.shape[1]
        self.tw = gauss_legendre(pt)
        nx = [[_mp(v) for v in r] for r in node_xyz]
        nn = [[_mp(v) for v in r] for r in node_nrm]
        es = [[[_mp(v) for v in r] for r in edge_samples[e]] for e in range(4)]
        self.frame = Frame(es, nn, self.tw)
        self.xl = [self.frame.point(r) for r in nx]
        self.nl = [self.frame.vector(v) for v in nn]
        N = q * q
        tq, wq = gauss_legendre(q)
        lsw = [wq[a] * wq[b] for a in range(q) for b in range(q)] if weighted else [mpmath.mpf(1)] * N
        idx = basis_index(q)
        n_p = len(idx)
        H = [[mpmath.mpf(0)] * n_p for _ in range(N)]
        F = [[[mpmath.mpf(0)] * n_p for _ in range(N)] for _ in range(3)]
        for i in range(N):
            S, gS, _ = S_harmonics(q, self.xl[i], order=1)
            for n, (l, m) in enumerate(idx):
                H[i][n] = mpmath.sqrt(2) * S[(l, m)].imag
                for a in range(3):
                    F[a][i][n] = mpmath.sqrt(2) * gS[a][(l, m)].imag
        # block system of eq. dlpdensitylinearsystem2, unknowns [c0; c1; c2; c3]
        Z = [[0] * n_p for _ in range(N)]
        neg = lambda B: [[-v for v in r] for r in B]
        blocks = [[Z, neg(F[0]), neg(F[1]), neg(F[2])],
                  [F[0], Z, neg(F[2]), F[1]],
                  [F[1], F[2], Z, neg(F[0])],
                  [F[2], neg(F[1]), F[0], Z]]
        A = [sum((blocks[bi][bj][i] for bj in range(4)), []) for bi in range(4) for i in range(N)]
        Ap = _lsq_pinv(A, lsw * 4)                      # 4 n_p x 4 N
        self.M_D = [[Ap[r, j] for j in range(N)] for r in range(4 * n_p)]
        self.M_Sp = [[sum(Ap[r, k * N + j] * self.nl[j][k - 1] for k in (1, 2, 3))
                      for j in range(N)] for r in range(4 * n_p)]
        Bm = [[sum(F[a][i][n] * self.nl[i][a] for a in range(3)) for n in range(n_p)]
              for i in range(N)]
        Bp = _lsq_pinv(Bm, lsw)                         # n_p x N
        HBp = [[sum(H[i][n] * Bp[n, j] for n in range(n_p)) for j in range(N)] for i in range(N)]
        MDH = [[sum(self.M_D[r][i] * HBp[i][j] for i in range(N)) for j in range(N)]
               for r in range(4 * n_p)]
        self.M_S = [[Bp[r, j] for j in range(N)] for r in range(n_p)] + MDH
        # edges (Step 3)
        self.edges_local = [[self.frame.point(r) for r in es[e]] for e in range(4)]
        self.edge_coef = [edge_coefficients(self.edges_local[e], self.tw) for e in range(4)]
        self.edge_tangent = [[poly_eval(self.edge_coef[e], t)[1] for t in self.tw[0]]
                             for e in range(4)]


# ---------------------------------------------------------------- target steps (4-8)

def _qmul(f, g):
    """Quaternion product (eq. qprule) of 4-lists."""
    f0, fv, g0, gv = f[0], f[1:], g[0], g[1:]
    s = f0 * g0 - _dot(fv, gv)
    c = _cross(fv, gv)
    return [s] + [f0 * gv[a] + g0 * fv[a] + c[a] for a in range(3)]


def _chord_far(coef, x, pt):
    """True if the chord root of the edge (the straight-chord preimage of the target) lies
    outside the Bernstein ellipse of radius rho_far: the edge is integrated by plain GL."""
    a = poly_eval(coef, mpmath.mpf(-1))[0]
    b = poly_eval(coef, mpmath.mpf(1))[0]
    m = [(a[c] + b[c]) / 2 for c in range(3)]
    d = [(b[c] - a[c]) / 2 for c in range(3)]
    dd = _dot(d, d)
    v = _sub(x, m)
    ts = complex(float(_dot(d, v) / dd), float(mpmath.sqrt(_dot(_cross(d, v), _cross(d, v))) / dd))
    return bernstein_radius(ts) > rho_far(pt)


def _terms(p, slp):
    """(l, m, j, k, weight) of the translation sums: eq. cdlp1dintegral (j >= 2, weight
    C_{j,l} T_{jk,lm}) or Theorem thm:cslp1form (j >= 1, weight D_{j,l} T_{jk,lm})."""
    out = []
    for (l, m) in basis_index(p):
        for j in range(1 if slp else 2, l + 1):
            for k in range(-j, j + 1):
                if abs(m - k) > l - j:
                    continue
                T = mpmath.sqrt(mpmath.binomial(l + m, j + k) * mpmath.binomial(l - m, j - k))
                if slp:
                    c = mpmath.factorial(j - 1) * mpmath.factorial(l - j) / mpmath.factorial(l)
                else:
                    c = mpmath.factorial(j - 2) * mpmath.factorial(l - j) / mpmath.factorial(l - 1)
                out.append((l, m, j, k, c * T))
    return out


def far_pair_weights(fit, x, nu_t, correction, node_xyz, node_nrm, node_wt):
    """S, D, S', D' weights of one far pair (target not a node of the patch), 40 digits,
    returned as double arrays.  Raises ValueError if an edge is not in the far class."""
    p, pt = fit.p, len(fit.tw[0])
    fr = fit.frame
    X = [_mp(v) for v in x]
    NT = [_mp(v) for v in nu_t]
    xl, nl = fr.point(X), fr.vector(NT)
    for e in range(4):
        if not _chord_far(fit.edge_coef[e], xl, pt):
            raise ValueError("edge %d is not in the far class" % e)
    # u: +-normal of the nearest node, pointing from the patch to the target
    dd = [_dot(_sub(xl, r), _sub(xl, r)) for r in fit.xl]
    n = min(range(len(dd)), key=lambda i: dd[i])
    u = fit.nl[n] if _dot(_sub(xl, fit.xl[n]), fit.nl[n]) >= 0 else _scale(fit.nl[n], -1)
    jk = [(j, k) for j in range(1, p + 1) for k in range(0, j + 1)]
    zero = lambda: mpmath.mpc(0)
    V = {t: zero() for t in jk}
    Q = {t: [zero() for _ in range(4)] for t in jk}
    dQ = {t: [zero() for _ in range(4)] for t in jk}
    Om = [mpmath.mpf(0)] * 4
    dOm = [mpmath.mpf(0)] * 4
    t_gl, w_gl = fit.tw
    for e in range(4):                              # Steps 5-6, far class
        for i in range(pt):
            r = fit.edges_local[e][i]
            rp = fit.edge_tangent[e][i]
            d = _sub(xl, r)
            R2 = _dot(d, d)
            R = mpmath.sqrt(R2)
            w1 = w_gl[i] / R
            w3 = w_gl[i] / (R2 * R)
            dn = _dot(d, nl)
            a = [w1 * nl[c] - w3 * dn * d[c] for c in range(3)]
            _, gS, hS = S_harmonics(p, r)
            for (j, k) in jk:
                g = [gS[c][(j, k)] for c in range(3)]
                cjk = _cross(g, rp)
                hjk = [sum(hS[c][b][(j, k)] * rp[b] for b in range(3)) for c in range(3)]
                V[(j, k)] += w1 * _dot(d, cjk)
                qd = _qmul([0] + d, [0] + hjk)
                qa = _qmul([0] + a, [0] + hjk)
                for c in range(4):
                    Q[(j, k)][c] += w1 * qd[c]
                    dQ[(j, k)][c] += qa[c]
            for c in range(3):
                Om[1 + c] += -w1 * rp[c]
                dOm[1 + c] += w3 * dn * rp[c]
            dOm[0] += -w3 * _dot(_cross(rp, d), nl)
            Om[0] += w_gl[i] * _dot(_cross(d, u), rp) / (R * (R + _dot(d, u)))
    # Steps 4, 7, 8
    S, gS, hS = S_harmonics(p, xl)

    def X_(tab, j, k):          # X^{(j,k)} with X^{(j,-k)} = (-1)^k conj X^{(j,k)}
        v = tab[(j, abs(k))]
        if k >= 0:
            return v
        s = (-1) ** (-k)
        return [s * mpmath.conj(c) for c in v] if isinstance(v, list) else s * mpmath.conj(v)

    idx = basis_index(p)
    four_pi = 4 * mpmath.pi
    Ia = {lm: [zero() for _ in range(4)] for lm in idx}
    dIa = {lm: [zero() for _ in range(4)] for lm in idx}
    for (l, m, j, k, wt) in _terms(p, False):
        s = S[(l - j, m - k)]
        gs = sum(nl[c] * gS[c][(l - j, m - k)] for c in range(3))
        q, dq = X_(Q, j, k), X_(dQ, j, k)
        for c in range(4):
            Ia[(l, m)][c] += q[c] * s * wt
            dIa[(l, m)][c] += (dq[c] * s + q[c] * gs) * wt
    sl = {lm: zero() for lm in idx}
    for (l, m, j, k, wt) in _terms(p, True):
        sl[(l, m)] += X_(V, j, k) * S[(l - j, m - k)] * wt
    Omq = [-Om[0], Om[1], Om[2], Om[3]]
    dOmq = [-dOm[0], dOm[1], dOm[2], dOm[3]]
    sq2 = mpmath.sqrt(2)
    Dq, dDq, Psi = {}, {}, {}
    for (l, m) in idx:
        g = [gS[c][(l, m)] for c in range(3)]
        hn = [sum(hS[c][b][(l, m)] * nl[b] for b in range(3)) for c in range(3)]
        Ig = _qmul(Omq, [0] + g)
        dIg = [u1 + u2 for u1, u2 in zip(_qmul(dOmq, [0] + g), _qmul(Omq, [0] + hn))]
        Dq[(l, m)] = [-sq2 * ((Ia[(l, m)][c] + Ig[c]) / four_pi).imag for c in range(4)]
        dDq[(l, m)] = [-sq2 * ((dIa[(l, m)][c] + dIg[c]) / four_pi).imag for c in range(4)]
        Psi[(l, m)] = sq2 * ((sl[(l, m)] - S[(l, m)] * Om[0]) / four_pi).imag
    sign = [1, -1, -1, -1]
    r_D = [sign[c] * Dq[lm][c] for c in range(4) for lm in idx]
    Eq = {lm: _qmul([0] + nl, Dq[lm]) for lm in idx}
    r_Sp = [sign[c] * Eq[lm][c] for c in range(4) for lm in idx]
    r_Dp = [sign[c] * dDq[lm][c] for c in range(4) for lm in idx]
    r_S = [Psi[lm] for lm in idx] + r_D
    N = len(fit.M_D[0])

    def rowmap(r, M):
        return [sum(r[i] * M[i][j] for i in range(len(r))) for j in range(N)]

    W = {"S": [v * fr.s for v in rowmap(r_S, fit.M_S)], "D": rowmap(r_D, fit.M_D),
         "Sp": rowmap(r_Sp, fit.M_Sp), "Dp": [v / fr.s for v in rowmap(r_Dp, fit.M_D)]}
    if correction:                                  # the smooth rule (eq. dlpsplitting)
        for j in range(N):
            rj = [_mp(v) for v in node_xyz[j]]
            nj = [_mp(v) for v in node_nrm[j]]
            wj = _mp(node_wt[j])
            d = _sub(X, rj)
            R2 = _dot(d, d)
            R = mpmath.sqrt(R2)
            R3 = R2 * R
            dn, dnt = _dot(d, nj), _dot(d, NT)
            W["S"][j] -= wj / (four_pi * R)
            W["D"][j] -= wj * dn / (four_pi * R3)
            W["Sp"][j] -= -wj * dnt / (four_pi * R3)
            W["Dp"][j] -= wj * (_dot(nj, NT) / R3 - 3 * dn * dnt / (R3 * R2)) / four_pi
    return {k: np.array([float(v) for v in W[k]]) for k in W}


def pair_weights_exact(surface, targets, t, P, correction=True, fits=None):
    """Far-pair weights of (target t, patch P) with 40 digits, for a surface / targets dict
    of the double oracle's format.  `fits` caches the 40-digit patch fits by patch."""
    with mpmath.workdps(DPS):
        a, b = int(surface["node_off"][P]), int(surface["node_off"][P + 1])
        ea, eb = int(surface["edge_off"][P]), int(surface["edge_off"][P + 1])
        xyz = np.asarray(surface["node_xyz"])[:, a:b].T
        nrm = np.asarray(surface["node_nrm"])[:, a:b].T
        wt = np.asarray(surface["node_wt"])[a:b]
        pt = (eb - ea) // 4
        edges = np.asarray(surface["edge_xyz"])[:, ea:eb].T.reshape(4, pt, 3)
        if fits is None or P not in fits:
            f = PatchFit(int(surface["order"][P]), xyz, nrm, edges)
            if fits is not None:
                fits[P] = f
        else:
            f = fits[P]
        if int(targets["self_patch"][t]) == P:
            raise ValueError("self target: not a far pair")
        return far_pair_weights(f, np.asarray(targets["xyz"])[:, t],
                                np.asarray(targets["nrm"])[:, t], correction, xyz, nrm, wt)
