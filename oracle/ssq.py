"""Singularity-swap quadrature on one patch edge (Sec. 2.4, Sec. 3.5, Step 5).

Oracle module (test infrastructure only).

For a boundary curve r(t), t in [-1, 1] (the degree ptilde-1 interpolant through
ptilde Gauss-Legendre samples) and a target x:
* t0 is the complex root of sum_c (r_c(t) - x_c)^2 (eq. complexparameter),
  found by Newton from the chord start (reading: the paper defers the root
  finder to the singularity-swap literature; chord start, tolerance 1e-14,
  at most 60 iterations, root with Im t0 > 0; an edge whose Newton solve does
  not converge is integrated with the plain rule and counted as a failure).
* the moments I_k^{(m)} = int t^k ((t - t0)(t - conj t0))^{-m/2} dt (eq.
  ssq1dintegrals) for m = 1, 3 come from recurrences derived by differentiating
  t^{k-1} R(t), R = |t - t0|;
* lambda^{(m)} = U^T I^{(m)} (eq. ssq1dintegrals2), so that
  int f(t) / |r(t) - x|^m dt ~= sum_i w_i^{(m)} f(t_i) with
  w_i^{(m)} = lambda_i^{(m)} |t_i - t0|^m / |r_i - x|^m.
  The recurrence and the product U^T I are evaluated in 40-digit arithmetic
  (mpmath) from the double-precision t0 and nodes, then rounded: in double
  precision this route loses up to 8 digits for ptilde >= 12 (growth of the
  forward recurrence for |t0| > 1 and cancellation in U^T I), so the oracle
  evaluates the paper's formula exactly instead.
* An edge whose root lies outside the Bernstein ellipse of radius rho_far is
  integrated with the plain GL rule (reading: the near/far split of point (3)
  in the introduction; rho_far = 10^{8/ptilde}).
"""
import math

import mpmath
import numpy as np

from .fit import gauss_legendre, poly_eval

NEWTON_TOL = 1e-14
NEWTON_MAXIT = 60


def rho_far(ptilde):
    return 10.0 ** (8.0 / ptilde)


def bernstein_radius(t):
    """rho(t) = |t + sqrt(t-1) sqrt(t+1)|, the branch with rho >= 1."""
    t = complex(t)
    z = t + np.sqrt(t - 1) * np.sqrt(t + 1)
    r = abs(z)
    return max(r, 1.0 / r) if r > 0 else 1.0


def chord_start(coef, x):
    """Root of the distance function for the straight chord through r(-1), r(1)."""
    a, _ = poly_eval(coef, np.array(-1.0))
    b, _ = poly_eval(coef, np.array(1.0))
    m = 0.5 * (a + b)
    d = 0.5 * (b - a)
    dd = d @ d
    v = x - m
    return complex(d @ v / dd, np.linalg.norm(np.cross(d, v)) / dd)


def newton_root(coef, x, t_start, tol=NEWTON_TOL, maxit=NEWTON_MAXIT):
    """Newton on f(t) = sum_c (r_c(t) - x_c)^2.  Returns (t0, iterations, converged)."""
    t = complex(t_start)
    for it in range(1, maxit + 1):
        r, dr = poly_eval(coef, np.array(t))
        e = r - x
        f = np.sum(e * e)
        fp = 2.0 * np.sum(e * dr)
        dt = f / fp
        t = t - dt
        if abs(dt) <= tol * max(1.0, abs(t)):
            if t.imag < 0:
                t = t.conjugate()
            return t, it, True
    if t.imag < 0:
        t = t.conjugate()
    return t, maxit, False


def moments(t0, n):
    """I^{(1)}_k and I^{(3)}_k, k = 0..n-1, for ((t-a)^2 + b^2)^{-m/2} on [-1, 1]."""
    a, b = t0.real, abs(t0.imag)
    b2 = b * b
    abs2 = a * a + b2
    Rp = math.sqrt((1 - a) ** 2 + b2)
    Rm = math.sqrt((1 + a) ** 2 + b2)
    I1 = np.zeros(n)
    I3 = np.zeros(n)
    I1[0] = math.asinh((1 - a) / b) + math.asinh((1 + a) / b)
    if n > 1:
        I1[1] = (Rp - Rm) + a * I1[0]
    for k in range(2, n):
        # k I_k = [t^{k-1} R] + (2k-1) a I_{k-1} - (k-1)|t0|^2 I_{k-2}
        bnd = Rp - (-1.0) ** (k - 1) * Rm
        I1[k] = (bnd + (2 * k - 1) * a * I1[k - 1] - (k - 1) * abs2 * I1[k - 2]) / k
    I3[0] = ((1 - a) / (b2 * Rp)) - ((-1 - a) / (b2 * Rm))
    if n > 1:
        I3[1] = -(1.0 / Rp - 1.0 / Rm) + a * I3[0]
    for k in range(2, n):
        I3[k] = I1[k - 2] + 2 * a * I3[k - 1] - abs2 * I3[k - 2]
    return I1, I3


_MP_DPS = 40
_U_EXACT = {}


def _exact_U(t):
    """U = V^{-1} of the (double) GL nodes, in 40-digit arithmetic."""
    key = tuple(t)
    if key not in _U_EXACT:
        with mpmath.workdps(_MP_DPS):
            n = len(t)
            V = mpmath.matrix(n, n)
            for i in range(n):
                for k in range(n):
                    V[i, k] = mpmath.mpf(float(t[i])) ** k
            _U_EXACT[key] = V ** -1
    return _U_EXACT[key]


def lagrange_moments_exact(t0, t):
    """lambda^{(1)}, lambda^{(3)} = U^T I^{(1)}, U^T I^{(3)} with the moment recurrences of
    `moments` carried out in 40-digit arithmetic (inputs: double t0 and nodes t)."""
    n = len(t)
    U = _exact_U(t)
    with mpmath.workdps(_MP_DPS):
        a = mpmath.mpf(float(t0.real))
        b = abs(mpmath.mpf(float(t0.imag)))
        b2 = b * b
        abs2 = a * a + b2
        Rp = mpmath.sqrt((1 - a) ** 2 + b2)
        Rm = mpmath.sqrt((1 + a) ** 2 + b2)
        I1 = [mpmath.asinh((1 - a) / b) + mpmath.asinh((1 + a) / b)]
        I1.append((Rp - Rm) + a * I1[0])
        for k in range(2, n):
            I1.append(((Rp - (-1) ** (k - 1) * Rm) + (2 * k - 1) * a * I1[k - 1]
                       - (k - 1) * abs2 * I1[k - 2]) / k)
        I3 = [(1 - a) / (b2 * Rp) - (-1 - a) / (b2 * Rm)]
        I3.append(-(1 / Rp - 1 / Rm) + a * I3[0])
        for k in range(2, n):
            I3.append(I1[k - 2] + 2 * a * I3[k - 1] - abs2 * I3[k - 2])
        lam1 = [float(mpmath.fsum(U[k, i] * I1[k] for k in range(n))) for i in range(n)]
        lam3 = [float(mpmath.fsum(U[k, i] * I3[k] for k in range(n))) for i in range(n)]
    return np.array(lam1), np.array(lam3)


class EdgeQuadrature:
    """Effective weights of one (target, edge) pair for 1/|r-x| and 1/|r-x|^3."""

    def __init__(self, coef, samples, x, ptilde):
        t, w = gauss_legendre(ptilde)
        self.t = t
        d = x[None, :] - samples
        dist = np.sqrt(np.sum(d * d, axis=1))
        self.dist = dist
        ts = chord_start(coef, x)
        self.t_start = ts
        self.newton_iters = 0
        self.converged = True
        self.near = False
        self.t0 = None
        rf = rho_far(ptilde)
        if bernstein_radius(ts) <= rf:
            t0, its, ok = newton_root(coef, x, ts)
            self.newton_iters = its
            self.converged = ok
            self.t0 = t0
            if ok and bernstein_radius(t0) <= rf:
                self.near = True
        if self.near:
            lam1, lam3 = lagrange_moments_exact(self.t0, t)
            tt = np.sqrt((t - self.t0.real) ** 2 + self.t0.imag ** 2)
            self.w1 = lam1 * tt / dist
            self.w3 = lam3 * tt ** 3 / dist ** 3
        else:
            self.w1 = w / dist
            self.w3 = w / dist ** 3


def omega0_integrand(coef, x, u, t):
    """omega_0 of eq. omega0def along the edge, per unit dt."""
    r, dr = poly_eval(coef, t)
    d = x[None, :] - r
    R = np.sqrt(np.sum(d * d, axis=1))
    num = np.sum(np.cross(d, u[None, :]) * dr, axis=1)
    return num / (R * (R + d @ u))


def graded_panels(t0, ptilde, maxlev=60):
    """Dyadic panels of [-1, 1], bisected until each panel sees t0 at Bernstein
    radius >= rho_far in its own scaled coordinate (reading of the remark on the
    solid angle in Sec. 3.5: 'very mild adaptive integration')."""
    rf = rho_far(ptilde)
    out = []
    stack = [(-1.0, 1.0, 0)]
    while stack:
        lo, hi, lev = stack.pop()
        c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
        if lev >= maxlev or bernstein_radius((t0 - c) / h) >= rf:
            out.append((lo, hi))
        else:
            stack.append((c, hi, lev + 1))
            stack.append((lo, c, lev + 1))
    out.sort()
    return out


def omega0_edge(coef, x, u, eq, ptilde):
    """Contribution of one edge to Omega_0 (eq. solidangle)."""
    t, w = gauss_legendre(ptilde)
    if not eq.near:
        return float(np.sum(w * omega0_integrand(coef, x, u, t)))
    total = 0.0
    for lo, hi in graded_panels(eq.t0, ptilde):
        c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
        total += h * float(np.sum(w * omega0_integrand(coef, x, u, c + h * t)))
    return total
