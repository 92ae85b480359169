"""Solid harmonics, the RRQ harmonic basis and the translation coefficients.

Oracle module (test infrastructure only).

* Regular solid harmonics R_l^m (Sec. 2.3, eqs. ylmdef and rlmdef): Racah
  normalisation, associated Legendre functions from the Rodrigues formula,
  i.e. WITHOUT the Condon-Shortley phase.  Values come from the three-term
  recurrence of eq. associatelegendrerecurrence written in Cartesian form
  (reading: the sign in front of the diagonal step is dropped, consistent with
  the statement that the phase is removed).
* Derivatives use the ladder identities of solid harmonics: d/dz, d/dx -+ i d/dy
  each map degree l to a multiple of a degree l-1 harmonic.  The identities are
  pinned in the tests against finite differences and the Laplacian.
* S^{(l,m)}(x,y,z) = R_l^m(y,z,x) (eq. slmdef), H^{(l,m)} = sqrt(2) Im S^{(l,m)}
  (eq. hlmslmconnection; basis of Theorem thm:trianglebasis, eq. hlmdef).
* T_{jk,lm} (eq. tjklmdef), C_{j,l} (Theorem thm:dlp1form), D_{j,l}
  (Theorem thm:cslp1form).

Tables are indexed [..., l, m + L] for 0 <= l <= L, -L <= m <= L; entries with
|m| > l are zero.
"""
import math

import numpy as np


def _zeros(shape, L):
    return np.zeros(tuple(shape) + (L + 1, 2 * L + 1), dtype=np.complex128)


def regular_solid_harmonics(L, pts):
    """R_l^m(pts) for 0<=l<=L, |m|<=l.  pts: (..., 3) real.  Returns (..., L+1, 2L+1).

    Recurrence (Cartesian form of eq. associatelegendrerecurrence, phase dropped):
      R_0^0 = 1
      R_l^l = sqrt((2l-1)/(2l)) (x+iy) R_{l-1}^{l-1}
      R_l^m = ((2l-1) z R_{l-1}^m - r^2 sqrt((l-1+m)(l-1-m)) R_{l-2}^m) / sqrt(l^2-m^2)
      R_l^{-m} = (-1)^m conj(R_l^m)
    """
    pts = np.asarray(pts, dtype=np.float64)
    x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
    r2 = x * x + y * y + z * z
    w = x + 1j * y
    out = _zeros(pts.shape[:-1], L)
    out[..., 0, L] = 1.0
    for l in range(1, L + 1):
        out[..., l, L + l] = math.sqrt((2 * l - 1) / (2 * l)) * w * out[..., l - 1, L + l - 1]
        for m in range(0, l):
            prev2 = out[..., l - 2, L + m] if l >= 2 else 0.0
            out[..., l, L + m] = ((2 * l - 1) * z * out[..., l - 1, L + m]
                                  - r2 * math.sqrt((l - 1 + m) * (l - 1 - m)) * prev2) / math.sqrt(l * l - m * m)
    for l in range(1, L + 1):
        for m in range(1, l + 1):
            out[..., l, L - m] = (-1) ** m * np.conj(out[..., l, L + m])
    return out


def _ladder(T, which):
    """Apply one derivative to a table of solid harmonics (as polynomials).

    which = 'z':  dz R_l^m  = sqrt((l+m)(l-m))       R_{l-1}^m
    which = '-':  (dx - i dy) R_l^m = sqrt((l+m)(l+m-1)) R_{l-1}^{m-1}
    which = '+':  (dx + i dy) R_l^m = -sqrt((l-m)(l-m-1)) R_{l-1}^{m+1}
    """
    L = T.shape[-2] - 1
    out = np.zeros_like(T)
    for l in range(1, L + 1):
        for m in range(-l, l + 1):
            if which == 'z':
                if abs(m) <= l - 1:
                    out[..., l, L + m] = math.sqrt((l + m) * (l - m)) * T[..., l - 1, L + m]
            elif which == '-':
                if abs(m - 1) <= l - 1:
                    out[..., l, L + m] = math.sqrt((l + m) * (l + m - 1)) * T[..., l - 1, L + m - 1]
            else:
                if abs(m + 1) <= l - 1:
                    out[..., l, L + m] = -math.sqrt((l - m) * (l - m - 1)) * T[..., l - 1, L + m + 1]
    return out


def _d(T, axis):
    """Cartesian partial derivative (axis 0,1,2 = x,y,z) of a harmonic table."""
    if axis == 2:
        return _ladder(T, 'z')
    p, mi = _ladder(T, '+'), _ladder(T, '-')
    if axis == 0:
        return 0.5 * (p + mi)
    return -0.5j * (p - mi)


def regular_solid_harmonics_derivs(L, pts, order=2):
    """Values, gradient (..., 3, L+1, 2L+1) and Hessian (..., 3, 3, L+1, 2L+1) of R_l^m."""
    R = regular_solid_harmonics(L, pts)
    g = np.stack([_d(R, a) for a in range(3)], axis=-3)
    if order < 2:
        return R, g, None
    h = np.stack([np.stack([_d(g[..., a, :, :], b) for b in range(3)], axis=-3)
                  for a in range(3)], axis=-4)
    return R, g, h


# cyclic permutation of eq. slmdef: S(x,y,z) = R(y,z,x)
_PERM = (1, 2, 0)        # argument of R is pts[..., _PERM]
_INV = (2, 0, 1)         # dS/dx_a = (dR/dq_{_INV[a]})(q)


def S_harmonics(L, pts, order=2):
    """S^{(l,m)} = R_l^m(y,z,x) with gradient and Hessian w.r.t. (x,y,z) (eq. slmdef)."""
    pts = np.asarray(pts, dtype=np.float64)
    q = pts[..., list(_PERM)]
    R, gR, hR = regular_solid_harmonics_derivs(L, q, order)
    g = gR[..., list(_INV), :, :]
    h = None
    if hR is not None:
        h = hR[..., list(_INV), :, :, :][..., list(_INV), :, :]
    return R, g, h


def basis_index(p):
    """Ordering of the basis H^{(l,m)}, 1 <= m <= l <= p: l major, m minor."""
    return [(l, m) for l in range(1, p + 1) for m in range(1, l + 1)]


def H_basis(p, pts):
    """H^{(l,m)} = sqrt(2) Im S^{(l,m)} (eq. hlmslmconnection) and its gradient.

    Returns H (..., n_p) and gradH (..., 3, n_p) in basis_index order.
    """
    S, gS, _ = S_harmonics(p, pts, order=1)
    idx = basis_index(p)
    H = np.stack([math.sqrt(2.0) * S[..., l, p + m].imag for (l, m) in idx], axis=-1)
    gH = np.stack([math.sqrt(2.0) * gS[..., :, l, p + m].imag for (l, m) in idx], axis=-1)
    return H, gH


def binom(n, k):
    if k < 0 or k > n or n < 0:
        return 0
    return math.comb(n, k)


def T_coef(j, k, l, m):
    """T_{jk,lm} = C(l+m, j+k)^{1/2} C(l-m, j-k)^{1/2} (eq. tjklmdef)."""
    return math.sqrt(binom(l + m, j + k) * binom(l - m, j - k))


def C_coef(j, l):
    """C_{j,l} = int_0^1 t^{j-2}(1-t)^{l-j} dt = (j-2)!(l-j)!/(l-1)!  (Theorem thm:dlp1form)."""
    return math.factorial(j - 2) * math.factorial(l - j) / math.factorial(l - 1)


def D_coef(j, l):
    """D_{j,l} = int_0^1 t^{j-1}(1-t)^{l-j} dt = (j-1)!(l-j)!/l!  (Theorem thm:cslp1form)."""
    return math.factorial(j - 1) * math.factorial(l - j) / math.factorial(l)
