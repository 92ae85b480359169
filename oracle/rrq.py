"""Per-pair RRQ weights for S, D, S', D' (Steps 4-8 and the matrix-row remark).

Oracle module (test infrastructure only).

For a target x (normal nu') and a source patch P, the weights W_K satisfy
sum_j W_K[j] f_j ~= K[f](x) restricted to P, for nodal data f.  They are formed
as in the remark after the algorithm in Sec. 4: the target row of moments is
multiplied with the patch's nodal-to-coefficient map (Step 2 skipped).

Steps, in the paper's order:
  Step 4  target harmonics S^{(a,b)}(x), grad, Hessian (Sec. 3.4)
  Step 5  per edge: root t0 and effective SSQ weights (ssq.py)
  Step 6  line integrals Q^{jk} (eq. qjkdef2), V^{jk} (eq. vjkdef), Omega
          (eqs. lineintegrals, solidangle) and, for D', their target
          derivatives (eq. dprimelineintegrals)
  Step 7  translation into I[alpha~] (eq. cdlp1dintegral), I[gamma]
          (Sec. 3.7), the SLP integrals of Theorem thm:cslp1form
  Step 8  D^{(l,m)} = -sqrt(2) Im(I[alpha~] + I[gamma]) (eq. wlmdef) and the rows
          for S (Theorem thm:slpreduction), S' (Sec. 3.6) and D' (Sec. 3.7).

Readings (all listed in the design notes):
* The SLP solid-angle term carries the factor 1/(4 pi) of (1/4pi) d omega_0 =
  -grad G . nu da (the proof of Theorem thm:dlp1form); the statement of
  Theorem thm:cslp1form omits it.
* S': with the quaternion product of eq. qprule, nu' . grad G = -[(0,nu')(0,grad G)]_0,
  so S'[sigma] = +[(0,nu') sum D^{(l,m)} w^{(l,m)}]_0 with the same D^{(l,m)}
  as the DLP (one sign differs from the printed final formula of Sec. 3.6).
* grad_x Omega_0 is taken from the Biot-Savart form -oint (r'(t) x (x - r)) /
  |x - r|^3 dt, which has the clean 1/|x-r|^3 singularity; it equals the
  derivative of eq. solidangle (the four-term expression of eq.
  dprimelineintegrals) but needs no adaptive integration.
* u: on-surface self targets use u = nu' (exterior one-sided limit, remark
  after Theorem thm:dlp1form); other targets use u = +-nu_n of the nearest node,
  signed to point from the patch to the target.
* On-surface self targets return the principal value for D and S' by the jump
  relations (the fitted density's own value at x).
* The correction weights subtract the smooth rule K(x, r_j) w_j for r_j != x
  (eq. dlpsplitting).
"""
import math

import numpy as np

from .harmonics import S_harmonics, H_basis, T_coef, C_coef, D_coef
from .quaternion import qmul, pure
from .ssq import EdgeQuadrature, omega0_edge

FOUR_PI = 4.0 * math.pi
SQRT2 = math.sqrt(2.0)
QSIGN = np.array([1.0, -1.0, -1.0, -1.0])   # [q c]_0 = q0 c0 - q1 c1 - q2 c2 - q3 c3


def choose_u(fit, xl, nl, self_node):
    if self_node is not None and self_node >= 0:
        return nl.copy()
    dd = np.sum((fit.xl - xl[None, :]) ** 2, axis=1)
    n = int(np.argmin(dd))
    sgn = 1.0 if (xl - fit.xl[n]) @ fit.nl[n] >= 0 else -1.0
    return sgn * fit.nl[n]


def line_integrals(fit, xl, nl, u, ptilde):
    """Steps 5-6, summed over the four edges of the closed boundary:

    V^{jk}  = oint [(x - r) x grad S^{jk}(r)] . dr / |x - r|            (eq. vjkdef)
    Q^{jk}  = oint (0, (x - r)/|x - r|)(0, d grad S^{jk}(r))            (eq. qjkdef2)
    dQ^{jk} = d/dnu' Q^{jk}                                   (eq. dprimelineintegrals)
    Omega   = (Omega_0, -oint dr / |x - r|)                  (eqs. solidangle, lineintegrals)
    dOmega  = d/dnu' Omega, with grad Omega_0 = -oint r' x (x - r) / |x - r|^3 dt
    for j >= 1 (V), j >= 2 (Q), 0 <= k <= j, in the order of fit.jk.
    """
    n_jk = len(fit.jk)
    V = np.zeros(n_jk, dtype=np.complex128)
    Q = np.zeros((n_jk, 4), dtype=np.complex128)
    dQ = np.zeros((n_jk, 4), dtype=np.complex128)
    Om = np.zeros(4)      # (Omega_0, Omega_vec)
    dOm = np.zeros(4)     # d/dnu' of the same
    stats = {"near_edges": 0, "newton_iters": 0, "newton_fail": 0}
    for e in range(4):
        coef = fit.edge_coef[e]
        samples = fit.edges_local[e]
        eq = EdgeQuadrature(coef, samples, xl, ptilde)
        stats["near_edges"] += int(eq.near)
        stats["newton_iters"] += eq.newton_iters
        stats["newton_fail"] += int(not eq.converged)
        rp = fit.edge_tangent[e]
        d = xl[None, :] - samples                      # (ptilde, 3)
        w1, w3 = eq.w1, eq.w3
        dn = d @ nl
        a = w1[:, None] * nl[None, :] - (w3 * dn)[:, None] * d
        c = fit.edge_c[e]                              # (ptilde, n_jk, 3)
        h = fit.edge_h[e]
        V += np.einsum('i,ia,ina->n', w1, d, c)
        Q += np.einsum('i,inq->nq', w1, qmul(pure(d)[:, None, :], pure(h)))
        dQ += np.einsum('inq->nq', qmul(pure(a)[:, None, :], pure(h)))
        Om[1:] += -np.sum(w1[:, None] * rp, axis=0)
        dOm[1:] += np.sum((w3 * dn)[:, None] * rp, axis=0)
        dOm[0] += -np.sum(w3 * (np.cross(rp, d) @ nl))
        Om[0] += omega0_edge(coef, xl, u, eq, ptilde)
    return V, Q, dQ, Om, dOm, stats


_TERMS = {}


def translation_terms(p):
    """Index lists of the sums of eq. cdlp1dintegral (j >= 2, weight C_{j,l} T_{jk,lm}) and
    Theorem thm:cslp1form (j >= 1, weight D_{j,l} T_{jk,lm}) over -j <= k <= j with
    |m - k| <= l - j, for every basis function (l, m), 1 <= m <= l <= p."""
    if p in _TERMS:
        return _TERMS[p]
    idx = [(l, m) for l in range(1, p + 1) for m in range(1, l + 1)]
    jk_pos = {jk: n for n, jk in enumerate((j, k) for j in range(1, p + 1) for k in range(0, j + 1))}
    out = {}
    for name, j0, wfun in (("dlp", 2, C_coef), ("slp", 1, D_coef)):
        rows = []
        for ii, (l, m) in enumerate(idx):
            for j in range(j0, l + 1):
                for k in range(-j, j + 1):
                    if abs(m - k) > l - j:
                        continue
                    sgn = 1.0 if k >= 0 else (-1.0) ** (-k)
                    rows.append((ii, jk_pos[(j, abs(k))], k < 0, sgn, l - j, m - k,
                                 wfun(j, l) * T_coef(j, k, l, m)))
        cols = list(zip(*rows))
        out[name] = dict(ii=np.array(cols[0]), n=np.array(cols[1]), neg=np.array(cols[2]),
                         sgn=np.array(cols[3]), a=np.array(cols[4]), b=np.array(cols[5]),
                         w=np.array(cols[6]))
    out["idx"] = idx
    _TERMS[p] = out
    return out


def _gather(X, tm):
    """X^{(j,k)} for the term list, using X^{(j,-k)} = (-1)^k conj X^{(j,k)}."""
    v = X[tm["n"]]
    neg = tm["neg"]
    if v.ndim == 2:
        neg = neg[:, None]
        sgn = tm["sgn"][:, None]
    else:
        sgn = tm["sgn"]
    return np.where(neg, np.conj(v), v) * sgn


def moments_rows(fit, xl, nl, V, Q, dQ, Om, dOm):
    """Steps 4, 7, 8: D^{(l,m)}, Psi^{(l,m)}, dD^{(l,m)} and the rows r_D, r_S', r_S, r_D'.

    I[alpha~]^{lm} = 1/(4pi) sum_j C_{j,l} sum_k Q^{jk} S^{(l-j,m-k)}(x) T_{jk,lm}
    I[gamma]^{lm}  = 1/(4pi) (-Omega_0, Omega_vec)(0, grad S^{lm}(x))
    D^{lm}         = -sqrt(2) Im(I[alpha~] + I[gamma])
    Psi^{lm}       = sqrt(2) Im 1/(4pi)[sum_j D_{j,l} sum_k V^{jk} S^{(l-j,m-k)}(x) T_{jk,lm}
                                        - S^{lm}(x) Omega_0]
    dD^{lm}        = d/dnu' D^{lm} by the product rule (Sec. 3.7).
    Reading: (-Omega_0, Omega_vec) is the integral of the 1-form whose exterior
    derivative is (0, grad G)(0, nu) da; with omega_0 as printed in eq. omega0def
    and the boundary oriented by the normal, oint omega_0 = +4pi int grad G . nu da,
    so the scalar part enters with a minus sign (pinned by brute force).
    """
    p = fit.p
    S, gS, hS = S_harmonics(p, xl)
    terms = translation_terms(p)
    idx = terms["idx"]
    n_p = len(idx)
    td, ts = terms["dlp"], terms["slp"]
    s_d = S[td["a"], p + td["b"]]
    gs_d = np.einsum('c,cn->n', nl, gS[:, td["a"], p + td["b"]])
    Qg = _gather(Q, td)
    dQg = _gather(dQ, td)
    Ia = np.zeros((n_p, 4), dtype=np.complex128)
    dIa = np.zeros((n_p, 4), dtype=np.complex128)
    np.add.at(Ia, td["ii"], Qg * (s_d * td["w"])[:, None])
    np.add.at(dIa, td["ii"], (dQg * s_d[:, None] + Qg * gs_d[:, None]) * td["w"][:, None])
    ls = np.array([l for (l, m) in idx])
    ms = np.array([m for (l, m) in idx])
    gS_lm = gS[:, ls, p + ms].T                          # (n_p, 3)
    hS_lm = np.einsum('abn,b->na', hS[:, :, ls, p + ms], nl)
    Omq = np.array([-Om[0], Om[1], Om[2], Om[3]], dtype=np.complex128)
    dOmq = np.array([-dOm[0], dOm[1], dOm[2], dOm[3]], dtype=np.complex128)
    Ig = qmul(Omq[None, :], pure(gS_lm))
    dIg = qmul(dOmq[None, :], pure(gS_lm)) + qmul(Omq[None, :], pure(hS_lm))
    Dq = -SQRT2 * ((Ia + Ig) / FOUR_PI).imag
    dDq = -SQRT2 * ((dIa + dIg) / FOUR_PI).imag
    sl = np.zeros(n_p, dtype=np.complex128)
    np.add.at(sl, ts["ii"], _gather(V, ts) * S[ts["a"], p + ts["b"]] * ts["w"])
    Psi = SQRT2 * ((sl - S[ls, p + ms] * Om[0]) / FOUR_PI).imag
    Eq = qmul(pure(nl)[None, :], Dq)
    r_D = (Dq * QSIGN[None, :]).T.reshape(-1)
    r_Sp = (Eq * QSIGN[None, :]).T.reshape(-1)
    r_Dp = (dDq * QSIGN[None, :]).T.reshape(-1)
    r_S = np.concatenate([Psi, r_D])
    return r_D, r_Sp, r_S, r_Dp


def pair_weights(fit, x, nu_t, self_node=-1, ptilde=None, onsurf_pv=True):
    """Raw RRQ weights (S, D, S', D'), each of length q^2, for one (target, patch) pair."""
    if ptilde is None:
        ptilde = 2 * fit.p
    fr = fit.frame
    xl = fr.point(x)
    nl = fr.vector(nu_t)
    u = choose_u(fit, xl, nl, self_node)
    V, Q, dQ, Om, dOm, stats = line_integrals(fit, xl, nl, u, ptilde)
    r_D, r_Sp, r_S, r_Dp = moments_rows(fit, xl, nl, V, Q, dQ, Om, dOm)
    W_D = r_D @ fit.M_D
    W_Sp = r_Sp @ fit.M_Sp
    W_S = (r_S @ fit.M_S) * fr.s
    W_Dp = (r_Dp @ fit.M_D) / fr.s
    if self_node is not None and self_node >= 0 and onsurf_pv:
        _, gH = H_basis(fit.p, xl)
        g = gH                                  # (3, n_p)
        eD = np.concatenate([np.zeros(g.shape[1]), -g[0], -g[1], -g[2]]) @ fit.M_D
        ng = nl @ g
        cr = np.cross(nl[None, :], g.T).T      # (3, n_p)
        eSp = np.concatenate([ng, cr[0], cr[1], cr[2]]) @ fit.M_Sp
        W_D = W_D - 0.5 * eD
        W_Sp = W_Sp + 0.5 * eSp
    return {"S": W_S, "D": W_D, "Sp": W_Sp, "Dp": W_Dp}, stats


def smooth_kernels(x, nu_t, r, nu, w):
    """K(x, r_j) w_j for the four kernels (the smooth rule of eq. dlpsplitting)."""
    d = x[None, :] - r
    R2 = np.sum(d * d, axis=1)
    R = np.sqrt(R2)
    R3 = R2 * R
    dn = np.sum(d * nu, axis=1)
    dnt = d @ nu_t
    kS = 1.0 / (FOUR_PI * R)
    kD = dn / (FOUR_PI * R3)
    kSp = -dnt / (FOUR_PI * R3)
    kDp = (nu @ nu_t / R3 - 3.0 * dn * dnt / (R3 * R2)) / FOUR_PI
    return {"S": kS * w, "D": kD * w, "Sp": kSp * w, "Dp": kDp * w}
