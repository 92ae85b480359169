"""Patch frame and the harmonic density fits (source-only Steps 1-3).

Oracle module (test infrastructure only).

Readings of the paper used here (each listed in the design notes):
* Patch shape: quadrilateral patch with a q x q tensor Gauss-Legendre grid of
  collocation nodes and four boundary edges ordered counter-clockwise about the
  outward normal.  The basis order is p = q, so n_p = q(q+1)/2 < q^2 and the
  collocation systems (eqs. dlpdensitylinearsystem2, slpdensitylinearsystem,
  sprimedensitylinearsystem) are solved in the weighted least-squares sense,
  with weights sqrt(w_a w_b) (the tensor GL parameter weights), by Householder
  QR (backward stable, as the conditioning discussion of Sec. 5.1 requires).
* Frame (Step 1 input/output, Sec. 5.1): origin at the mean of the four corner
  points, z axis along (c2 - c0) x (c3 - c1) oriented with the mean node normal,
  x axis along the first side, scale s = longest side, so that local
  coordinates are R^T (r - o) / s.
"""
import numpy as np

from .harmonics import H_basis, S_harmonics


def gauss_legendre(n):
    """n-point Gauss-Legendre nodes (increasing) and weights on [-1, 1]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return t, w


def monomial_interp_matrix(t):
    """U = V^{-1}, V_{ik} = t_i^k (the matrix U of Sec. 3.5)."""
    V = np.vander(t, len(t), increasing=True)
    return np.linalg.inv(V)


def edge_coefficients(samples):
    """Legendre coefficients (ptilde, 3) of the degree ptilde-1 interpolant through the GL
    samples of an edge: c_k = (2k+1)/2 sum_i w_i P_k(t_i) s_i (exact, since the GL rule
    integrates P_k times the interpolant exactly).  The paper leaves the representation of
    the boundary curve open; the Legendre basis keeps its evaluation well conditioned."""
    n = samples.shape[0]
    t, w = gauss_legendre(n)
    P = np.polynomial.legendre.legvander(t, n - 1)          # P[i, k] = P_k(t_i)
    return ((2 * np.arange(n) + 1) / 2.0)[:, None] * (P.T @ (w[:, None] * samples))


def poly_eval(coef, t):
    """Value and t-derivative of the Legendre series sum_k coef[k] P_k(t) (coef (n, 3)) at t
    (real or complex), by the three-term recurrence P_{k+1} = ((2k+1) t P_k - k P_{k-1})/(k+1)
    and P'_{k+1} = P'_{k-1} + (2k+1) P_k."""
    t = np.asarray(t)
    n = coef.shape[0]
    dt = np.result_type(t, coef)
    p_prev, p = np.zeros(t.shape, dtype=dt), np.ones(t.shape, dtype=dt)
    d_prev, d = np.zeros(t.shape, dtype=dt), np.zeros(t.shape, dtype=dt)
    val = p[..., None] * coef[0]
    der = np.zeros_like(val)
    for k in range(0, n - 1):
        p_next = ((2 * k + 1) * t * p - k * p_prev) / (k + 1)
        d_next = d_prev + (2 * k + 1) * p
        p_prev, p = p, p_next
        d_prev, d = d, d_next
        val = val + p[..., None] * coef[k + 1]
        der = der + d[..., None] * coef[k + 1]
    return val, der


class Frame:
    """Translation, rotation and scaling of one patch (Step 1 input/output)."""

    def __init__(self, edge_samples, node_nrm):
        corners = []
        for e in range(4):
            coef = edge_coefficients(edge_samples[e])
            v, _ = poly_eval(coef, np.array(-1.0))
            corners.append(v)
        c = np.array(corners)
        self.corners = c
        self.o = c.mean(axis=0)
        ez = np.cross(c[2] - c[0], c[3] - c[1])
        ez /= np.linalg.norm(ez)
        if ez @ node_nrm.mean(axis=0) < 0:
            ez = -ez
        ex = (c[1] - c[0]) - ((c[1] - c[0]) @ ez) * ez
        ex /= np.linalg.norm(ex)
        ey = np.cross(ez, ex)
        self.R = np.stack([ex, ey, ez], axis=1)          # columns are the local axes
        self.s = max(np.linalg.norm(c[(k + 1) % 4] - c[k]) for k in range(4))

    def point(self, x):
        return (np.asarray(x) - self.o) @ self.R / self.s

    def vector(self, v):
        return np.asarray(v) @ self.R


def _weighted_pinv(M, w, solver="qr"):
    """(Omega M)^+ Omega with Omega = diag(sqrt(w)), via Householder QR (default) or, as an
    independent backward-stable alternative used to measure conditioning, the SVD."""
    sw = np.sqrt(w)
    if solver == "svd":
        X, *_ = np.linalg.lstsq(sw[:, None] * M, np.diag(sw), rcond=None)
        return X
    Q, Rr = np.linalg.qr(sw[:, None] * M)
    return np.linalg.solve(Rr, Q.T * sw[None, :])


def dlp_system_matrix(gH):
    """Block system matrix of eq. dlpdensitylinearsystem2 from grad H at the nodes.

    gH: (N, 3, n_p).  Returns A (4N, 4n_p); unknowns ordered [c0; c1; c2; c3].
    """
    F1, F2, F3 = gH[:, 0, :], gH[:, 1, :], gH[:, 2, :]
    Z = np.zeros_like(F1)
    return np.block([[Z, -F1, -F2, -F3],
                     [F1, Z, -F3, F2],
                     [F2, F3, Z, -F1],
                     [F3, -F2, F1, Z]])


class PatchFit:
    """Coefficient maps of one patch (Steps 1-2 with Step 2 skipped as in the
    matrix-row remark after the algorithm: maps from nodal data to coefficients).

    M_D  (4 n_p, N): nodal mu            -> quaternion c of eq. dlpdensappr
    M_Sp (4 n_p, N): nodal sigma         -> quaternion w of eq. sprimedensappr
    M_S  (5 n_p, N): nodal sigma         -> [d; g] of Theorem thm:slpreduction
    """

    def __init__(self, q, node_xyz, node_nrm, edge_samples, lsq_solver="qr", weighted=True):
        self.q = q
        self.p = q
        self.frame = Frame(edge_samples, node_nrm)
        self.xl = self.frame.point(node_xyz)
        self.nl = self.frame.vector(node_nrm)
        t, w = gauss_legendre(q)
        # least-squares row weights: the tensor GL parameter weights, or all ones (the
        # unweighted fit; the paper leaves the weighting open)
        self.lsw = np.outer(w, w).reshape(-1) if weighted else np.ones(q * q)
        H, gH = H_basis(self.p, self.xl)
        self.Hmat = H
        self.gH = gH
        N = node_xyz.shape[0]
        A = dlp_system_matrix(gH)
        self.A = A
        Ap = _weighted_pinv(A, np.tile(self.lsw, 4), lsq_solver)
        self.M_D = Ap[:, :N]
        self.M_Sp = sum(Ap[:, k * N:(k + 1) * N] * self.nl[None, :, k - 1] for k in (1, 2, 3))
        B = np.einsum('ikn,ik->in', gH, self.nl)
        self.B = B
        Bp = _weighted_pinv(B, self.lsw, lsq_solver)
        self.M_S = np.vstack([Bp, self.M_D @ H @ Bp])
        edges_local = [self.frame.point(edge_samples[e]) for e in range(4)]
        self.edges_local = np.array(edges_local)
        self.edge_coef = np.array([edge_coefficients(es) for es in edges_local])
        # Step 3 (source-only): harmonics at the edge nodes and the per-node
        # factors of the line integrals, for j >= 1, k >= 0:
        #   c^{jk}_i = grad S^{jk}(r_i) x r'(t_i)         (integrand of eq. vjkdef)
        #   h^{jk}_i = Hess S^{jk}(r_i) r'(t_i) = d(grad S^{jk})/dt   (eq. qjkdef2)
        pt = self.edges_local.shape[1]
        te, _ = gauss_legendre(pt)
        self.edge_tangent = np.array([poly_eval(self.edge_coef[e], te)[1] for e in range(4)])
        p = self.p
        self.jk = [(j, k) for j in range(1, p + 1) for k in range(0, j + 1)]
        cj = np.zeros((4, pt, len(self.jk), 3), dtype=np.complex128)
        hj = np.zeros((4, pt, len(self.jk), 3), dtype=np.complex128)
        for e in range(4):
            _, gS, hS = S_harmonics(p, self.edges_local[e])
            rp = self.edge_tangent[e]
            for n, (j, k) in enumerate(self.jk):
                cj[e, :, n] = np.cross(gS[:, :, j, p + k], rp)
                hj[e, :, n] = np.einsum('iab,ib->ia', hS[:, :, :, j, p + k], rp)
        self.edge_c = cj
        self.edge_h = hj
