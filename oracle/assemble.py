"""Assembly of the sparse near-field correction matrix over a near list.

Oracle module (test infrastructure only).

Input/output follow the problem statement of Sec. 4 (patches, nodes, targets
in; weights out) and the matrix splitting D = D_smooth + D_RRQ of Sec. 5
(eq. dlpsplitting): for every near pair (target x, patch P) a block of q_P^2
weights per kernel, stored target-major in the order of the near list.
"""
import numpy as np

from .fit import PatchFit
from .rrq import pair_weights, smooth_kernels

KERNELS = ("S", "D", "Sp", "Dp")


def patch_arrays(surface, P):
    a, b = int(surface["node_off"][P]), int(surface["node_off"][P + 1])
    ea, eb = int(surface["edge_off"][P]), int(surface["edge_off"][P + 1])
    xyz = np.asarray(surface["node_xyz"])[:, a:b].T
    nrm = np.asarray(surface["node_nrm"])[:, a:b].T
    wt = np.asarray(surface["node_wt"])[a:b]
    pt = (eb - ea) // 4
    edges = np.asarray(surface["edge_xyz"])[:, ea:eb].T.reshape(4, pt, 3)
    return xyz, nrm, wt, edges


def fit_patch(surface, P, lsq_solver="qr", weighted=True):
    q = int(surface["order"][P])
    xyz, nrm, wt, edges = patch_arrays(surface, P)
    return PatchFit(q, xyz, nrm, edges, lsq_solver, weighted)


def pair_offsets(surface, targets):
    order = np.asarray(surface["order"], dtype=np.int64)
    near_patch = np.asarray(targets["near_patch"], dtype=np.int64)
    sizes = order[near_patch] ** 2
    off = np.zeros(len(near_patch) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def pair_block(surface, targets, fits, t, P, correction=True, onsurf_pv=True, lsq_solver="qr",
               weighted=True):
    """Weights (dict of 4 arrays of length q_P^2) of the near pair (target t, patch P).  `fits`
    caches the patch fits by patch index (one cache per solver and weighting)."""
    if P not in fits:
        fits[P] = fit_patch(surface, P, lsq_solver, weighted)
    fit = fits[P]
    x = np.asarray(targets["xyz"])[:, t]
    nu_t = np.asarray(targets["nrm"])[:, t]
    self_node = -1
    if int(targets["self_patch"][t]) == P:
        self_node = int(targets["self_node"][t])
    pt = (int(surface["edge_off"][P + 1]) - int(surface["edge_off"][P])) // 4
    W, stats = pair_weights(fit, x, nu_t, self_node, pt, onsurf_pv)
    if correction:
        xyz, nrm, wt, _ = patch_arrays(surface, P)
        keep = np.ones(len(wt), dtype=bool)
        if self_node >= 0:
            keep[self_node] = False
        K = smooth_kernels(x, nu_t, xyz[keep], nrm[keep], wt[keep])
        for k in KERNELS:
            W[k] = W[k].copy()
            W[k][keep] -= K[k]
    return W, stats


def assemble(surface, targets, correction=True, onsurf_pv=True, pairs=None):
    """All near-pair weight blocks, target-major CSR order.

    Returns (weights dict of 4 arrays [nweights], pair_off [nnz+1]).  With
    `pairs` (indices into the near list) only those blocks are computed and the
    others stay zero.
    """
    off = pair_offsets(surface, targets)
    near_ptr = np.asarray(targets["near_ptr"], dtype=np.int64)
    near_patch = np.asarray(targets["near_patch"], dtype=np.int64)
    owner = np.repeat(np.arange(len(near_ptr) - 1), np.diff(near_ptr))
    out = {k: np.zeros(off[-1]) for k in KERNELS}
    fits = {}
    idx = range(len(near_patch)) if pairs is None else pairs
    for i in idx:
        W, _ = pair_block(surface, targets, fits, int(owner[i]), int(near_patch[i]),
                          correction, onsurf_pv)
        for k in KERNELS:
            out[k][off[i]:off[i + 1]] = W[k]
    return out, off
