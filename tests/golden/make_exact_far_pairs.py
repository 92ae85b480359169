"""Writes exact_far_pairs_star.npz: the weights of ten far pairs of the star-shaped benchmark
surface (1536 patches, order 8, node targets, near radius 1.5 patch diameters) computed by the
oracle's steps in 40-digit arithmetic (oracle/exact.py), rounded to double.  Calls only the
oracle and the seeded workload generator.

Run from the repository root:  python tests/golden/make_exact_far_pairs.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_far_pairs_star.npz")
NPAIRS = 10
SEED = 77


def _workload():
    from paper_2411_08342_amd import workloads as wl
    surf, tg, _ = wl.star()
    return surf, tg


def _far_pairs(surf, tg, n, seed):
    """Seeded pairs whose target is not a node of the patch and whose four edges all lie in
    the far class (no singularity swap), as the double oracle classifies them."""
    from oracle.assemble import fit_patch
    from oracle.ssq import EdgeQuadrature
    rng = np.random.default_rng(seed)
    owner = np.repeat(np.arange(tg["ntarget"]), np.diff(tg["near_ptr"]))
    out, fits = [], {}
    for i in rng.permutation(len(tg["near_patch"])):
        t, P = int(owner[i]), int(tg["near_patch"][i])
        if int(tg["self_patch"][t]) == P:
            continue
        if P not in fits:
            fits[P] = fit_patch(surf, P)
        f = fits[P]
        xl = f.frame.point(tg["xyz"][:, t])
        if any(EdgeQuadrature(f.edge_coef[e], f.edges_local[e], xl, 2 * f.p).near for e in range(4)):
            continue
        out.append(int(i))
        if len(out) == n:
            return sorted(out)
    raise RuntimeError("not enough far pairs")


def _one(i):
    from oracle.exact import pair_weights_exact
    surf, tg = _workload()
    owner = np.repeat(np.arange(tg["ntarget"]), np.diff(tg["near_ptr"]))
    W = pair_weights_exact(surf, tg, int(owner[i]), int(tg["near_patch"][i]), True)
    return i, W


def main():
    surf, tg = _workload()
    pairs = _far_pairs(surf, tg, NPAIRS, SEED)
    with ProcessPoolExecutor(min(len(pairs), os.cpu_count() or 1)) as ex:
        res = dict(ex.map(_one, pairs))
    np.savez(OUT, pairs=np.array(pairs, dtype=np.int64),
             **{k: np.stack([res[i][k] for i in pairs]) for k in ("S", "D", "Sp", "Dp")})
    print("wrote", OUT, "pairs", pairs)


if __name__ == "__main__":
    main()
