"""Parity gates of the GPU tests: the HIP library's weight blocks against the oracle's.

Test infrastructure (imports the oracle).  For one near pair (target t, patch P) and kernel K:

* flat gate:      ||W_gpu - W_or||_inf <= 1e-11 ||W_raw||_inf, and for a smooth nodal density f
                  |(W_gpu - W_or) . f| <= 1e-11 sum_j |W_raw,j f_j|,
  W_raw being the oracle block without the smooth-rule subtraction;
* ensemble gate (blocks that miss a flat bound): ||W_gpu - W_or||_inf <= 1e-11 ||W_raw||_inf
  + ENS_FACTOR * spread and the same for the potential, where spread = max_e ||W_e - W_or||
  over an ensemble of oracle evaluations of the same pair: ENS_MEMBERS members whose inputs
  (target point and normal, the patch's nodes, normals and weights, its edge samples) are
  each moved by one relative ulp (2^-52) with independent random signs, and one member whose
  least-squares fits are solved by the SVD instead of Householder QR (another backward-stable
  solver: the rounding of the fit itself, which input perturbations do not reproduce when the
  fit is ill-conditioned).

The ensemble measures how far rounding moves the oracle's own block: for pairs about a patch
diameter away the weights are small differences of large moment x map products, and one ulp
of input moves single weights by up to 4e-4 of the block on the benchmark surface; the
potential of a smooth density does not see most of those directions.  ENS_FACTOR = 3 was
chosen from the measured distribution of ||W_gpu - W_or|| / spread (largest ratio 1.6 over
the parity workloads).
"""
import numpy as np

from oracle.assemble import pair_block

TOL = 1e-11
ENS_MEMBERS = 16
ENS_FACTOR = 3.0
KERNELS = ("S", "D", "Sp", "Dp")
ULP = 2.0 ** -52


def smooth_density(surf):
    x, y, z = surf["node_xyz"]
    return 0.7 + x * x - 0.4 * y * z + 0.3 * z + 0.2 * x * y * z


def sub_problem(surf, tg, t, P):
    """The pair (t, P) as a one-patch surface and a one-target list (same numbers)."""
    a, b = int(surf["node_off"][P]), int(surf["node_off"][P + 1])
    ea, eb = int(surf["edge_off"][P]), int(surf["edge_off"][P + 1])
    s1 = dict(npatch=1, order=np.array([surf["order"][P]]), node_off=np.array([0, b - a]),
              edge_off=np.array([0, eb - ea]),
              node_xyz=np.array(surf["node_xyz"][:, a:b]), node_nrm=np.array(surf["node_nrm"][:, a:b]),
              node_wt=np.array(surf["node_wt"][a:b]), edge_xyz=np.array(surf["edge_xyz"][:, ea:eb]))
    selfp = 0 if int(tg["self_patch"][t]) == P else -1
    t1 = dict(ntarget=1, xyz=np.array(tg["xyz"][:, t:t + 1]), nrm=np.array(tg["nrm"][:, t:t + 1]),
              self_patch=np.array([selfp]), self_node=np.array([int(tg["self_node"][t]) if selfp == 0 else -1]),
              near_ptr=np.array([0, 1]), near_patch=np.array([0]))
    return s1, t1


def _bump(a, rng):
    return a * (1.0 + ULP * rng.choice([-1.0, 1.0], size=np.shape(a)))


def perturbed(s1, t1, member, P, t, seed=0):
    """Ensemble member `member`: every input of the pair moved by one relative ulp."""
    rs = np.random.default_rng((seed, member, 1, P))
    rt = np.random.default_rng((seed, member, 2, t))
    s2 = dict(s1)
    for k in ("node_xyz", "node_nrm", "node_wt", "edge_xyz"):
        s2[k] = _bump(s1[k], rs)
    t2 = dict(t1)
    t2["xyz"] = _bump(t1["xyz"], rt)
    t2["nrm"] = _bump(t1["nrm"], rt)
    return s2, t2


def oracle_pair(surf, tg, t, P, correction, onsurf_pv, fits=None, weighted=True):
    s1, t1 = sub_problem(surf, tg, t, P)
    f = {} if fits is None else fits
    ref, _ = pair_block(s1, t1, f, 0, 0, correction, onsurf_pv, weighted=weighted)
    raw, _ = pair_block(s1, t1, f, 0, 0, False, onsurf_pv, weighted=weighted)
    return ref, raw


def ensemble_spread(surf, tg, t, P, ref, correction, onsurf_pv, members=ENS_MEMBERS, cache=None,
                    weighted=True):
    """Per kernel: max over the ensemble (input perturbations and the SVD-solved fits) of
    ||W_e - W_or||_inf and of |(W_e - W_or) . f|."""
    s1, t1 = sub_problem(surf, tg, t, P)
    f = smooth_density(s1)
    sw = {k: 0.0 for k in ref}
    sp = {k: 0.0 for k in ref}
    for e in range(members):
        s2, t2 = perturbed(s1, t1, e, P, t)
        key = (e, P)
        fits = {}
        if cache is not None:
            if key in cache:
                fits = {0: cache[key]}
        We, _ = pair_block(s2, t2, fits, 0, 0, correction, onsurf_pv, weighted=weighted)
        if cache is not None:
            cache[key] = fits[0]
        for k in ref:
            d = We[k] - ref[k]
            sw[k] = max(sw[k], float(np.max(np.abs(d))))
            sp[k] = max(sp[k], float(abs(d @ f)))
    key = ("svd", P)
    fits = {0: cache[key]} if cache is not None and key in cache else {}
    Ws, _ = pair_block(s1, t1, fits, 0, 0, correction, onsurf_pv, "svd", weighted)
    if cache is not None:
        cache[key] = fits[0]
    for k in ref:
        d = Ws[k] - ref[k]
        sw[k] = max(sw[k], float(np.max(np.abs(d))))
        sp[k] = max(sp[k], float(abs(d @ f)))
    return sw, sp


def block_scales(raw, f, s):
    """Scales of one pair's blocks for the relative gates: ||W_raw,K||_inf (weights) and
    sum_j |W_raw,K,j f_j| (potential), with a floor from the single layer of the same pair
    for the kernels whose exact block can vanish (D and S' for a target in the plane of a
    flat patch, D' likewise): ||W_S|| / s for D and S', ||W_S|| / s^2 for D', s being the
    patch size (the weights of S scale with s, those of D and S' are dimensionless, those of
    D' scale with 1/s)."""
    fS_w = float(np.max(np.abs(raw["S"])))
    fS_p = float(np.sum(np.abs(raw["S"] * f)))
    expo = {"S": 0, "D": 1, "Sp": 1, "Dp": 2}
    sw, sp = {}, {}
    for k in raw:
        sw[k] = max(float(np.max(np.abs(raw[k]))), fS_w / s ** expo[k])
        sp[k] = max(float(np.sum(np.abs(raw[k] * f))), fS_p / s ** expo[k])
    return sw, sp


def compare_pairs(surf, tg, pairs, gpu_block=None, gpu_pot=None, correction=True,
                  onsurf_pv=True, flat_potential=False, tol=TOL, label="", strict=True,
                  weighted=True):
    """Check GPU results of the near pairs `pairs` (indices into the near list) against the
    oracle with the gates above.  gpu_block(i) gives the dict of the four weight blocks of
    pair i, gpu_pot(i) the dict of its four pair potentials for the density smooth_density
    (either may be None).  With flat_potential every pair's potential must meet the flat
    bound with no allowance; `weighted` selects the oracle's least-squares weighting.
    Returns per-kernel statistics; asserts the gates (with strict=False it counts the blocks
    that miss them instead)."""

    def gate(ok, *what):
        if strict:
            assert ok, (label,) + what
        return bool(ok)

    owner = np.repeat(np.arange(len(tg["near_ptr"]) - 1), np.diff(tg["near_ptr"]))
    cache, fitc = {}, {}
    st = {k: dict(max_rel=0.0, max_abs=0.0, wmax=0.0, pot=0.0, ens=0, ratio=[], pratio=[],
                  pot_flat=0, n=0, fail=0) for k in KERNELS}
    for i in pairs:
        t, P = int(owner[i]), int(tg["near_patch"][i])
        fits = fitc.setdefault(P, {})
        ref, raw = oracle_pair(surf, tg, t, P, correction, onsurf_pv, fits, weighted)
        s1, _ = sub_problem(surf, tg, t, P)
        f = smooth_density(s1)
        sw, sp = block_scales(raw, f, fits[0].frame.s)
        g = gpu_block(i) if gpu_block is not None else None
        gp = gpu_pot(i) if gpu_pot is not None else None
        ew, ep = {}, {}
        for k in KERNELS:
            if g is not None and g[k] is None:
                continue
            if g is not None:
                assert np.all(np.isfinite(g[k])), (label, k, i)
                ew[k] = float(np.max(np.abs(g[k] - ref[k])))
                ep[k] = float(abs((g[k] - ref[k]) @ f))
            else:
                assert np.isfinite(gp[k]), (label, k, i)
                ew[k] = 0.0
                ep[k] = float(abs(gp[k] - ref[k] @ f))
            s = st[k]
            s["n"] += 1
            s["max_rel"] = max(s["max_rel"], ew[k] / sw[k])
            s["max_abs"] = max(s["max_abs"], ew[k])
            s["wmax"] = max(s["wmax"], float(np.max(np.abs(ref[k]))))
            s["pot"] = max(s["pot"], ep[k] / sp[k])
            s["pot_flat"] += ep[k] <= tol * sp[k]
            if flat_potential and not gate(ep[k] <= tol * sp[k], "flat potential gate", k, i,
                                           ep[k] / sp[k]):
                s["fail"] += 1
        miss = [k for k in ew if ew[k] > tol * sw[k] or ep[k] > tol * sp[k]]
        if not miss:
            continue
        spw, spp = ensemble_spread(surf, tg, t, P, ref, correction, onsurf_pv, cache=cache,
                                   weighted=weighted)
        for k in miss:
            s = st[k]
            s["ens"] += 1
            if ew[k] > tol * sw[k]:
                s["ratio"].append((ew[k] - tol * sw[k]) / max(spw[k], 1e-300))
            if ep[k] > tol * sp[k]:
                s["pratio"].append((ep[k] - tol * sp[k]) / max(spp[k], 1e-300))
            ok = gate(ew[k] <= tol * sw[k] + ENS_FACTOR * spw[k], "weights", k, i, ew[k], sw[k],
                      spw[k])
            ok &= gate(ep[k] <= tol * sp[k] + ENS_FACTOR * spp[k], "potential", k, i, ep[k],
                       sp[k], spp[k])
            s["fail"] += not ok
    summary = {}
    for k, s in st.items():
        if not s["n"]:
            continue
        r = np.array(s["ratio"]) if s["ratio"] else np.zeros(0)
        pr = np.array(s["pratio"]) if s["pratio"] else np.zeros(0)
        summary[k] = dict(
            pairs=s["n"], max_rel=s["max_rel"], global_maxnorm=s["max_abs"] / max(s["wmax"], 1e-300),
            potential=s["pot"], potential_flat_rate=s["pot_flat"] / s["n"], ensemble_pairs=s["ens"],
            ratio_p50=float(np.median(r)) if len(r) else 0.0, ratio_max=float(r.max()) if len(r) else 0.0,
            pot_ratio_max=float(pr.max()) if len(pr) else 0.0,
            gate_pass_rate=1.0 - s["fail"] / s["n"])
    if strict:
        print(f"parity {label} over {len(pairs)} pairs: " + "; ".join(
            f"{k}: rel {v['max_rel']:.1e}, pot {v['potential']:.1e} "
            f"(flat {v['potential_flat_rate']:.2f}), ensemble {v['ensemble_pairs']} "
            f"(ratio p50 {v['ratio_p50']:.2f} max {v['ratio_max']:.2f}, "
            f"pot {v['pot_ratio_max']:.2f})" for k, v in summary.items()), flush=True)
    return summary
