"""Benchmark: near-correction weights/sec (FP64, S/D/S'/D') for the star-shaped surface workload
(1536 quadrilateral patches of order 8, 98,304 on-surface targets, near radius 1.5 patch
diameters).  One step = the whole hot path on device-resident inputs: source-only plan
(frames, edge tables, least-squares fits), pair offsets, and assembly of the four kernels'
correction weights.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "near-correction weights/sec (FP64, S/D/S'/D') at ≤1e-11 err; batched vs plain"
FP64_VALU_PEAK = 78.6   # TFLOP/s, MI355X vector FP64 (256 CU x 2.4 GHz x 128 flop/clk)

# HBM traffic of the dominant kernel per launch, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this benchmark, scaled by the same counters for a 1 GiB copy
# (bench.py --copy-probe: FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the kernel
# source it was measured on (sha256 of csrc/rrq_batch.hip); null otherwise.
TRAFFIC = {"src_sha256": "90dfa7d221b8c7d25c5335b5f5ce7865dc75141df4643b54e0ac330ca982db8f",
           "fetch_bytes": 1641407026, "write_bytes": 3599471744}


def flops_per_pair(q):
    """Algorithmic FP64 flops of one (target, patch) pair at order q (p = q, ptilde = 2q, an FMA
    counted as 2), data-independent work only (Newton iterations and the extra panel points of
    near edges excluded):
      edge weights and contractions   4 [12 J1 pt + 72 J2 pt + 4 pt^2 + 90 pt]
      translations, target harmonics  32 tD + 8 tS + 64 tD + 50 (p+1)^2 + 200 n_p
      rows x maps                     2 q^2 17 n_p
    with J1 = p(p+3)/2 (j >= 1, k >= 0), J2 = J1 - 2 (j >= 2) and tD, tS the (l, m, j, k) term
    counts of the double- and single-layer translation sums (489 and 574 at p = 8): 378,306
    flops per pair at q = 8."""
    p, pt = q, 2 * q
    n_p = p * (p + 1) // 2
    J1 = p * (p + 3) // 2
    J2 = J1 - 2
    tD = tS = 0
    for l in range(1, p + 1):
        for m in range(1, l + 1):
            for j in range(1, l + 1):
                for k in range(-j, j + 1):
                    if abs(m - k) <= l - j:
                        tS += 1
                        if j >= 2:
                            tD += 1
    edges = 4 * (12 * J1 * pt + 72 * J2 * pt + 4 * pt * pt + 90 * pt)
    trans = 32 * tD + 8 * tS + 64 * tD + 50 * (p + 1) ** 2 + 200 * n_p
    return edges + trans + 2 * q * q * 17 * n_p


def kernel_src_sha():
    import hashlib
    path = os.path.join(ROOT, "paper_2411_08342_amd", "csrc", "rrq_batch.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def assemble_ms(asm, flags, reps):
    """Mean device time of whole rrq_assemble calls (binning, root pre-pass and pair kernels),
    from events on the stream the calls run on."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        asm.assemble(flags=flags)
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def _p99_bound(st):
    """Smallest of the iteration thresholds 2, 4, 6, 8, 12 that at most 1% of the Newton solves
    exceed (None if more than 1% take over 12)."""
    n = st["newton_slots"]
    for thr, over in zip((2, 4, 6, 8, 12), st["newton_over"]):
        if over <= 0.01 * n:
            return thr
    return None


def _newton_summary(st, ms, nweights):
    return {"assemble_ms": ms, "weights_per_s": 4 * nweights / (ms / 1e3),
            "newton_iters": st["newton_iters"], "newton_slots": st["newton_slots"],
            "newton_iters_mean": st["newton_iters"] / max(1, st["newton_slots"]),
            "newton_iters_p99_at_most": _p99_bound(st), "newton_iters_max": st["newton_max"],
            "newton_wave_iters": st["newton_wave_iters"],
            "newton_slots_over_2_4_6_8_12": st["newton_over"],
            "learned_accept": st["learned_accept"], "newton_fail": st["newton_fail"]}


def learned_form(rrq, reps=8, train_per_patch=110):
    """The learned Newton start on the star surface plus the 2048-patch torus: trained on
    about 2M samples the method produces on its own seeded training geometry (a deformed
    sphere and a torus with off-surface targets, kept apart from the evaluation surfaces),
    then plain and learned batched assemblies of the same near list compared on Newton
    iterations (mean, tail, per-wavefront), assembly time and weights."""
    import torch
    from paper_2411_08342_amd import workloads as wl
    t0 = time.perf_counter()
    surf, tg, _ = wl.learned_guess_training(per_patch=train_per_patch)
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    feat, dt, _ = rrq.collect_roots(plan, rrq.DeviceTargets(tg), 4 * len(tg["near_patch"]))
    plan.close()
    params, curve = rrq.mlp_train(feat, dt, steps=4000, batch=8192, lr=3e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del surf, tg
    surf, tg, _ = wl.star_torus()
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    asm = rrq.Assembler(plan, rrq.DeviceTargets(tg))
    flags = rrq.RRQ_F_CORRECTION | rrq.RRQ_F_ONSURF_PV
    out = {"workload": "star r=1+0.2ReY43+0.1ReY21 (1536 quads) + torus R=1 r=0.35 (2048 quads), "
                       "q=8, node targets, near 1.5 patch diameters",
           "pairs": int(len(tg["near_patch"])), "train_samples": int(feat.shape[1]),
           "train_s": t_train}
    c = curve.cpu().numpy()
    out["train_loss_first_last"] = [float(c[:10].mean()), float(c[-100:].mean())]
    sp = asm.assemble(flags=flags, stats=True)
    w_plain = {k: asm.out[k].clone() for k in rrq.KERNELS}
    plan.set_mlp(params)
    sl = asm.assemble(flags=flags | rrq.RRQ_F_LEARNED, stats=True)
    # the two forms alternate, so that slow drifts of the clock affect both alike; the tile
    # kernels are the same work in both, the forms differ in the root passes before them
    t = {"plain": [], "learned": []}
    pre = {"plain": [], "learned": []}
    for _ in range(reps):
        for name, fl in (("plain", flags), ("learned", flags | rrq.RRQ_F_LEARNED)):
            ms = assemble_ms(asm, fl, 1)
            st = asm.assemble(flags=fl, stats=True)
            t[name].append(ms)
            pre[name].append(ms - st["kernel_ms"])
    out["plain"] = _newton_summary(sp, float(np.mean(t["plain"])), asm.nweights)
    out["learned"] = _newton_summary(sl, float(np.mean(t["learned"])), asm.nweights)
    for name in ("plain", "learned"):
        out[name]["assemble_ms_runs"] = [round(v, 3) for v in t[name]]
        out[name]["outside_tile_kernel_ms"] = float(np.mean(pre[name]))
    out["max_rel_weight_dev_learned_vs_plain"] = max(
        ((asm.out[k] - w_plain[k]).abs().max() / w_plain[k].abs().max()).item()
        for k in rrq.KERNELS)
    plan.set_mlp(None)
    del asm, w_plain
    plan.close()
    torch.cuda.empty_cache()
    return out


def other_workload(rrq, name, steps=3):
    """A whole step (refit, pair offsets, assembly; one HIP graph, autotuned per order) on one
    of the other workloads, with each order's tile kernel against the FP64 roofline."""
    import torch
    from paper_2411_08342_amd import workloads as wl
    t0 = time.perf_counter()
    if name == "ellipsoids":
        surf, tg, _ = wl.ellipsoids_mixed_orders()
        desc = ("12 ellipsoids, semi-axes U[0.5, 2], 96..1536 quads each, per-patch order "
                "from {4, 6, 8, 10}, Poisson(150) off-surface targets per patch at "
                "1e-5..0.5 patch sizes, near 1 patch diameter")
    else:
        surf, tg, _ = wl.forty_spheres()
        desc = ("40 deformed spheres, 24,576 quads q=8, node targets and a 200k-point cloud at "
                "1e-6..0.3, near 1 patch diameter")
    t_gen = time.perf_counter() - t0
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    asm = rrq.Assembler(plan, rrq.DeviceTargets(tg))
    flags = rrq.RRQ_F_CORRECTION | rrq.RRQ_F_ONSURF_PV
    tune = rrq.autotune(asm, flags)
    graph = rrq.Graph(asm, flags)
    graph.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        graph.launch()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t1) / steps
    st = asm.assemble(flags=flags, stats=True)
    order = np.asarray(surf["order"])[np.asarray(tg["near_patch"])]
    per_order = {}
    for i, q in enumerate(rrq.ORDERS):
        npq = int(np.count_nonzero(order == q))
        if not npq:
            continue
        kms = st["order_kernel_ms"][i]
        tf = npq * flops_per_pair(q) / (kms / 1e3) / 1e12
        per_order[str(q)] = {"pairs": npq, "kernel_ms": kms, "tile": tune["order_tile"][i],
                             "grid": tune["order_grid"][i], "achieved_TFLOPs": tf,
                             "frac": tf / FP64_VALU_PEAK, "flops_per_pair": flops_per_pair(q)}
    out = {"workload": desc, "pairs": int(len(tg["near_patch"])),
           "weights_per_step": int(4 * asm.nweights), "ms_per_step": ms,
           "value": 4 * asm.nweights / (ms / 1e3), "unit": "weights/s", "steps": steps,
           "kernel_ms": st["kernel_ms"], "per_order": per_order,
           "near_edges": st["near_edges"], "newton_fail": st["newton_fail"],
           "panel_overflow": st["panel_overflow"], "nonfinite": st["nonfinite"],
           "generate_s": t_gen}
    graph.close()
    del asm
    plan.close()
    torch.cuda.empty_cache()
    return out


def potentials_form(rrq, asm, flags, w_ref, reps=3):
    """Potentials mode on the same near list: the correction applied to a smooth density
    without storing weights, timed like the assembly, and compared with rrq_apply on the
    assembled weights (max |difference| over targets relative to the largest potential)."""
    import torch
    x, y, z = asm.plan.dsurf.node_xyz
    dens = (0.7 + x * x - 0.4 * y * z + 0.3 * z + 0.2 * x * y * z).contiguous()
    ev = rrq.Evaluator(asm.plan, asm.dtg)
    st = [ev.potentials(dens, flags=flags, stats=True)[1] for _ in range(reps)]
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        got = ev.potentials(dens, flags=flags)
        b.record()
    torch.cuda.synchronize()
    for k in rrq.KERNELS:
        asm.out[k].copy_(w_ref[k])
    ref = asm.apply(dens)
    torch.cuda.synchronize()
    dev = max(((got[k] - ref[k]).abs().max() / ref[k].abs().max()).item() for k in rrq.KERNELS)
    del ev
    return {"call_ms": float(np.mean([a.elapsed_time(b) for a, b in evs])),
            "kernel_ms": float(np.mean([r["kernel_ms"] for r in st])),
            "max_rel_dev_vs_apply_of_weights": dev}


def build_workload(name):
    from paper_2411_08342_amd import workloads as wl
    if name == "star":
        surf, tg, dens = wl.star()
        desc = ("star r=1+0.2ReY43+0.1ReY21, 1536 quads q=8, 98304 node targets, "
                "near 1.5 patch diameters")
    elif name == "star-small":
        surf, tg, dens = wl.star(n=4)
        desc = "star, 96 quads q=8, node targets, near 1.5 patch diameters"
    elif name == "sphere":
        surf, tg, dens = wl.sphere_q6()
        desc = ("unit sphere, 6 quads q=6, 216 node targets and 200 off-surface targets "
                "1e-4..1e-1 away, near 1 patch diameter")
    else:
        raise SystemExit(f"unknown workload {name}")
    return surf, tg, desc


# ---------------------------------------------------------------------------------------
# CPU baseline: the oracle, as it stands, timed on the host cores.  The worker processes are
# started before this process initialises the GPU, each limited to one BLAS thread.
# ---------------------------------------------------------------------------------------
_W = {}


def _worker_init():
    from threadpoolctl import threadpool_limits
    _W["limits"] = threadpool_limits(limits=1)
    sys.path.insert(0, os.path.join(ROOT, "tests"))


def _worker_workload(name):
    if name not in _W:
        surf, tg, _ = build_workload(name)
        owner = np.repeat(np.arange(len(tg["near_ptr"]) - 1), np.diff(tg["near_ptr"]))
        _W[name] = (surf, tg, owner)
    return _W[name]


def _w_ready(name):
    _worker_workload(name)
    return os.getpid()


def _w_time(name, targets, seconds, keep):
    """The oracle on all near pairs of `targets` in order, until `seconds` have passed (at least
    one target).  Returns (elapsed s, weights, pairs, targets done, fits, blocks of the pairs
    listed in `keep` or of all pairs if keep is True)."""
    from oracle.assemble import pair_block
    surf, tg, _ = _worker_workload(name)
    fits, blocks = {}, {}
    nw = npairs = ntg = 0
    t0 = time.perf_counter()
    for t in targets:
        for i in range(tg["near_ptr"][t], tg["near_ptr"][t + 1]):
            W, _ = pair_block(surf, tg, fits, int(t), int(tg["near_patch"][i]))
            nw += 4 * len(W["S"])
            npairs += 1
            if keep is True or i in keep:
                blocks[int(i)] = (W, fits[int(tg["near_patch"][i])].frame.s)
        ntg += 1
        if seconds and time.perf_counter() - t0 > seconds:
            break
    return time.perf_counter() - t0, nw, npairs, ntg, len(fits), blocks


def _w_gate(name, pairs, gpu):
    """The parity gates of the tests (tests/_parity.py) on GPU blocks of `pairs`, counting
    instead of asserting."""
    from _parity import compare_pairs
    surf, tg, _ = _worker_workload(name)
    return compare_pairs(surf, tg, pairs, gpu_block=lambda i: gpu[i], strict=False)


def _merge_gate(parts):
    out = {}
    for part in parts:
        for k, v in part.items():
            if k not in out:
                out[k] = dict(v)
                continue
            o, n0, n1 = out[k], out[k]["pairs"], v["pairs"]
            for f in ("max_rel", "global_maxnorm", "potential", "ratio_max", "pot_ratio_max"):
                o[f] = max(o[f], v[f])
            for f in ("potential_flat_rate", "gate_pass_rate", "ratio_p50"):
                o[f] = (o[f] * n0 + v[f] * n1) / (n0 + n1)
            o["pairs"] = n0 + n1
            o["ensemble_pairs"] += v["ensemble_pairs"]
    return out


def start_cpu_pool(name, workers):
    """Worker processes for the oracle, started and warmed (workload built) before the GPU is
    touched."""
    import concurrent.futures as cf
    import multiprocessing as mp
    pool = cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"),
                                  initializer=_worker_init)
    pids = list(pool.map(_w_ready, [name] * workers))
    list(pool.map(_w_ready, ["sphere"] * workers))
    return pool, len(set(pids))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def exact_reference(name, surf, tg, gpu_block):
    """GPU and double oracle against the exact-arithmetic weights of ten far pairs of the
    benchmark surface (tests/golden, written from the oracle's steps in 40 digits): the
    largest difference relative to the pair's raw block and to the double oracle's rounding
    spread (one-ulp input perturbations, SVD-solved fits)."""
    path = os.path.join(ROOT, "tests", "golden", "exact_far_pairs_star.npz")
    if name != "star" or not os.path.exists(path):
        return None
    from _parity import oracle_pair, ensemble_spread
    g = np.load(path)
    owner = np.repeat(np.arange(len(tg["near_ptr"]) - 1), np.diff(tg["near_ptr"]))
    out = {"pairs": int(len(g["pairs"]))}
    for k in ("S", "D", "Sp", "Dp"):
        out[k] = {"gpu_rel_to_raw": 0.0, "oracle_rel_to_raw": 0.0, "gpu_over_spread": 0.0,
                  "oracle_over_spread": 0.0}
    for n, i in enumerate(g["pairs"]):
        t, P = int(owner[i]), int(tg["near_patch"][i])
        ref, raw = oracle_pair(surf, tg, t, P, True, True)
        spw, _ = ensemble_spread(surf, tg, t, P, ref, True, True)
        gb = gpu_block(int(i))
        for k in ("S", "D", "Sp", "Dp"):
            sc = float(np.max(np.abs(raw[k])))
            dg = float(np.max(np.abs(gb[k] - g[k][n])))
            do = float(np.max(np.abs(ref[k] - g[k][n])))
            o = out[k]
            o["gpu_rel_to_raw"] = max(o["gpu_rel_to_raw"], dg / sc)
            o["oracle_rel_to_raw"] = max(o["oracle_rel_to_raw"], do / sc)
            o["gpu_over_spread"] = max(o["gpu_over_spread"], dg / spw[k])
            o["oracle_over_spread"] = max(o["oracle_over_spread"], do / spw[k])
    return out


def cpu_baseline(pool, workers, name, surf, tg, gpu_block, seconds=10.0, seed=0, gate_pairs=150):
    """The oracle timed (i) on one core over all near pairs of a run of consecutive targets from
    a seeded start, (ii) on `workers` cores (one process each, a run from its own start), (iii)
    on `workers` cores over every pair of the unit-sphere workload (6 patches, q = 6: all of
    it); then the parity gates of the tests applied to the GPU blocks of the first
    `gate_pairs` sampled pairs and the flat potential gate to all of them."""
    rng = np.random.default_rng(seed)
    T = len(tg["near_ptr"]) - 1
    # consecutive targets (neighbouring nodes) share their near patches, so the patch fits are
    # amortised over the pairs as in a whole assembly; each leg starts at a seeded target
    starts = rng.integers(0, T, size=workers + 1)
    run = lambda a: [int((a + j) % T) for j in range(T)]
    # (i) one core
    dt, nw, npairs, ntg, nfit, blocks = pool.submit(_w_time, name, run(starts[0]), seconds,
                                                    True).result()
    single = dict(value=nw / dt, unit="weights/s", cores=1,
                  sample=f"all {npairs} near pairs of {ntg} consecutive targets from a seeded "
                         f"start ({nfit} patch fits included), {dt:.1f} s")
    # (ii) all workers, each from its own seeded start
    chunks = [run(a) for a in starts[1:]]
    t0 = time.perf_counter()
    res = list(pool.map(_w_time, [name] * workers, chunks, [seconds] * workers,
                        [set()] * workers))
    wall = time.perf_counter() - t0
    nw_all = sum(r[1] for r in res)
    allc = dict(value=nw_all / wall, unit="weights/s", cores=workers, kind="oracle",
                sample=f"all near pairs of {sum(r[3] for r in res)} targets, runs of consecutive "
                       f"targets from {workers} seeded starts ({sum(r[2] for r in res)} pairs, "
                       f"{sum(r[4] for r in res)} patch fits), one process per core, "
                       f"{wall:.1f} s wall")
    # (iii) the unit-sphere workload in full, static split by target
    s1, t1, _ = build_workload("sphere")
    T1 = len(t1["near_ptr"]) - 1
    chunks = [list(range(w * T1 // workers, (w + 1) * T1 // workers)) for w in range(workers)]
    t0 = time.perf_counter()
    res = list(pool.map(_w_time, ["sphere"] * workers, chunks, [0] * workers,
                        [set()] * workers))
    wall1 = time.perf_counter() - t0
    cfg1 = dict(value=sum(r[1] for r in res) / wall1, unit="weights/s", cores=workers,
                sample=f"unit sphere, 6 patches q=6: all {sum(r[2] for r in res)} pairs, "
                       f"{wall1:.1f} s wall")
    # parity gates on the sampled blocks (pair-wise, spread over the workers)
    pairs = sorted(blocks)
    gpu = {i: gpu_block(i) for i in pairs}
    gsel = pairs[:gate_pairs]
    parts = list(pool.map(_w_gate, [name] * workers, [gsel[w::workers] for w in range(workers)],
                          [{i: gpu[i] for i in gsel[w::workers]} for w in range(workers)]))
    gate = _merge_gate([p for p in parts if p])
    # flat potential gate (no allowance) over every sampled pair; the raw block is the
    # corrected one plus the smooth rule it subtracts
    if os.path.join(ROOT, "tests") not in sys.path:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _parity import block_scales, smooth_density, TOL
    from oracle.assemble import patch_arrays
    from oracle.rrq import smooth_kernels
    owner = np.repeat(np.arange(T), np.diff(tg["near_ptr"]))
    dens = smooth_density(surf)
    flat = {k: 0 for k in ("S", "D", "Sp", "Dp")}
    worst = {k: 0.0 for k in flat}
    for i in pairs:
        t, P = int(owner[i]), int(tg["near_patch"][i])
        W, scale = blocks[i]
        xyz, nrm, wt, _ = patch_arrays(surf, P)
        keep = np.ones(len(wt), dtype=bool)
        if int(tg["self_patch"][t]) == P:
            keep[int(tg["self_node"][t])] = False
        sm = smooth_kernels(tg["xyz"][:, t], tg["nrm"][:, t], xyz[keep], nrm[keep], wt[keep])
        raw = {}
        for k in flat:
            raw[k] = W[k].copy()
            raw[k][keep] += sm[k]
        f = dens[surf["node_off"][P]:surf["node_off"][P + 1]]
        _, sp = block_scales(raw, f, scale)
        for k in flat:
            e = abs((gpu[i][k] - W[k]) @ f) / sp[k]
            worst[k] = max(worst[k], e)
            flat[k] += e <= TOL
    acc = {k: dict(gate[k], potential_flat_all_sampled=flat[k] / len(pairs),
                   potential_max_all_sampled=worst[k]) for k in gate}
    exact = exact_reference(name, surf, tg, gpu_block)
    if exact is not None:
        acc["exact_far_pairs"] = exact
    allc.update(single_core=single, sphere_full=cfg1, nproc=os.cpu_count(), cpu_model=cpu_model(),
                gpu_vs_oracle_on_sample=acc)
    return allc


PHASES = ["targets", "roots_and_target_harmonics", "effective_weights", "contraction",
          "translation", "rows_x_maps_and_stores", "tile_fetch"]


def phase_split(args, reps=3):
    """Shares of the tile kernel's phases: the profiling build reads the shader clock at the
    workgroup barriers between phases (thread 0 of each workgroup) and sums the differences
    per phase over all workgroups.  The shares are of workgroup time, so a phase whose waves
    wait for other workgroups' work on the same compute unit is charged that wait."""
    import ctypes
    import torch
    from paper_2411_08342_amd import rrq
    from paper_2411_08342_amd.build import LIB_PHASES
    if not os.path.exists(LIB_PHASES):
        raise SystemExit(f"profiling build missing: {LIB_PHASES} (run __graft_entry__.build())")
    rrq.LIB_PATH = LIB_PHASES
    L = rrq.lib()
    surf, tg, desc = build_workload(args.workload)
    plan = rrq.Plan(rrq.DeviceSurface(surf), tile_targets=args.tile)
    asm = rrq.Assembler(plan, rrq.DeviceTargets(tg))
    flags = rrq.RRQ_F_CORRECTION | rrq.RRQ_F_ONSURF_PV
    tune = rrq.autotune(asm, flags)
    asm.assemble(flags=flags)
    torch.cuda.synchronize()
    if L.rrq_phase_reset() != 0:
        raise SystemExit("rrq_phase_reset failed")
    ks = [asm.assemble(flags=flags, stats=True)["kernel_ms"] for _ in range(reps)]
    torch.cuda.synchronize()
    h = (ctypes.c_ulonglong * 8)()
    if L.rrq_phase_read(h) != 0:
        raise SystemExit("rrq_phase_read failed")
    tot = float(sum(h[i] for i in range(len(PHASES))))
    print(json.dumps({"phase_split": {PHASES[i]: h[i] / tot for i in range(len(PHASES))},
                      "workgroup_cycles": {PHASES[i]: int(h[i]) for i in range(len(PHASES))},
                      "kernel_ms": float(np.mean(ks)), "assemblies": reps,
                      "tile_targets": tune["tile_targets"], "grid": tune["grid"],
                      "config": {"workload": desc}}))


def copy_probe(nbytes=1 << 30, reps=3):
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                      "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="star")
    ap.add_argument("--form", default="batched", choices=["plain", "batched"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="seconds of oracle work per core in the CPU baseline legs")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle worker processes (0: min(16, cores))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the plain-form and learned-guess measurements")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the mixed-order ellipsoids and the forty-sphere workloads")
    ap.add_argument("--phase-split", action="store_true",
                    help="only time the tile kernel's phases with the profiling build "
                         "(librrq_phases.so) and print their shares")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "known-size reference for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.phase_split:
        phase_split(args)
        return

    pool = None
    workers = args.cpu_workers or min(16, os.cpu_count() or 1)
    if not args.no_cpu_baseline:
        # before anything initialises the GPU: the workers are plain CPU processes
        pool, workers = start_cpu_pool(args.workload, workers)
        print(f"[bench] {workers} oracle workers ready", flush=True)

    import torch
    from paper_2411_08342_amd import rrq

    surf, tg, desc = build_workload(args.workload)
    print(f"[bench] workload ready: {surf['npatch']} patches, {tg['ntarget']} targets, "
          f"{len(tg['near_patch'])} pairs", flush=True)
    ds = rrq.DeviceSurface(surf)
    dt = rrq.DeviceTargets(tg)
    plan = rrq.Plan(ds, tile_targets=args.tile)
    asm = rrq.Assembler(plan, dt)
    flags = rrq.RRQ_F_CORRECTION | rrq.RRQ_F_ONSURF_PV
    if args.form == "plain":
        flags |= rrq.RRQ_F_PLAIN
    nweights = 4 * asm.nweights
    tune = None
    if args.form == "batched":
        tune = rrq.autotune(asm, flags)
        print(f"[bench] autotune: {tune}", flush=True)
    graph = rrq.Graph(asm, flags)       # refit + pair offsets + assembly, one HIP graph

    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        graph.launch()
        print(f"[bench] step {k + 1}/{args.steps} queued", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = nweights / (ms_per_step / 1e3)
    # duration of the dominant kernel (the pair kernel of the assembly), from HIP events the
    # library records around it on the stream it runs on
    runs = [asm.assemble(flags=flags, stats=True) for _ in range(args.steps)]
    stats = runs[-1]
    kern_ms = float(np.mean([r["kernel_ms"] for r in runs]))
    asm_ms = assemble_ms(asm, flags, args.steps)
    w_ref = {k: asm.out[k].clone() for k in rrq.KERNELS}
    forms = {args.form + "_assemble_ms": asm_ms, args.form + "_kernel_ms": kern_ms,
             args.form + "_newton_iters": stats["newton_iters"]}
    if not args.no_forms and args.form == "batched":
        pr = [asm.assemble(flags=flags | rrq.RRQ_F_PLAIN, stats=True) for _ in range(2)]
        forms["plain_kernel_ms"] = float(np.mean([r["kernel_ms"] for r in pr]))
        forms["plain_assemble_ms"] = assemble_ms(asm, flags | rrq.RRQ_F_PLAIN, 2)
        forms["plain_max_rel_weight_dev_vs_batched"] = max(
            ((asm.out[k] - w_ref[k]).abs().max() / w_ref[k].abs().max()).item() for k in rrq.KERNELS)
        forms["learned_star_torus"] = learned_form(rrq)
        forms["potentials"] = potentials_form(rrq, asm, flags, w_ref)
        print(f"[bench] forms: {forms}", flush=True)
        asm.assemble(flags=flags)      # leave the batched weights in the outputs

    q = int(surf["order"][0])
    alg_tflop = len(tg["near_patch"]) * flops_per_pair(q) / 1e12
    achieved = alg_tflop / (kern_ms / 1e3)
    tr = TRAFFIC if TRAFFIC["src_sha256"] == kernel_src_sha() else None
    traffic, traffic_detail = None, None
    if tr is not None and args.form == "batched" and tune and tune["tile_targets"] == 4:
        traffic = tr["fetch_bytes"] + tr["write_bytes"]
        traffic_detail = {"fetch_bytes": tr["fetch_bytes"], "write_bytes": tr["write_bytes"],
                          "GB_per_s": traffic / (kern_ms / 1e3) / 1e9,
                          "algorithmic_write_bytes": 8 * int(nweights)}
    out = {
        "metric": METRIC, "value": value, "unit": "weights/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "form": args.form, "graph": True, "autotune": tune,
                   "pairs": int(len(tg["near_patch"])),
                   "weights_per_step": int(nweights), "kernel_ms": kern_ms,
                   "assemble_ms": asm_ms,
                   "newton_iters_per_near_edge": stats["newton_iters"] / max(1, stats["near_edges"]),
                   "near_edges": stats["near_edges"], "newton_fail": stats["newton_fail"],
                   "newton_wave_iters": stats["newton_wave_iters"],
                   "panel_overflow": stats["panel_overflow"], "nonfinite": stats["nonfinite"],
                   "flagged_pairs": stats["flagged_pairs"],
                   "forms": forms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK, "traffic": traffic,
                     "traffic_detail": traffic_detail,
                     "kernel": (f"k_pair_plain<{q}>" if args.form == "plain"
                                else f"k_pair_tile<{q},{tune['tile_targets'] if tune else 'T'}>"),
                     "flops_per_pair": flops_per_pair(q)},
    }
    if not args.no_other_workloads:
        out["other_workloads"] = {}
        for name in ("ellipsoids", "forty_spheres"):
            out["other_workloads"][name] = other_workload(rrq, name)
            print(f"[bench] {name}: {out['other_workloads'][name]}", flush=True)
    if pool is not None:
        off = asm.pair_off.cpu().numpy()

        def gpu_block(i):
            return {k: asm.out[k][off[i]:off[i + 1]].cpu().numpy() for k in rrq.KERNELS}

        out["cpu_baseline"] = cpu_baseline(pool, workers, args.workload, surf, tg, gpu_block,
                                           args.cpu_seconds)
        pool.shutdown()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
