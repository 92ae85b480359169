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
TRAFFIC = {"src_sha256": "8f8d22ce8d25613e2c644f860e889d97d3a18b2611ea5fd8a5808eca016e09d0",
           "fetch_bytes": 1785462638, "write_bytes": 3601301248}


def flops_per_pair(q):
    """Algorithmic FP64 flops of one (target, patch) pair at order q (ptilde = 2q), counting
    only data-independent work (Newton iterations and panel points excluded):
      edge contractions  4 ptilde (16 J1 + 76 J2)      V: 16, Q and dQ: 38 each per (j,k,node)
      edge weights/Omega 4 ptilde * 60
      translations       100 tD + 10 tS                  terms of the DLP/SLP sums
      target harmonics   60 (q+1)^2
      weight contraction 2 q^2 17 n_p                    rows x maps
    """
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
    return (4 * pt * (16 * J1 + 76 * J2) + 4 * pt * 60 + 100 * tD + 10 * tS
            + 60 * (p + 1) ** 2 + 2 * q * q * 17 * n_p)


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


def learned_form(rrq, asm, flags, w_ref, reps=2):
    """Train the learned Newton guess on its own seeded geometry (not the benchmark surface),
    then time the batched form with it.  Returns a summary dict."""
    import torch
    from paper_2411_08342_amd import workloads as wl
    t0 = time.perf_counter()
    surf, tg, _ = wl.learned_guess_training()
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    feat, dt, _ = rrq.collect_roots(plan, rrq.DeviceTargets(tg), 4 * len(tg["near_patch"]))
    plan.close()
    params, curve = rrq.mlp_train(feat, dt, steps=4000, batch=8192, lr=3e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    asm.plan.set_mlp(params)
    lf = flags | rrq.RRQ_F_LEARNED
    st = [asm.assemble(flags=lf, stats=True) for _ in range(reps)]
    a_ms = assemble_ms(asm, lf, reps)
    dev = max(((asm.out[k] - w_ref[k]).abs().max() / w_ref[k].abs().max()).item()
              for k in rrq.KERNELS)
    asm.plan.set_mlp(None)
    c = curve.cpu().numpy()
    return {"assemble_ms": a_ms, "kernel_ms": float(np.mean([x["kernel_ms"] for x in st])),
            "newton_iters": st[-1]["newton_iters"], "learned_accept": st[-1]["learned_accept"],
            "max_rel_weight_dev_vs_batched": dev, "train_samples": int(feat.shape[1]),
            "train_s": t_train, "train_loss_first_last": [float(c[:10].mean()), float(c[-100:].mean())]}


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
        surf, tg, dens = wl.config2()
        desc = ("star r=1+0.2ReY43+0.1ReY21, 1536 quads q=8, 98304 node targets, "
                "near 1.5 patch diameters")
    elif name == "star-small":
        surf, tg, dens = wl.config2(n=4)
        desc = "star, 96 quads q=8, node targets, near 1.5 patch diameters"
    else:
        raise SystemExit(f"unknown workload {name}")
    return surf, tg, desc


def cpu_baseline(surf, tg, seconds=20.0, seed=0):
    """The oracle, as it stands, on all near pairs of seeded targets (fits of the touched
    patches included), one thread, until about `seconds` of work."""
    from threadpoolctl import threadpool_limits
    from oracle.assemble import pair_block
    rng = np.random.default_rng(seed)
    T = len(tg["near_ptr"]) - 1
    order = rng.permutation(T)
    fits = {}
    nw = 0
    npairs = 0
    ntg = 0
    results = {}
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for t in order:
            for i in range(tg["near_ptr"][t], tg["near_ptr"][t + 1]):
                P = int(tg["near_patch"][i])
                W, _ = pair_block(surf, tg, fits, int(t), P)
                results[int(i)] = W
                nw += 4 * len(W["S"])
                npairs += 1
            ntg += 1
            if time.perf_counter() - t0 > seconds:
                break
        dt = time.perf_counter() - t0
    return dict(value=nw / dt, unit="weights/s", cores=1, kind="oracle",
                sample=f"all {npairs} near pairs of {ntg} seeded targets "
                       f"({len(fits)} patch fits included), {dt:.1f} s"), results


def parity_gate(surf, tg, res, gpu_blocks, owner, max_pairs=150, tol=1e-11, ulp_factor=30.0):
    """On the sampled pair blocks (the first max_pairs): the fraction that passes the weights
    gate of the parity tests, ||W_gpu - W_or|| <= tol ||W_raw|| + ulp_factor ||dW_ulp||, dW_ulp
    the largest change of the oracle block under rounding-level perturbations (target moved by
    one relative ulp, edge samples by one ulp, fits solved by SVD instead of QR); and, over
    the same blocks, the max-norm difference GPU - oracle and oracle(SVD) - oracle(QR), both
    relative to the largest oracle weight."""
    from oracle.assemble import pair_block
    KERNELS = ("S", "D", "Sp", "Dp")
    fits, fits_svd = {}, {}
    ok = {k: 0 for k in KERNELS}
    dg = {k: 0.0 for k in KERNELS}
    ds = {k: 0.0 for k in KERNELS}
    wm = {k: 0.0 for k in KERNELS}
    pairs = sorted(res)[:max_pairs]
    for i in pairs:
        t, P = int(owner[i]), int(tg["near_patch"][i])
        W = res[i]
        raw, _ = pair_block(surf, tg, fits, t, P, False)
        svd = pair_block(surf, tg, fits_svd, t, P, True, True, "svd")[0]
        for k in KERNELS:
            dg[k] = max(dg[k], float(np.max(np.abs(gpu_blocks[i][k] - W[k]))))
            ds[k] = max(ds[k], float(np.max(np.abs(svd[k] - W[k]))))
            wm[k] = max(wm[k], float(np.max(np.abs(W[k]))))
        need = [k for k in KERNELS
                if np.max(np.abs(gpu_blocks[i][k] - W[k])) > tol * np.max(np.abs(raw[k]))]
        for k in KERNELS:
            ok[k] += k not in need
        if not need:
            continue
        tg2 = dict(tg)
        x = np.array(tg["xyz"], copy=True)
        x[:, t] *= 1.0 + 2.0 ** -52
        tg2["xyz"] = x
        s2 = dict(surf)
        e = np.array(surf["edge_xyz"], copy=True)
        sg = np.random.default_rng(i).choice([-1.0, 1.0], size=e.shape)
        s2["edge_xyz"] = e * (1.0 + 2.0 ** -52 * sg)
        pert = (pair_block(surf, tg2, fits, t, P)[0], svd, pair_block(s2, tg, {}, t, P)[0])
        for k in need:
            dw = max(np.max(np.abs(pp[k] - W[k])) for pp in pert)
            ok[k] += np.max(np.abs(gpu_blocks[i][k] - W[k])) <= (tol * np.max(np.abs(raw[k]))
                                                                + ulp_factor * dw)
    return {k: {"pairs_within_parity_gate": ok[k] / len(pairs),
                "global_maxnorm_rel_gpu_vs_oracle": dg[k] / wm[k],
                "global_maxnorm_rel_oracle_svd_vs_qr": ds[k] / wm[k]} for k in KERNELS}


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
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the plain-form and learned-guess measurements")
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
        forms["learned"] = learned_form(rrq, asm, flags, w_ref)
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
                   "forms": forms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK, "traffic": traffic,
                     "traffic_detail": traffic_detail,
                     "kernel": (f"k_pair_plain<{q}>" if args.form == "plain"
                                else f"k_pair_tile<{q},{tune['tile_targets'] if tune else 'T'}>"),
                     "flops_per_pair": flops_per_pair(q)},
    }
    if not args.no_cpu_baseline:
        cb, res = cpu_baseline(surf, tg, args.cpu_seconds)
        off = asm.pair_off.cpu().numpy()
        x, y, z = surf["node_xyz"]
        dens = 0.7 + x * x - 0.4 * y * z + 0.3 * z + 0.2 * x * y * z   # smooth nodal density
        # scale of each block: the oracle block without the smooth-rule subtraction (the
        # corrected weights of far pairs are small differences of large numbers)
        from oracle.assemble import patch_arrays
        from oracle.rrq import smooth_kernels
        owner = np.repeat(np.arange(len(tg["near_ptr"]) - 1), np.diff(tg["near_ptr"]))
        raw = {}
        for i, W in res.items():
            t, P = int(owner[i]), int(tg["near_patch"][i])
            xyz, nrm, wt, _ = patch_arrays(surf, P)
            sm = smooth_kernels(tg["xyz"][:, t], tg["nrm"][:, t], xyz, nrm, wt)
            if int(tg["self_patch"][t]) == P:
                for k in rrq.KERNELS:
                    sm[k][int(tg["self_node"][t])] = 0.0
            raw[i] = {k: W[k] + sm[k] for k in rrq.KERNELS}
        gpu_blocks = {i: {k: asm.out[k][off[i]:off[i + 1]].cpu().numpy() for k in rrq.KERNELS}
                      for i in res}
        gate = parity_gate(surf, tg, res, gpu_blocks, owner, max_pairs=150)
        acc = {}
        for k in rrq.KERNELS:
            wrel = pot = 0.0
            within = 0
            for i, W in res.items():
                g = gpu_blocks[i][k]
                P = int(tg["near_patch"][i])
                f = dens[surf["node_off"][P]:surf["node_off"][P + 1]]
                d = np.max(np.abs(g - W[k]))
                sc = np.max(np.abs(raw[i][k]))
                wrel = max(wrel, d / sc)
                within += d <= 1e-11 * sc
                pot = max(pot, abs((g - W[k]) @ f) / np.sum(np.abs(raw[i][k] * f)))
            acc[k] = {"weights_max_rel_to_raw_block": wrel,
                      "pairs_within_1e-11_of_raw_block": within / len(res),
                      "potential_max_rel_to_raw_block": pot}
            acc[k].update(gate[k])
        cb["gpu_vs_oracle_on_sample"] = acc
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
