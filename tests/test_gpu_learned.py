"""GPU tests of the learned Newton guess: training samples, network kernels and gradient
against the oracle, reproducible training, and what the trained network gains over plain
Newton without changing the weights."""
import numpy as np
import pytest

from paper_2411_08342_amd import workloads as wl

pytestmark = pytest.mark.gpu

KERNELS = ("S", "D", "Sp", "Dp")


def _oracle_samples(surf, tg):
    """Oracle: features, chord start and plain Newton root for every (pair, edge) in pair
    order, kept when both the chord start and the converged root lie inside the Bernstein
    ellipse of radius rho_far (the edges the singularity swap integrates)."""
    from oracle import mlp
    from oracle.assemble import patch_arrays
    from oracle.fit import Frame, edge_coefficients
    from oracle.ssq import bernstein_radius, newton_root, rho_far
    owner = np.repeat(np.arange(len(tg["near_ptr"]) - 1), np.diff(tg["near_ptr"]))
    frames = {}
    feats, dts, t0s = [], [], []
    for k in range(len(tg["near_patch"])):
        P = int(tg["near_patch"][k])
        if P not in frames:
            xyz, nrm, wt, edges = patch_arrays(surf, P)
            fr = Frame(edges, nrm)
            frames[P] = (fr, [edge_coefficients(fr.point(edges[e])) for e in range(4)])
        fr, coefs = frames[P]
        x = fr.point(tg["xyz"][:, owner[k]])
        rf = rho_far(2 * int(surf["order"][P]))
        for e in range(4):
            f, ts = mlp.edge_features(coefs[e], x)
            if bernstein_radius(ts) > rf:
                continue
            t0, _, conv = newton_root(coefs[e], x, ts)
            if conv and bernstein_radius(t0) <= rf:
                feats.append(f)
                dts.append([t0.real - ts.real, t0.imag - ts.imag])
                t0s.append([t0.real, t0.imag])
    return np.array(feats).T, np.array(dts).T, np.array(t0s).T


def test_collected_samples_match_oracle():
    import torch
    from paper_2411_08342_amd import rrq
    surf, tg, _ = wl.sphere_q6()
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    dtg = rrq.DeviceTargets(tg)
    feat, dt, t0 = rrq.collect_roots(plan, dtg, 4 * len(tg["near_patch"]))
    torch.cuda.synchronize()
    of, odt, ot0 = _oracle_samples(surf, tg)
    print(f"samples: gpu {feat.shape[1]}, oracle {of.shape[1]}", flush=True)
    assert feat.shape[1] == of.shape[1] > 100
    g = feat.cpu().numpy().astype(np.float64)
    # features are computed in double and rounded to float on both sides
    assert np.max(np.abs(g - of.astype(np.float32))) <= 2e-6 * max(1.0, np.max(np.abs(of)))
    # Conditioning of the root: the two sides build the local edge (Legendre coefficients) and
    # target with different rounding.  A coefficient change of eps moves r(t0) by about
    # eps rho(t0)^(ptilde-1) (|P_k(t)| <= rho(t)^k off [-1, 1]) and t0 by as much over |r'|;
    # a change of the distance function by eps moves t0 by about eps / Im t0 (t0 and its
    # conjugate merge as Im t0 -> 0).  Gate: 8 ulp of each.
    from oracle.ssq import bernstein_radius
    owner_q = 6
    rho = np.array([bernstein_radius(complex(a, b)) for a, b in ot0.T])
    eps = 2.0 ** -52
    cond = 8 * eps * (rho ** (2 * owner_q - 1) + 1.0 / ot0[1])
    e_t0 = np.max(np.abs(t0.cpu().numpy() - ot0), axis=0)
    worst = np.argsort(e_t0 / (1e-12 + cond))[-3:]
    for i in worst:
        print(f"t0 {ot0[:, i]} rho {rho[i]:.3f}: diff {e_t0[i]:.2e}, allowance {1e-12 + cond[i]:.2e}")
    assert np.all(e_t0 <= 1e-12 + cond)
    e_dt = np.max(np.abs(dt.cpu().numpy() - odt.astype(np.float32)), axis=0)
    assert np.all(e_dt <= 1e-6 * np.maximum(1.0, np.max(np.abs(odt), axis=0)) + cond)
    # capacity is respected and a prefix is returned
    f2, d2, _ = rrq.collect_roots(plan, dtg, 50)
    assert f2.shape[1] == 50 and torch.equal(f2, feat[:, :50])
    plan.close()


def _rand_params(rng, scale=0.3):
    from oracle import mlp
    return rng.normal(scale=scale, size=mlp.N_PARAMS).astype(np.float32)


def test_mlp_forward_and_gradient_match_oracle():
    """Network outputs and the gradient of the loss from the HIP kernels (float32) against
    the oracle (float64 on the same float32 numbers)."""
    import torch
    from oracle import mlp
    from paper_2411_08342_amd import rrq
    rng = np.random.default_rng(3)
    for n in (1, 257, 3000):
        p = _rand_params(rng)
        X = rng.normal(size=(n, 8)).astype(np.float32)
        Yt = rng.normal(scale=0.5, size=(n, 2)).astype(np.float32)
        pt = torch.tensor(p, device="cuda")
        ft = torch.tensor(X.T.copy(), device="cuda")
        yt = torch.tensor(Yt.T.copy(), device="cuda")
        out = rrq.mlp_predict(pt, ft).cpu().numpy().T
        _, _, Yo = mlp.forward(p.astype(np.float64), X.astype(np.float64))
        assert np.max(np.abs(out - Yo)) <= 2e-5 * max(1.0, np.max(np.abs(Yo)))
        loss, grad = rrq.mlp_loss_grad(pt, ft, yt)
        L, g = mlp.loss_grad(p.astype(np.float64), X.astype(np.float64), Yt.astype(np.float64))
        gg = grad.cpu().numpy().astype(np.float64)
        err = np.max(np.abs(gg - g)) / np.max(np.abs(g))
        print(f"n={n}: loss {loss.item():.6e} vs {L:.6e}; grad max-norm rel err {err:.2e}")
        assert abs(loss.item() - L) <= 1e-5 * L
        assert err <= 1e-5


def _train_samples(small=True):
    import torch
    from paper_2411_08342_amd import rrq
    kw = dict(n=4, nt=8, nphi=16, per_patch=6) if small else {}
    surf, tg, _ = wl.learned_guess_training(**kw)
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    feat, dt, _ = rrq.collect_roots(plan, rrq.DeviceTargets(tg), 4 * len(tg["near_patch"]))
    torch.cuda.synchronize()
    plan.close()
    return feat, dt


def test_training_reduces_loss_and_is_reproducible():
    import torch
    from paper_2411_08342_amd import rrq
    feat, dt = _train_samples()
    print(f"training samples: {feat.shape[1]}", flush=True)
    p1, c1 = rrq.mlp_train(feat, dt, steps=600, batch=2048, lr=3e-3, seed=9)
    p2, c2 = rrq.mlp_train(feat, dt, steps=600, batch=2048, lr=3e-3, seed=9)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(c1, c2)
    c = c1.cpu().numpy()
    print(f"loss: first {c[:10].mean():.4e}, last {c[-50:].mean():.4e}")
    assert np.all(np.isfinite(c)) and c[-50:].mean() < 0.2 * c[:10].mean()
    p3, _ = rrq.mlp_train(feat, dt, steps=10, batch=64, lr=3e-3, seed=10)
    assert not torch.equal(p1[:512], p3[:512])


def test_learned_guess_gains_iterations_and_keeps_weights():
    """Trained on the training geometry, evaluated on the star surface: fewer Newton
    iterations, the learned start accepted on most near edges, the same near/far split, and
    weights equal to the plain-Newton ones to rounding."""
    import torch
    from paper_2411_08342_amd import rrq
    feat, dt = _train_samples(small=False)
    params, _ = rrq.mlp_train(feat, dt, steps=4000, batch=8192, lr=3e-3, seed=1)
    surf, tg, _ = wl.star(n=6)
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    asm = rrq.Assembler(plan, rrq.DeviceTargets(tg))
    flags = rrq.RRQ_F_CORRECTION | rrq.RRQ_F_ONSURF_PV
    with pytest.raises(rrq.RRQError):
        asm.assemble(flags=flags | rrq.RRQ_F_LEARNED)          # no network installed
    s0 = asm.assemble(flags=flags, stats=True)
    w0 = {k: asm.out[k].clone() for k in KERNELS}
    plan.set_mlp(params)
    s1 = asm.assemble(flags=flags | rrq.RRQ_F_LEARNED, stats=True)
    torch.cuda.synchronize()
    print(f"plain: {s0}\nlearned: {s1}")
    assert s1["near_edges"] == s0["near_edges"] > 0
    assert s1["learned_accept"] >= 0.99 * s1["near_edges"]
    assert s1["newton_iters"] <= 0.95 * s0["newton_iters"]
    assert s1["newton_wave_iters"] < s0["newton_wave_iters"]
    # both solves stop at a step below 1e-14 |t0|, so the roots agree to rounding; the
    # weights then agree within the parity target (1e-11 of the largest weight)
    for k in KERNELS:
        d = (asm.out[k] - w0[k]).abs().max().item()
        sc = w0[k].abs().max().item()
        print(f"{k}: max |learned - plain| = {d:.3e} (max |w| {sc:.3e})")
        assert d <= 1e-11 * sc
    with pytest.raises(rrq.RRQError):
        asm.assemble(flags=flags | rrq.RRQ_F_LEARNED | rrq.RRQ_F_PLAIN)
    plan.set_mlp(None)
    plan.close()


def test_learned_guess_star_torus():
    """The learned start on the star surface plus the 2048-patch torus, trained on about 2M
    samples of the separately seeded training geometry: the same near edges, the learned
    start accepted on nearly all of them, fewer Newton iterations in total and per
    wavefront, and weights equal to the plain-Newton ones within the parity target."""
    import torch
    from paper_2411_08342_amd import rrq
    surf, tg, _ = wl.learned_guess_training(per_patch=110)
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    feat, dt, _ = rrq.collect_roots(plan, rrq.DeviceTargets(tg), 4 * len(tg["near_patch"]))
    plan.close()
    print(f"training samples: {feat.shape[1]}", flush=True)
    assert feat.shape[1] >= 1_900_000
    params, _ = rrq.mlp_train(feat, dt, steps=4000, batch=8192, lr=3e-3, seed=1)
    del feat, dt
    surf, tg, _ = wl.star_torus()
    plan = rrq.Plan(rrq.DeviceSurface(surf))
    asm = rrq.Assembler(plan, rrq.DeviceTargets(tg))
    flags = rrq.RRQ_F_CORRECTION | rrq.RRQ_F_ONSURF_PV
    s0 = asm.assemble(flags=flags, stats=True)
    w0 = {k: asm.out[k].clone() for k in KERNELS}
    plan.set_mlp(params)
    s1 = asm.assemble(flags=flags | rrq.RRQ_F_LEARNED, stats=True)
    torch.cuda.synchronize()
    print(f"plain: {s0}\nlearned: {s1}")
    assert s1["near_edges"] == s0["near_edges"] > 0
    assert s1["newton_slots"] == s0["newton_slots"]
    assert s1["learned_accept"] >= 0.99 * s1["near_edges"]
    assert s1["newton_iters"] < s0["newton_iters"]
    assert s1["newton_wave_iters"] < s0["newton_wave_iters"]
    for k in KERNELS:
        d = (asm.out[k] - w0[k]).abs().max().item()
        sc = w0[k].abs().max().item()
        print(f"{k}: max |learned - plain| = {d:.3e} (max |w| {sc:.3e})")
        assert d <= 1e-11 * sc
    plan.set_mlp(None)
