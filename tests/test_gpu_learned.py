"""Learned coarse correction on the GPU: feature rows, forward pass and
gradients against the FP64 oracle (BF16 MFMA products, FP32 accumulation;
errors stated), then harvest -> train -> use inside FGMRES on a held-out
state, and the fallback to plain pMG when the network is useless."""
import numpy as np
import pytest

from oracle import mlp
from paper_2202_09733_amd import capi
from paper_2202_09733_amd import workloads as W
from gpu_util import announce, rel, require_gpu

pytestmark = pytest.mark.gpu


def _fr(n=(8, 8), seed=2):
    wl = W.make_vortical_workload(n=n, seed=seed, dt_factor=1000.0)
    return wl, capi.FR.from_workload(wl)


def test_feature_rows_parity(orc):
    require_gpu()
    announce("lcc feature rows")
    for wl, fr in [_fr(), (lambda w: (w, capi.FR.from_workload(w)))(W.make_tgv_workload(n=(4, 2, 4)))]:
        d = fr.lcc_dims()
        rng = np.random.default_rng(1)
        in_scale = rng.uniform(0.5, 2.0, wl.nv).astype(np.float32)
        fr.lcc_set_scales(in_scale, np.ones(wl.nv, dtype=np.float32))
        d1 = rng.standard_normal(fr.shape(1))
        rows, s = fr.lcc_features_of(fr.to_dev(d1))
        rows_ref, s_ref = mlp.features(d1, wl.dim, wl.n, wl.p1 + 1, in_scale.astype(np.float64), d["nin_pad"], wl.h)
        assert rel(s, s_ref) <= 1e-6
        assert rel(rows, rows_ref) <= 1e-6


def test_forward_parity(orc):
    """BF16-input MFMA products with FP32 accumulation against the oracle's
    forward pass with the same BF16 operands (inputs, weights and hidden
    activations rounded where the GPU stores them): only the accumulation
    order differs.  The error against the plain FP64 network is stated."""
    require_gpu()
    announce("lcc forward")
    wl, fr = _fr()
    d = fr.lcc_dims()
    Ws = [w.astype(np.float64) for w in fr.lcc_get_weights()]
    rng = np.random.default_rng(2)
    X = np.zeros((128, d["nin_pad"]))
    X[:, :d["nin"]] = rng.standard_normal((128, d["nin"]))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Y = fr.lcc_forward(X)
    e_emul = rel(Y, mlp.forward(Ws, X, bf16=True)[0])
    e_fp64 = rel(Y, mlp.forward(Ws, X)[0])
    print("forward: vs BF16-emulating FP64 %.2e, vs plain FP64 %.2e" % (e_emul, e_fp64))
    assert e_emul <= 1e-5 and e_fp64 <= 3e-2


def test_gradient_parity(orc):
    """Loss and gradient of a batch against the oracle's chain rule with the
    GPU's BF16 operands (inputs, weights, activations, output and hidden
    gradients); relative error and cosine similarity stated."""
    require_gpu()
    announce("lcc loss/gradient")
    wl, fr = _fr()
    d = fr.lcc_dims()
    Ws = [w.astype(np.float64) for w in fr.lcc_get_weights()]
    rng = np.random.default_rng(3)
    B = 256
    X = np.zeros((B, d["nin_pad"]))
    X[:, :d["nin"]] = rng.standard_normal((B, d["nin"]))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    T = np.zeros((B, d["nout_pad"]))
    T[:, :d["nout"]] = 0.1 * rng.standard_normal((B, d["nout"]))
    loss, g = fr.lcc_loss_grad(X, T)
    loss_ref, g_ref = mlp.loss_grad(Ws, X, T, d["nout"], bf16=True)
    _, g64 = mlp.loss_grad(Ws, X, T, d["nout"])
    print("loss %.9e vs %.9e" % (loss, loss_ref))
    assert abs(loss - loss_ref) <= 1e-6 * loss_ref
    for l in range(3):
        e = rel(g[l], g_ref[l])
        cos = float(np.sum(g[l] * g_ref[l]) / (np.linalg.norm(g[l]) * np.linalg.norm(g_ref[l])))
        print("layer %d gradient: rel err %.2e (vs plain FP64 %.2e), cosine %.8f" % (l + 1, e, rel(g[l], g64[l]), cos))
        assert e <= 1e-4 and cos >= 0.9999999


def test_adam_step_parity(orc):
    """Three Adam steps of the master weights with seeded gradients against
    the oracle's FP64 Adam: the weight changes agree to FP32 rounding."""
    require_gpu()
    announce("lcc adam step")
    wl, fr = _fr()
    rng = np.random.default_rng(4)
    W0 = [(0.05 * rng.standard_normal(w.shape)).astype(np.float32) for w in fr.lcc_get_weights()]
    fr.lcc_set_weights(W0)
    W = [w.astype(np.float64) for w in W0]
    M = [np.zeros_like(w) for w in W]
    V = [np.zeros_like(w) for w in W]
    for t in range(1, 4):
        G = [(rng.standard_normal(w.shape) * 10.0 ** rng.uniform(-4, 0, w.shape)).astype(np.float32) for w in W0]
        fr.lcc_adam_step(G, 2e-3)
        for l in range(3):
            W[l], M[l], V[l] = mlp.adam_step(W[l], G[l].astype(np.float64), M[l], V[l], t, 2e-3)
    Wg = fr.lcc_get_weights()
    for l in range(3):
        e = rel(Wg[l].astype(np.float64) - W0[l], W[l] - W0[l])
        print("layer %d: weight change rel err %.2e" % (l + 1, e))
        assert e <= 1e-5


def _seeded_network(fr, rng):
    d = fr.lcc_dims()
    nh, nin, nout = d["nh"], d["nin"], d["nout"]
    W1 = np.zeros((nh, d["nin_pad"]))
    W1[:, :nin] = rng.standard_normal((nh, nin)) * np.sqrt(2.0 / nin)
    W2 = rng.standard_normal((nh, nh)) * np.sqrt(2.0 / nh)
    W3 = np.zeros((d["nout_pad"], nh))
    W3[:nout] = rng.standard_normal((nout, nh)) * np.sqrt(2.0 / nh)
    return [w.astype(np.float32) for w in (W1, W2, W3)], d


@pytest.mark.parametrize("case", ["vortical_8x8_p42", "tgv_4cubed_p32"])
def test_learned_vcycle_matches_oracle(orc, case):
    """pmg_precond_apply with the learned coarse correction (FR_COARSE_LEARNED)
    against the oracle's V-cycle with the same network (seeded host weights and
    scales, BF16 operands emulated): pre-smoothing, defect, restriction, C1 =
    B1^{-1} Gamma d, feature rows, both network evaluations, the odd/homogeneous
    output, prolongation and post-smoothing.  The two sides form their EJ
    blocks independently by finite differences (the plain V-cycle's agreement
    is printed beside it)."""
    require_gpu()
    announce("learned V-cycle vs oracle: " + case)
    if case == "vortical_8x8_p42":
        wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
        sigA = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
        sigS = 1.0 / wl.dt + sigA
    else:
        wl = W.make_tgv_workload(n=(4, 4, 4))
        sigA = 1.0 / (wl.a_ii * wl.dt)
        sigS = 1.0 / wl.dt + sigA
    fr = capi.FR.from_workload(wl)
    rng = np.random.default_rng(21)
    Ws32, d = _seeded_network(fr, rng)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    P0, P1 = wl.p0 + 1, wl.p1 + 1
    fac0 = orc.lu_factor(L0.ej_blocks(wl.dq, sigS))
    q1 = orc.restrict(wl.dq, wl.dim, P0, P1)
    fac1 = orc.lu_factor(L1.ej_blocks(q1, sigS))
    rq = L0.residual(wl.dq)
    X = rng.standard_normal(L0.shape)
    X /= np.linalg.norm(X)
    # input scales: the per-variable RMS of the oracle's C1 of this X; the
    # network contributes a fifth of the coarse step's size
    pm_plain = orc.PMG(L0, L1, fac0, fac1, orc.PMGParams(sigma_D=sigA))
    pm_plain.set_point(wl.dq, rq)
    Y_plain_ref = pm_plain.apply(X)
    C1_probe = orc.lu_solve(fac1, orc.restrict(X, wl.dim, P0, P1))
    in_scale = np.sqrt(np.mean(C1_probe ** 2, axis=(1, 2))).astype(np.float32)
    out_scale = (0.2 * in_scale).astype(np.float32)
    lc = mlp.LearnedCoarse([w.astype(np.float64) for w in Ws32], in_scale.astype(np.float64),
                           out_scale.astype(np.float64), wl.dim, wl.n, wl.h, P1, d["nin_pad"], bf16=True)
    pm = orc.PMG(L0, L1, fac0, fac1, orc.PMGParams(sigma_D=sigA, learned=lc))
    pm.set_point(wl.dq, rq)
    Y_ref = pm.apply(X)
    fr.lcc_set_weights(Ws32)
    fr.lcc_set_scales(in_scale, out_scale)
    d_q = fr.to_dev(wl.dq)
    fr.ej_factor(0, d_q, sigS)
    fr.ej_factor(1, fr.to_dev(q1), sigS)
    fr.pmg_set_point(d_q, fr.to_dev(rq))
    Y = fr.pmg_apply(fr.to_dev(X), sigA, coarse_mode=capi.COARSE_LEARNED).cpu().numpy()
    Yp = fr.pmg_apply(fr.to_dev(X), sigA, coarse_mode=capi.COARSE_EJ).cpu().numpy()
    e_l, e_p = rel(Y, Y_ref), rel(Yp, Y_plain_ref)
    print("%s: learned V-cycle vs oracle %.2e (plain V-cycle %.2e); learned vs plain %.3f"
          % (case, e_l, e_p, rel(Y_ref, Y_plain_ref)))
    assert rel(Y_ref, Y_plain_ref) > 1e-3      # the network changes the cycle
    # the GPU forms the feature rows in FP32 and the oracle in FP64 before
    # both round them to BF16: an entry near a rounding boundary can round
    # one BF16 step (2^-8 of itself) apart; measured 1.5e-7 (2D), 8.7e-6 (3D)
    assert e_l <= 3e-5


def test_harvest_capacity_change_keeps_pairs_and_trains(orc):
    """Harvest into a small buffer, train, re-enable harvesting with a larger
    capacity (the pairs so far are kept), harvest more and train again; then
    shrink the capacity below the count (the first pairs are kept)."""
    require_gpu()
    announce("lcc harvest capacity change")
    wl, fr = _fr(n=(16, 16))
    cfg = capi.stage_config_for(wl)
    dq = fr.to_dev(wl.dq)
    fr.lcc_harvest(enable=1, max_pairs=1024, stride=2, target_sweeps=2, reset=1)
    fr.solve_stage(cfg, dq)
    n1 = fr.lcc_count()
    assert n1 == 1024
    fr.lcc_train(epochs=1, batch=64, lr=1e-3, seed=1, holdout=0.1, reinit=1)
    fr.lcc_harvest(enable=1, max_pairs=8192, stride=2, target_sweeps=2, reset=0)
    assert fr.lcc_count() == n1
    fr.solve_stage(cfg, dq)
    n2 = fr.lcc_count()
    assert n2 > n1
    ts = fr.lcc_train(epochs=2, batch=64, lr=1e-3, seed=2, holdout=0.1, reinit=0)
    assert np.isfinite(ts["loss_last"]) and np.isfinite(ts["val_loss"])
    fr.lcc_harvest(enable=1, max_pairs=512, stride=2, target_sweeps=2, reset=0)
    assert fr.lcc_count() == 512
    ts = fr.lcc_train(epochs=1, batch=64, lr=1e-3, seed=3, holdout=0.1, reinit=0)
    assert np.isfinite(ts["loss_last"])
    fr.lcc_harvest(enable=0)


def _oracle_rel_F(orc, wl, q):
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    R0 = L0.residual(wl.dq)
    b = wl.dq + wl.a_ii * wl.dt * R0
    F = (q - b) / (wl.a_ii * wl.dt) - L0.residual(q)
    return np.linalg.norm(F) / np.linalg.norm(2 * R0)


def harvest_with_probes(fr, wl, nprobe, rng):
    """Harvest pairs from one plain-pMG stage of wl, then from nprobe V-cycles
    of the same preconditioner (set up at wl's state) on random directions,
    half of them white noise and half restricted-and-prolonged noise: the
    Krylov directions of a stage span a narrow set, and the network has to
    cover the directions it meets with its own preconditioner."""
    fr.solve_stage(capi.stage_config_for(wl), fr.to_dev(wl.dq))
    dq = fr.to_dev(wl.dq)
    sig_a = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    sig_s = 1.0 / wl.dt + sig_a
    fr.ej_factor(0, dq, sig_s)
    fr.ej_factor(1, fr.restrict(0, dq), sig_s)
    fr.pmg_set_point(dq, fr.residual(0, dq))
    for i in range(nprobe):
        x = fr.to_dev(rng.standard_normal(fr.shape(0)))
        if i % 2 == 1:
            x = fr.prolong(1, fr.restrict(0, x))
        fr.pmg_apply(x, sig_a)


def test_harvest_train_and_use_on_held_out_state(orc):
    """Harvest from plain-pMG stages and probe V-cycles on two random states,
    train, then solve the stage of a different (held-out) state with the
    learned coarse correction and the stall fallback switched off.  Gates:
    the network learns (validation loss falls), the learned preconditioner
    stays close to plain pMG on random directions, and the learned stage
    reaches 1e-8 in the oracle's own F on its own, within 1.2x plain pMG's
    FGMRES iterations, and within 1.1x with the stall fallback on.  Iteration
    counts and DOF/s of both preconditioners are printed (the A/B
    comparison)."""
    require_gpu()
    announce("lcc harvest/train/use, 64x64 vortical mesh")
    wl_eval = W.make_vortical_workload(seed=2)
    fr = capi.FR.from_workload(W.make_vortical_workload(seed=12))
    rng = np.random.default_rng(11)
    fr.lcc_harvest(enable=1, max_pairs=400000, stride=4, target_sweeps=2, reset=1)
    for seed in (12, 13):
        harvest_with_probes(fr, W.make_vortical_workload(seed=seed), 200, rng)
    fr.lcc_harvest(enable=0)
    n = fr.lcc_count()
    ts = fr.lcc_train(epochs=60, batch=256, lr=1e-3, seed=7, holdout=0.1, reinit=1)
    print("harvested %d pairs; training %s" % (n, ts))
    assert n >= 300000
    assert ts["val_loss"] < 1e-2 * ts["val_loss_init"]
    dq = fr.to_dev(wl_eval.dq)
    # the learned V-cycle against the plain one on random directions
    sig_a = 1.0 / wl_eval.dt + 1.0 / (wl_eval.a_ii * wl_eval.dt)
    sig_s = 1.0 / wl_eval.dt + sig_a
    fr.ej_factor(0, dq, sig_s)
    fr.ej_factor(1, fr.restrict(0, dq), sig_s)
    fr.pmg_set_point(dq, fr.residual(0, dq))
    for kind in ("noise", "smooth"):
        x = fr.to_dev(rng.standard_normal(fr.shape(0)))
        if kind == "smooth":
            x = fr.prolong(1, fr.restrict(0, x))
        yp = fr.pmg_apply(x, sig_a, coarse_mode=capi.COARSE_EJ).cpu().numpy()
        yl = fr.pmg_apply(x, sig_a, coarse_mode=capi.COARSE_LEARNED).cpu().numpy()
        yn = fr.pmg_apply(x, sig_a, coarse_mode=capi.COARSE_NONE).cpu().numpy()
        e_l = np.linalg.norm(yl - yp) / np.linalg.norm(yp)
        e_n = np.linalg.norm(yn - yp) / np.linalg.norm(yp)
        print("%s direction: learned vs plain V-cycle %.3f, no coarse level vs plain %.3f" % (kind, e_l, e_n))
        assert e_l <= 0.2 * e_n
    _, st_plain = fr.solve_stage(capi.stage_config_for(wl_eval), dq)
    q, st_l = fr.solve_stage(capi.stage_config_for(wl_eval, precond=capi.PRECOND_PMG_LEARNED, stall_ratio=1e9), dq)
    print("plain pMG: %d PTC / %d FGMRES, %.3f s; learned: %d PTC / %d FGMRES, %.3f s, fallbacks %d"
          % (st_plain["ptc_iters"], st_plain["gmres_iters"], st_plain["t_total"], st_l["ptc_iters"],
             st_l["gmres_iters"], st_l["t_total"], st_l["fallbacks"]))
    assert st_l["converged"] == 1 and st_l["fallbacks"] == 0
    assert st_l["gmres_iters"] <= 1.2 * st_plain["gmres_iters"]
    assert _oracle_rel_F(orc, wl_eval, q.cpu().numpy()) <= 1.5e-8
    # the product configuration (stall fallback on): the gain or loss over
    # plain pMG, as measured (the network replaces the coarse sweeps; it
    # gains only where it saves FGMRES iterations or coarse work)
    qf, st_f = fr.solve_stage(capi.stage_config_for(wl_eval, precond=capi.PRECOND_PMG_LEARNED), dq)
    _, st_p2 = fr.solve_stage(capi.stage_config_for(wl_eval), dq)
    ratio_it = st_f["gmres_iters"] / st_p2["gmres_iters"]
    ratio_t = st_p2["t_total"] / st_f["t_total"]
    print("learned with fallback: %d FGMRES (%.3fx plain pMG's), %d fallbacks, DOF/s %.3fx plain pMG's"
          % (st_f["gmres_iters"], ratio_it, st_f["fallbacks"], ratio_t))
    assert st_f["converged"] == 1 and ratio_it <= 1.1
    assert _oracle_rel_F(orc, wl_eval, qf.cpu().numpy()) <= 1.5e-8


def test_useless_network_falls_back_to_plain_pmg(orc):
    require_gpu()
    announce("lcc fallback with garbage weights")
    wl, fr = _fr(n=(16, 16))
    rng = np.random.default_rng(9)
    fr.lcc_set_scales(np.ones(wl.nv, np.float32), np.ones(wl.nv, np.float32))
    fr.lcc_set_weights([1e3 * rng.standard_normal(w.shape).astype(np.float32) for w in fr.lcc_get_weights()])
    q, st = fr.solve_stage(capi.stage_config_for(wl, precond=capi.PRECOND_PMG_LEARNED), fr.to_dev(wl.dq))
    print("garbage network: fallbacks %d, %d PTC / %d FGMRES" % (st["fallbacks"], st["ptc_iters"], st["gmres_iters"]))
    assert st["fallbacks"] >= 1
    assert st["converged"] == 1
    assert _oracle_rel_F(orc, wl, q.cpu().numpy()) <= 1.5e-8


def test_learned_on_the_3d_mesh_harvest_train_and_use():
    """The learned correction on the 32^3 p = 3 mesh (p{3-2}, features of
    7 x 135 defect entries + 3 geometry entries): pairs harvested from a few
    Rosenbrock-Euler (ROW, gamma = 1) steps and probe V-cycles, trained on the
    GPU (validation loss on the held-out last stages falls), then the ROW stage
    of a held-out state solved with the learned preconditioner (stall
    fallback on) to the recomputed 1e-8, within 1.2x plain pMG's FGMRES
    iterations; both counts and DOF/s are printed."""
    require_gpu()
    announce("lcc 3D: harvest/train/use on the 32^3 TGV mesh")
    import torch
    wl = W.make_tgv_workload(seed=5)
    fr = capi.FR.from_workload(wl)
    d = fr.lcc_dims()
    assert d["nin"] == 7 * 135 + 3 and d["nout"] == 135
    q = fr.to_dev(wl.dq)
    sig_a = 1.0 / (wl.a_ii * wl.dt)
    sig_s = 1.0 / wl.dt + sig_a
    fr.lcc_harvest(enable=1, max_pairs=60000, stride=256, target_sweeps=2, reset=1)
    fr.ej_factor(0, q, sig_s)
    fr.ej_factor(1, fr.restrict(0, q), sig_s)
    fr.pmg_set_point(q, fr.residual(0, q))
    for i in range(20):
        x = torch.randn_like(q)
        if i % 2 == 1:
            x = fr.prolong(1, fr.restrict(0, x))
        fr.pmg_apply(x, sig_a)
    Y = fr.empty(0)
    for _ in range(6):
        _, st = fr.solve_stage(capi.stage_config_for(wl, a_ii=1.0, verify=0), q, out=Y)
        q = q + Y
    fr.lcc_harvest(enable=0)
    n = fr.lcc_count()
    ts = fr.lcc_train(epochs=20, batch=256, lr=1e-3, seed=7, holdout=0.15, reinit=1)
    print("3D: %d pairs; training %s" % (n, ts))
    assert n >= 20000 and ts["val_loss"] < 0.5 * ts["val_loss_init"]
    wl_eval = W.make_tgv_workload(seed=40)
    dq = fr.to_dev(wl_eval.dq)
    _, st_p = fr.solve_stage(capi.stage_config_for(wl_eval), dq)
    Yl, st_l = fr.solve_stage(capi.stage_config_for(wl_eval, precond=capi.PRECOND_PMG_LEARNED), dq)
    print("3D held-out stage: plain pMG %d FGMRES %.3f s; learned %d FGMRES %.3f s, %d fallbacks, true rel. res %.2e"
          % (st_p["gmres_iters"], st_p["t_total"], st_l["gmres_iters"], st_l["t_total"], st_l["fallbacks"],
             st_l["true_rel_res"]))
    assert st_l["converged"] == 1 and st_l["true_rel_res"] <= 1e-8
    assert st_l["gmres_iters"] <= 1.2 * st_p["gmres_iters"]
