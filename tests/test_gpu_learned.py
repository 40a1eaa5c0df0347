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


def _bf16_forward(Ws, X):
    Wb = [mlp.bf16_round(w) for w in Ws]
    H1 = mlp.bf16_round(np.maximum(mlp.bf16_round(X) @ Wb[0].T, 0))
    H2 = mlp.bf16_round(np.maximum(H1 @ Wb[1].T, 0))
    return H2 @ Wb[2].T


def test_forward_parity(orc):
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
    e_emul = rel(Y, _bf16_forward(Ws, X))
    e_fp64 = rel(Y, mlp.forward(Ws, X)[0])
    print("forward: vs BF16-emulating FP64 %.2e, vs plain FP64 %.2e" % (e_emul, e_fp64))
    assert e_emul <= 1e-2 and e_fp64 <= 3e-2


def test_gradient_parity(orc):
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
    loss_ref, g_ref = mlp.loss_grad([mlp.bf16_round(w) for w in Ws], mlp.bf16_round(X), T, d["nout"])
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    for l in range(3):
        e = rel(g[l], g_ref[l])
        cos = float(np.sum(g[l] * g_ref[l]) / (np.linalg.norm(g[l]) * np.linalg.norm(g_ref[l])))
        print("layer %d gradient: rel err %.2e, cosine %.6f" % (l + 1, e, cos))
        assert e <= 5e-2 and cos >= 0.999


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
    reaches 1e-8 in the oracle's own F on its own, within 1.25x plain pMG's
    FGMRES iterations.  Iteration counts and times of both preconditioners
    are printed (the A/B comparison)."""
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
    assert st_l["gmres_iters"] <= 1.25 * st_plain["gmres_iters"]
    assert _oracle_rel_F(orc, wl_eval, q.cpu().numpy()) <= 1.5e-8


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
