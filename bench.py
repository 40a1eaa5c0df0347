"""Benchmark: DOF/s of one implicit stage solve to 1e-8 relative residual on
one MI355X, plus the residual/JVP/EJ kernel rates.

Workload (the headline `value`): 3D Navier-Stokes FR on the periodic 32^3 hex
mesh, p = 3 (10,485,760 DOF, EJ blocks 320 x 320), Taylor-Green vortex plus
seeded noise, Ma 0.1, Re 1600; the first ROW stage (gamma 0.25) at
dt = 100 dt_exp, solved by FGMRES(30) with the nonlinear pMG p{3-2}
preconditioner (n{2-2}, EJ smoothing on both levels), FP64, until the
residual of the FD operator recomputed at the solution, ||R - A_h Y||, is at
most 1e-8 ||R||.  One step = one full stage solve, including the
per-time-step preconditioner set-up (EJ formation and inversion on both
levels) at the start.  The 2D 64x64 p = 4 ESDIRK stage and the other
comparisons are extras of the same JSON line.

Prints ONE JSON line (see the fields in main()).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# precision forms of the preconditioner (values of the library's FR_PREC_* codes)
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16s": 3}


def measured_traffic(profile="k_ej_apply_tgv32.md"):
    """HBM bytes per fine-level FP64 k_ej_apply launch from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None if the kernel source has
    changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", profile)
    csrc = os.path.join(ROOT, "paper_2202_09733_amd", "csrc")
    try:
        txt = open(path).read()
        want = re.search(r"ej_apply.hip \+ ej.hip sha256: (\w+)", txt).group(1)
        val = float(re.search(r"fp64 traffic bytes per launch: (\d+)", txt).group(1))
    except (OSError, AttributeError):
        return None
    # the kernel's source and the factorisation that fixes its inputs' layout
    h = hashlib.sha256()
    for f in ("ej_apply.hip", "ej.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return val if h.hexdigest() == want else None


def _events_time(fn, reps):
    """Average duration (s) of fn() over reps calls, HIP events on the current stream."""
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def kernel_rates(fr, wl, dq_dev, reps=50):
    """Live per-launch durations of the hot kernels at the workload's size."""
    import torch
    from paper_2202_09733_amd import capi
    N = wl.dof()
    nb = wl.nv * (wl.p0 + 1) ** wl.dim
    out = {}
    rq = fr.residual(0, dq_dev)
    r_out = fr.empty(0)
    t_r = _events_time(lambda: fr.residual(0, dq_dev, out=r_out), reps)
    out["residual"] = dict(s_per_call=t_r, alg_bytes=16.0 * N, launches=2)
    v = torch.randn_like(dq_dev)
    v /= torch.linalg.norm(v)
    w = fr.empty(0)
    sig = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    t_j = _events_time(lambda: fr.jvp(0, dq_dev, rq, v, sig, out=w), reps)
    out["jvp"] = dict(s_per_call=t_j, alg_bytes=32.0 * N, launches=4)
    # EJ apply on the fine level (factors of the last stage solve)
    y = fr.empty(0)
    t_e = _events_time(lambda: fr.ej_solve(0, v, out=y), reps)
    fac_bytes = wl.Ne * nb * nb * (8 if fr_prec(fr) == capi.PREC_FP64 else 4)
    # blocks above 64 unknowns are inverted in blocked form, whose column
    # placement (one int per block column) the apply reads with the blocks
    cols_bytes = wl.Ne * nb * 4 if nb > 64 else 0
    out["ej_apply_fine"] = dict(s_per_call=t_e, alg_bytes=float(fac_bytes + cols_bytes + 16 * N), launches=1,
                                kernel="k_ej_apply")
    # reference: a plain device copy of 512 MiB (256 MiB read + 256 MiB written)
    a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dq_dev.device).normal_()
    b = torch.empty_like(a)
    t_c = _events_time(lambda: b.copy_(a), 20)
    out["device_copy_512MiB"] = dict(s_per_call=t_c, alg_bytes=float(2 * a.numel() * 8), launches=1)
    for k, d in out.items():
        d["GBps"] = d["alg_bytes"] / d["s_per_call"] / 1e9
    return out


def kernel_rates_3d(reps=20, nsets=4):
    """R and JVP at the 3D workload (32^3 hexes, p = 3, 10,485,760 DOF, 84 MB
    per vector), rotating over nsets independent buffer sets (> 1 GB in all)
    so that the 256 MB last-level cache cannot serve them from one launch to
    the next."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    wl = W.tgv_32cubed_p3()
    fr = capi.FR.from_workload(wl, levels=[wl.p0])
    N = wl.dof()
    base = fr.to_dev(wl.dq)
    sets = []
    for i in range(nsets):
        dq = base + 1e-4 * torch.randn_like(base) if i else base
        v = torch.randn_like(base)
        v /= torch.linalg.norm(v)
        sets.append(dict(dq=dq, rq=fr.residual(0, dq), v=v, out=fr.empty(0)))
    sig = 1.0 / (wl.a_ii * wl.dt)
    it = {"i": 0}

    def nxt():
        it["i"] = (it["i"] + 1) % nsets
        return sets[it["i"]]

    def r_call():
        b = nxt()
        fr.residual(0, b["dq"], out=b["out"])

    def j_call():
        b = nxt()
        fr.jvp(0, b["dq"], b["rq"], b["v"], sig, out=b["out"])
    out = {
        "residual_3d": dict(s_per_call=_events_time(r_call, reps), alg_bytes=16.0 * N, launches=2),
        "jvp_3d": dict(s_per_call=_events_time(j_call, reps), alg_bytes=32.0 * N, launches=4),
    }
    for d in out.values():
        d["GBps"] = d["alg_bytes"] / d["s_per_call"] / 1e9
        d["frac_hbm"] = d["GBps"] / HBM_PEAK_GBS
    fr.close()
    del sets, base
    torch.cuda.empty_cache()
    return out


def time_steps():
    """Full implicit time steps (every stage, EJ factors formed once at q^n)
    of the 2D (64x64, p = 4) and 3D (32^3, p = 3) workloads with the ESDIRK
    (PTC + inexact Newton per implicit stage) and ROW (one linear solve per
    stage) schemes of orders 2, 3 and 4, each pair of one order sharing its
    diagonal; preconditioner in FP64 and in the BF16-storage form: DOF per
    second of step time, after one warm-up step each.  The 3D workload runs
    the order-2 pair in FP64 and the order-3 pair in both forms."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    tabs = {"esdirk2": capi.TAB_ESDIRK2, "row2": capi.TAB_ROW2, "esdirk3": capi.TAB_ESDIRK3,
            "row3": capi.TAB_ROW3, "esdirk4": capi.TAB_ESDIRK4, "row4": capi.TAB_ROW4}
    precs = {"fp64": capi.PREC_FP64, "bf16_storage": capi.PREC_BF16_STORE}
    plans = (("vortical2d", W.vortical_64x64_p4, 2, ((2, ("fp64", "bf16_storage")), (3, ("fp64", "bf16_storage")),
                                                      (4, ("fp64", "bf16_storage")))),
             ("tgv3d", W.tgv_32cubed_p3, 1, ((2, ("fp64",)), (3, ("fp64", "bf16_storage")))))
    out = {}
    for wname, mk, reps, orders in plans:
        wl = mk()
        fr = capi.FR.from_workload(wl)
        dq = fr.to_dev(wl.dq)
        q = fr.empty(0)
        res = {}
        for order, pkeys in orders:
            for pkey in pkeys:
                for tkey in ("esdirk%d" % order, "row%d" % order):
                    cfg = capi.stage_config_for(wl, precision=precs[pkey])
                    fr.time_step(cfg, dq, tableau=tabs[tkey], out=q)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        _, st = fr.time_step(cfg, dq, tableau=tabs[tkey], out=q)
                    torch.cuda.synchronize()
                    el = (time.perf_counter() - t0) / reps
                    res["%s_%s" % (tkey, pkey)] = {
                        "dof_per_s": wl.dof() / el, "s_per_step": el, "t_setup_s": st["t_setup"],
                        "t_solve_s": st["t_solve"], "gmres_iters": st["gmres_iters"],
                        "gmres_per_stage": [x["gmres_iters"] for x in st["stages"]], "ptc_iters": st["ptc_iters"]}
                res["row%d_vs_esdirk%d_%s" % (order, order, pkey)] = (
                    res["row%d_%s" % (order, pkey)]["dof_per_s"] / res["esdirk%d_%s" % (order, pkey)]["dof_per_s"])
        out.setdefault(wname, {}).update(res)
        fr.close()
        torch.cuda.empty_cache()
    out["note"] = ("one full step at the workload's dt from its state; ESDIRK stages to ||F|| <= 1e-8 "
                   "||F(q_{i-1})|| with eta 0.1, ROW stages by FGMRES to 1e-8; pMG p{p0-p0/2} n{2-2}; "
                   "gamma = 1 - 1/sqrt(2) (order 2), 0.4359 (order 3), 1/4 (ESDIRK4), 0.5728 (ROW4)")
    return out


def hierarchies():
    """Other p-hierarchies and pMG as the nonlinear solver (one stage, set-up
    included, after a warm-up): the 2D 64x64 workload (ESDIRK stage) with JFNK-pMG
    p{4-2}, p{4-2-1}, p{4-2-1-0} and the p{4-0} negative control, and with
    the pMG nonlinear solver p{4-2}, p{4-2-1} and p{4-2-1-0} (to 1e-8 and to
    1e-4 of ||F(q^n)||); the 3D 32^3 workload (ROW stage) with GMRES-pMG p{3-2},
    p{3-2-1} and the p{3-0} negative control."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    out = {}
    for wname, mk, levels, runs in (
            ("vortical2d", W.vortical_64x64_p4, [4, 2, 1], (
                ("jfnk_pmg_p42", dict(pmg_levels=2)),
                ("jfnk_pmg_p421", dict(pmg_levels=3)),
                ("pmg_solver_p42", dict(pmg_levels=2, solver=1, max_ptc=1000)),
                ("pmg_solver_p42_refresh20", dict(pmg_levels=2, solver=1, max_ptc=1000, smoother_refresh=20)),
                ("pmg_solver_p421", dict(pmg_levels=3, solver=1, max_ptc=1000)),
                ("jfnk_pmg_p42_tol1e-4", dict(pmg_levels=2, tol=1e-4)),
                ("pmg_solver_p42_tol1e-4", dict(pmg_levels=2, solver=1, tol=1e-4, max_ptc=1000)))),
            ("vortical2d", W.vortical_64x64_p4, [4, 0], (
                ("jfnk_pmg_p40", dict()),
                ("jfnk_pmg_p40_mbnk", dict(coarse_smoother=1)))),
            ("vortical2d", W.vortical_64x64_p4, [4, 2, 1, 0], (
                ("jfnk_pmg_p4210", dict()),
                ("pmg_solver_p4210", dict(solver=1, max_ptc=1000)))),
            ("tgv3d", W.tgv_32cubed_p3, [3, 2, 1], (
                ("gmres_pmg_p32", dict(pmg_levels=2)),
                ("gmres_pmg_p321", dict(pmg_levels=3)))),
            ("tgv3d", W.tgv_32cubed_p3, [3, 0], (
                ("gmres_pmg_p30", dict()),))):
        wl = mk()
        fr = capi.FR.from_workload(wl, levels=levels)
        dq = fr.to_dev(wl.dq)
        q = fr.empty(0)
        res = {}
        for key, kw in runs:
            cfg = capi.stage_config_for(wl, **kw)
            try:
                fr.solve_stage(cfg, dq, out=q, raise_on_noconv=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = fr.solve_stage(cfg, dq, out=q, raise_on_noconv=False)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                res[key] = {"dof_per_s": wl.dof() / el, "s_per_stage": el, "ptc_or_vcycles": st["ptc_iters"],
                            "gmres_iters": st["gmres_iters"], "rel_res": st["rel_res"],
                            "converged": st["converged"]}
            except capi.FRError as ex:
                res[key] = {"failed": str(ex)}
        out.setdefault(wname, {}).update(res)
        fr.close()
        torch.cuda.empty_cache()
    out["note"] = ("stage tolerance 1e-8 unless marked; the pMG nonlinear solver smooths with dtau = dt and "
                   "counts V-cycles in ptc_or_vcycles; a failure entry records a diverged solve")
    return out


def smoothers():
    """Coarsest-level smoother (Sec. 3.2: EJ or MBNK) on the 64x64 vortical ESDIRK
    stage for the hierarchies p{4-2}, p{4-2-1} and p{4-1}: one stage each,
    set-up included, after a warm-up; JFNK-pMG and the pMG nonlinear solver."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    wl = W.vortical_64x64_p4()
    out = {}
    for levels, runs in (
            ([4, 2, 1], (("p42_ej", dict(pmg_levels=2)),
                         ("p42_mbnk", dict(pmg_levels=2, coarse_smoother=1)),
                         ("p42_mbnk_graphs", dict(pmg_levels=2, coarse_smoother=1, graphs=1)),
                         ("p421_ej", dict(pmg_levels=3)),
                         ("p421_mbnk", dict(pmg_levels=3, coarse_smoother=1)),
                         ("pmg_solver_p42_ej", dict(pmg_levels=2, solver=1, max_ptc=1000)),
                         ("pmg_solver_p42_mbnk", dict(pmg_levels=2, solver=1, max_ptc=1000, coarse_smoother=1)))),
            ([4, 1], (("p41_ej", dict()),
                      ("p41_mbnk", dict(coarse_smoother=1))))):
        fr = capi.FR.from_workload(wl, levels=levels)
        dq = fr.to_dev(wl.dq)
        q = fr.empty(0)
        for key, kw in runs:
            cfg = capi.stage_config_for(wl, **kw)
            try:
                fr.solve_stage(cfg, dq, out=q, raise_on_noconv=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = fr.solve_stage(cfg, dq, out=q, raise_on_noconv=False)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                out[key] = {"dof_per_s": wl.dof() / el, "s_per_stage": el, "t_setup": st["t_setup"],
                            "ptc_or_vcycles": st["ptc_iters"], "gmres_iters": st["gmres_iters"],
                            "rel_res": st["rel_res"], "converged": st["converged"]}
            except capi.FRError as ex:
                out[key] = {"failed": str(ex)}
        fr.close()
        torch.cuda.empty_cache()
    out["note"] = ("64x64 vortical stage to 1e-8; MBNK: GMRES(5, 1e-1) with red-black ILU0 on the coarsest level, "
                   "n1 = 2 sweeps; ptc_or_vcycles counts V-cycles for the pMG nonlinear solver")
    return out


def learned_ab(wl, steps=3):
    """The learned coarse correction on the 64x64 vortical mesh: pairs harvested by
    the solver from plain-pMG stages and from V-cycles on random directions
    at two other seeded states, the network trained on the GPU, then the
    64x64 stage timed with the learned and with the plain preconditioner
    (FP64 factors both)."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    fr = capi.FR.from_workload(wl)
    rng = np.random.default_rng(11)
    t0 = time.perf_counter()
    fr.lcc_harvest(enable=1, max_pairs=400000, stride=4, target_sweeps=2, reset=1)
    for seed in (12, 13):
        w = W.make_vortical_workload(seed=seed)
        fr.solve_stage(capi.stage_config_for(w), fr.to_dev(w.dq))
        dq = fr.to_dev(w.dq)
        sig_a = 1.0 / w.dt + 1.0 / (w.a_ii * w.dt)
        sig_s = 1.0 / w.dt + sig_a
        fr.ej_factor(0, dq, sig_s)
        fr.ej_factor(1, fr.restrict(0, dq), sig_s)
        fr.pmg_set_point(dq, fr.residual(0, dq))
        for i in range(200):
            x = fr.to_dev(rng.standard_normal(fr.shape(0)))
            if i % 2 == 1:
                x = fr.prolong(1, fr.restrict(0, x))
            fr.pmg_apply(x, sig_a)
    fr.lcc_harvest(enable=0)
    t_harvest = time.perf_counter() - t0
    ts = fr.lcc_train(epochs=60, batch=256, lr=1e-3, seed=7, holdout=0.1, reinit=1)
    dq = fr.to_dev(wl.dq)
    out = {"pairs": fr.lcc_count(), "t_harvest_s": t_harvest, "t_train_s": ts["t_train"],
           "val_loss_ratio": ts["val_loss"] / ts["val_loss_init"]}
    for key, cfg in (("plain_pmg", capi.stage_config_for(wl)),
                     ("learned", capi.stage_config_for(wl, precond=capi.PRECOND_PMG_LEARNED))):
        fr.solve_stage(cfg, dq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = fr.solve_stage(cfg, dq)
        torch.cuda.synchronize()
        out[key] = {"dof_per_s": wl.dof() * steps / (time.perf_counter() - t0), "gmres_iters": st["gmres_iters"],
                    "ptc_iters": st["ptc_iters"], "rel_res": st["rel_res"], "fallbacks": st["fallbacks"]}
    out["speedup_vs_plain"] = out["learned"]["dof_per_s"] / out["plain_pmg"]["dof_per_s"]
    fr.close()
    return out


def learned_3d(n_steps=50, holdout_steps=10, pairs_per_step=2000, n_probe=40):
    """The learned coarse correction on the 32^3 p = 3 mesh (p{3-2}): pairs
    harvested by the solver from n_steps Rosenbrock-Euler steps (ROW stages
    with gamma = 1, each a pMG-preconditioned FGMRES solve) from the seeded
    Taylor-Green state, about pairs_per_step per stage, plus V-cycles of the
    same preconditioner on random directions at the first state; the last
    holdout_steps stages held out; the network trained on the GPU; then the
    ROW stage of a held-out state (noise seed 40) solved with the learned and
    with the plain preconditioner (FP64 factors both)."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    wl = W.make_tgv_workload(seed=5)
    fr = capi.FR.from_workload(wl)
    t0 = time.perf_counter()
    cfg_re = capi.stage_config_for(wl, a_ii=1.0, verify=0)
    q = fr.to_dev(wl.dq)
    # about pairs_per_step per stage: ~26 V-cycles per stage
    stride = max(1, wl.Ne * 26 // pairs_per_step)
    fr.lcc_harvest(enable=1, max_pairs=(n_steps + 1) * pairs_per_step + n_probe * (wl.Ne // stride + 1),
                   stride=stride, target_sweeps=2, reset=1)
    rng = np.random.default_rng(17)
    # random probe directions at the first state (white and smooth)
    sig_a = 1.0 / (wl.a_ii * wl.dt)
    sig_s = 1.0 / wl.dt + sig_a
    fr.ej_factor(0, q, sig_s)
    fr.ej_factor(1, fr.restrict(0, q), sig_s)
    fr.pmg_set_point(q, fr.residual(0, q))
    for i in range(n_probe):
        x = torch.randn_like(q)
        if i % 2 == 1:
            x = fr.prolong(1, fr.restrict(0, x))
        fr.pmg_apply(x, sig_a)
    n_probe_pairs = fr.lcc_count()
    Y = fr.empty(0)
    iters = []
    for step in range(n_steps):
        _, st = fr.solve_stage(cfg_re, q, out=Y)
        iters.append(st["gmres_iters"])
        q = q + Y
    fr.lcc_harvest(enable=0)
    t_harvest = time.perf_counter() - t0
    n = fr.lcc_count()
    holdout = holdout_steps / float(n_steps) * (n - n_probe_pairs) / n
    ts = fr.lcc_train(epochs=40, batch=256, lr=1e-3, seed=7, holdout=holdout, reinit=1)
    out = {"pairs": n, "probe_pairs": n_probe_pairs, "stride": stride, "t_harvest_s": t_harvest,
           "harvest_gmres_per_step": iters, "t_train_s": ts["t_train"],
           "val_loss_ratio": ts["val_loss"] / ts["val_loss_init"], "holdout_fraction": holdout}
    wl_eval = W.make_tgv_workload(seed=40)
    dq = fr.to_dev(wl_eval.dq)
    for key, cfg in (("plain_pmg", capi.stage_config_for(wl_eval)),
                     ("learned", capi.stage_config_for(wl_eval, precond=capi.PRECOND_PMG_LEARNED)),
                     ("learned_no_fallback", capi.stage_config_for(wl_eval, precond=capi.PRECOND_PMG_LEARNED,
                                                                   stall_ratio=1e9))):
        fr.solve_stage(cfg, dq, out=Y, raise_on_noconv=False)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, st = fr.solve_stage(cfg, dq, out=Y, raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - ta
        out[key] = {"dof_per_s": wl_eval.dof() / el, "s_per_stage": el, "gmres_iters": st["gmres_iters"],
                    "restarts": st["restarts"], "true_rel_res": st["true_rel_res"], "fallbacks": st["fallbacks"],
                    "converged": st["converged"]}
    out["speedup_vs_plain"] = out["learned"]["dof_per_s"] / out["plain_pmg"]["dof_per_s"]
    out["workload"] = ("32^3 p{3-2} TGV: harvest from Rosenbrock-Euler (gamma = 1) steps at dt = 100 dt_exp from "
                       "noise seed 5; evaluation: the first ROW stage (gamma 0.25) of noise seed 40")
    fr.close()
    torch.cuda.empty_cache()
    return out


def fr_prec(fr):
    return getattr(fr, "_last_prec", 0)


def cpu_baseline(wl, st):
    """The oracle (plain FP64 C + numpy, one thread) on a bounded sample of
    the headline stage (32^3, p = 3): one fine and one coarse residual
    evaluation at full size, the LU factorisation and solve of 32 blocks of
    each level's size, and 13 FGMRES iterations of its Gram-Schmidt at full
    vector length (with a diagonal operator and no preconditioner, so that
    they time the orthogonalisation alone).  Extrapolated to the whole stage
    with the oracle's own algorithm (EJ blocks by parity-coloured differencing:
    2^3 n_b + 1 residual evaluations per level, block LU of every element)
    and the GPU stage's operation counts; the sample says so."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t_begin = time.perf_counter()
        L0 = oracle.Level(**wl.level_kwargs(wl.p0))
        L1 = oracle.Level(**wl.level_kwargs(wl.p1))
        P0, P1 = wl.p0 + 1, wl.p1 + 1
        t0 = time.perf_counter()
        L0.residual(wl.dq)
        t_r0 = time.perf_counter() - t0
        q1 = oracle.restrict(wl.dq, wl.dim, P0, P1)
        t0 = time.perf_counter()
        L1.residual(q1)
        t_r1 = time.perf_counter() - t0
        rng = np.random.default_rng(0)
        t_lu, t_sv = [], []
        for L in (L0, L1):
            B = rng.standard_normal((32, L.nb, L.nb)) + 4.0 * np.sqrt(L.nb) * np.eye(L.nb)
            t0 = time.perf_counter()
            fac = oracle.lu_factor(B)
            t_lu.append((time.perf_counter() - t0) / 32)
            x = rng.standard_normal((L.nv, L.Np, 32))
            t0 = time.perf_counter()
            oracle.lu_solve(fac, x)
            t_sv.append((time.perf_counter() - t0) / 32)
        d = rng.uniform(1.0, 2.0, L0.shape)
        b = rng.standard_normal(L0.shape)
        t0 = time.perf_counter()
        _, ks = oracle.fgmres(lambda v: d * v, lambda v: v, b, m=13, tol=1e-300, max_restarts=0, max_iters=13)
        t_cgs = time.perf_counter() - t0
        del d, b
    c_orth = t_cgs / sum(j + 1 for j in range(ks.iters))   # per (basis vector x iteration)
    Ne = wl.Ne
    nb0, nb1 = L0.nb, L1.nb
    t_setup = ((2 ** wl.dim * nb0 + 1) * t_r0 + (2 ** wl.dim * nb1 + 1) * t_r1
               + Ne * (t_lu[0] + t_lu[1]))
    it = st["gmres_iters"]
    cycles = st["restarts"] + 1
    per = [it // cycles + (1 if i < it % cycles else 0) for i in range(cycles)]
    t_orth = c_orth * sum(sum(j + 1 for j in range(n)) for n in per)
    t_solve = (st["n_R_fine"] * t_r0 + st["n_R_coarse"] * t_r1 + st["n_ej_fine"] * Ne * t_sv[0]
               + st["n_ej_coarse"] * Ne * t_sv[1] + t_orth)
    total = t_setup + t_solve
    return dict(value=wl.dof() / total, unit="DOF/s", cores=1, kind="oracle", extrapolated=True,
                sample=("oracle, one thread, on the 32^3 p=3 stage's data: fine residual %.2f s, coarse residual "
                        "%.2f s, LU %.2f / %.2f ms and solve %.3f / %.3f ms per 320^2 / 135^2 block (32 sampled), "
                        "Gram-Schmidt %.3f s over %d iterations at full length; measuring took %.1f s.  "
                        "Extrapolated: set-up %.0f s (coloured formation %d + %d residuals, %d block LUs per "
                        "level), solve %.0f s (the GPU stage's %d fine / %d coarse residuals, %d / %d EJ "
                        "applies, %d FGMRES iterations) = %.0f s")
                % (t_r0, t_r1, 1e3 * t_lu[0], 1e3 * t_lu[1], 1e3 * t_sv[0], 1e3 * t_sv[1], t_cgs, ks.iters,
                   time.perf_counter() - t_begin, t_setup, 2 ** wl.dim * nb0 + 1, 2 ** wl.dim * nb1 + 1, Ne,
                   t_solve, st["n_R_fine"], st["n_R_coarse"], st["n_ej_fine"], st["n_ej_coarse"], it, total),
                seconds_extrapolated=total)


def cpu_full_stage_2d():
    """The oracle's complete 64x64 p = 4 ESDIRK stage (set-up and every PTC
    step, pMG p{4-2}), one thread, timed end to end: nothing extrapolated."""
    import oracle
    from threadpoolctl import threadpool_limits
    from paper_2202_09733_amd import workloads as W
    wl = W.vortical_64x64_p4()
    with threadpool_limits(limits=1):
        L0 = oracle.Level(**wl.level_kwargs(wl.p0))
        L1 = oracle.Level(**wl.level_kwargs(wl.p1))
        t0 = time.perf_counter()
        _, so = oracle.esdirk_stage(L0, L1, wl.dq, wl.dt, wl.a_ii)
        el = time.perf_counter() - t0
    return dict(value=wl.dof() / el, unit="DOF/s", cores=1, kind="oracle", seconds=el, ptc_iters=so.ptc_iters,
                gmres_iters=so.gmres_iters, rel_res=so.rel_res, converged=bool(so.converged),
                sample="the whole 64x64 p=4 ESDIRK3 stage (409,600 DOF), set-up included, one thread")


def only_kernel(args):
    """Profiling driver: build the chosen workload's state, launch one kernel
    family --reps times, then a plain 256 MiB device copy whose counter
    readings calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    if args.workload == "padapt2d":
        wl = W.make_padapt_workload()
        fr = capi.FR.from_padapt(wl, wl.extra["deg"], nlevels=2, gap=2)
    else:
        wl = W.vortical_64x64_p4() if args.workload == "vortical2d" else W.tgv_32cubed_p3()
        fr = capi.FR.from_workload(wl)
    prec = PRECISIONS[args.precision]
    dq = fr.to_dev(wl.dq)
    sig = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    x = torch.randn_like(dq)
    y = fr.empty(0)
    if args.only_kernel == "step":
        # whole time steps (every stage, set-up included) with the requested tableau
        tab = {"esdirk2": capi.TAB_ESDIRK2, "row2": capi.TAB_ROW2, "esdirk3": capi.TAB_ESDIRK3,
               "row3": capi.TAB_ROW3, "esdirk4": capi.TAB_ESDIRK4, "row4": capi.TAB_ROW4}[args.tableau]
        for _ in range(args.reps):
            _, st = fr.time_step(capi.stage_config_for(wl, precision=prec), dq, tableau=tab)
            print("[bench] %s step: %d FGMRES %s, set-up %.3f s, solve %.3f s"
                  % (args.tableau, st["gmres_iters"], [x["gmres_iters"] for x in st["stages"]], st["t_setup"],
                     st["t_solve"]), file=sys.stderr)
        torch.cuda.synchronize()
        return
    if args.only_kernel == "stage":
        # whole stage solves (set-up included) in the requested precision and coarse smoother
        sm = capi.SMOOTHER_MBNK if args.coarse_smoother == "mbnk" else capi.SMOOTHER_EJ
        for _ in range(args.reps):
            _, st = fr.solve_stage(capi.stage_config_for(wl, precision=prec, coarse_smoother=sm), dq)
            print("[bench] stage: %d FGMRES, set-up %.3f s, solve %.3f s" % (st["gmres_iters"], st["t_setup"],
                                                                           st["t_solve"]), file=sys.stderr)
        torch.cuda.synchronize()
        return
    if args.only_kernel == "ej_apply":
        fr.ej_factor(0, dq, sig, prec)
    rq = fr.residual(0, dq)
    torch.cuda.synchronize()
    print("[bench] only-kernel %s on %s, precision %s" % (args.only_kernel, args.workload, args.precision),
          file=sys.stderr, flush=True)
    for _ in range(args.reps):
        if args.only_kernel == "ej_apply":
            fr.ej_solve(0, x, out=y)
        elif args.only_kernel == "ej_factor":
            fr.ej_factor(0, dq, sig, prec)
        elif args.only_kernel == "residual":
            fr.residual(0, dq, out=y)
        else:
            fr.jvp(0, dq, rq, x, sig, out=y)
    torch.cuda.synchronize()
    a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dq.device).normal_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("[bench] only-kernel %s x%d done" % (args.only_kernel, args.reps), file=sys.stderr)


def _timed_stages(fr, cfg, dq, out, steps, tag):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        _, st = fr.solve_stage(cfg, dq, out=out)
        stats.append(st)
        print("[bench] %s step %d: %.3f s (setup %.3f s), %d PTC, %d FGMRES, %d restarts, rel. residual %.2e"
              % (tag, i, st["t_total"], st["t_setup"], st["ptc_iters"], st["gmres_iters"], st["restarts"],
                 st["true_rel_res"] if cfg.scheme == 1 else st["rel_res"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats


def headline(args, prec):
    """The 32^3 p = 3 ROW stage: warm-up, the timed steps, the roofline
    kernel (fine FP64 EJ apply) timed live on the library's stream, and (with
    extras) the precision forms and the central FD product."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    wl = W.tgv_32cubed_p3()
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    cfg = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=prec)
    out = fr.empty(0)
    print("[bench] 32^3 p=3 ROW stage: warmup %d" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        fr.solve_stage(cfg, dq, out=out)
    elapsed, stats = _timed_stages(fr, cfg, dq, out, args.steps, "32^3")
    dof = wl.dof()
    st = stats[-1]
    solve_only = float(np.mean([x["t_solve"] for x in stats]))
    setup = float(np.mean([x["t_setup"] for x in stats]))
    res = {
        "value": dof * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps, "dof": dof,
        "stage": {"dof_per_s_without_setup": dof / solve_only, "t_setup_s": setup, "t_solve_s": solve_only,
                  "gmres_iters": st["gmres_iters"], "restarts": st["restarts"], "krylov_rel_res": st["rel_res"],
                  "true_rel_res": st["true_rel_res"], "n_R_fine": st["n_R_fine"], "n_R_coarse": st["n_R_coarse"],
                  "n_ej_fine": st["n_ej_fine"], "n_ej_coarse": st["n_ej_coarse"]},
        "stats": st,
    }
    # the dominant kernel: the fine EJ apply with the FP64 inverse of the last stage
    if prec == capi.PREC_FP64:
        nb = wl.nv * (wl.p0 + 1) ** wl.dim
        v = torch.randn_like(dq)
        y = fr.empty(0)
        t_ap = _events_time(lambda: fr.ej_solve(0, v, out=y), 10)
        alg = float(wl.Ne * nb * nb * 8 + wl.Ne * nb * 4 + 16 * dof)
        res["roofline"] = {
            "kernel": "k_ej_apply (fine level, 32,768 blocks of 320 x 320, FP64 inverse, column placement)",
            "bound": "hbm", "achieved": alg / t_ap / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg / t_ap / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "alg_bytes_per_launch": alg, "launch_us": t_ap * 1e6}
    if not args.no_extras:
        variants = [("central_fd", dict(eps_mode=capi.EPS_SCALED | capi.FD_CENTRAL),
                     "the same stage with the central FD product (O(h^2); two residuals per product)")]
        if prec == capi.PREC_FP64:
            variants += [
                ("precision_fp32_factors", dict(precision=capi.PREC_FP32),
                 "EJ inverses stored FP32 on both levels; R, JVP, FGMRES, stage update FP64"),
                ("precision_bf16_mfma_factors", dict(precision=capi.PREC_FP32_BF16),
                 "blocked Gauss-Jordan with BF16-MFMA (hi/lo, FP32 accumulate) updates, inverses stored FP32"),
                ("precision_bf16_storage", dict(precision=capi.PREC_BF16_STORE),
                 "as precision_bf16_mfma_factors, inverses stored BF16 (FP64 accumulation in the apply)")]
        for key, kw, note in variants:
            print("[bench] 32^3 variant " + key, file=sys.stderr, flush=True)
            cfgv = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=prec)
            for k, val in kw.items():
                setattr(cfgv, k, val)
            fr.solve_stage(cfgv, dq, out=out)
            el, sts = _timed_stages(fr, cfgv, dq, out, 1, key)
            stv = sts[-1]
            vv = dof / el
            v_ap = torch.randn_like(dq)
            t_ap = _events_time(lambda: fr.ej_solve(0, v_ap, out=out), 5)
            res[key] = {"value": vv, "speedup_vs_headline": vv / res["value"], "t_setup_s": stv["t_setup"],
                        "t_solve_s": stv["t_solve"], "gmres_iters": stv["gmres_iters"], "restarts": stv["restarts"],
                        "true_rel_res": stv["true_rel_res"], "fine_ej_apply_ms": t_ap * 1e3, "note": note}
    fr.close()
    del dq, out
    torch.cuda.empty_cache()
    return wl, res


def vortical2d_extras(args, prec):
    """The 64x64 p = 4 ESDIRK stage (the paper's low-Mach, high-aspect-ratio
    regime): FP64 pMG, the plain-EJ stage, graph replay, the precision forms,
    and the 2D kernel rates."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    wl = W.vortical_64x64_p4()
    fr = capi.FR.from_workload(wl)
    fr._last_prec = prec
    dq = fr.to_dev(wl.dq)
    dof = wl.dof()
    cfg = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=prec)
    out = fr.empty(0)
    fr.solve_stage(cfg, dq, out=out)
    elapsed, stats = _timed_stages(fr, cfg, dq, out, args.steps, "64x64")
    st = stats[-1]
    res = {"value": dof * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
           "workload": "2D NS FR 64x64 y-stretched (AR 1-100), p=4 (409,600 DOF), Ma 1e-3, ESDIRK3 stage at "
                       "dt=1000 dt_exp, PTC+JFNK+FGMRES(30), pMG p{4-2} n{2-2} EJ smoothers, FP64",
           "t_setup_s": float(np.mean([x["t_setup"] for x in stats])),
           "t_solve_s": float(np.mean([x["t_solve"] for x in stats])), "ptc_iters": st["ptc_iters"],
           "gmres_iters": st["gmres_iters"], "gmres_per_newton": st["gmres_per_newton"], "rel_res": st["rel_res"]}
    print("[bench] 64x64 plain-EJ comparison stage", file=sys.stderr, flush=True)
    for key, kw in (("plain_ej", dict()), ("plain_ej_eta1e-3_kdim100", dict(eta=1e-3, m=100))):
        cfg_ej = capi.stage_config_for(wl, precond=capi.PRECOND_EJ, precision=prec, **kw)
        _, st_ej = fr.solve_stage(cfg_ej, dq, out=fr.empty(0), raise_on_noconv=False)
        res[key] = {k: st_ej[k] for k in ("ptc_iters", "gmres_iters", "rel_res", "t_total", "t_setup",
                                          "converged")}
        res[key]["dof_per_s"] = dof / st_ej["t_total"]
    print("[bench] 64x64 graph-replay comparison stage", file=sys.stderr, flush=True)
    cfg_e = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=prec, graphs=1)
    fr.solve_stage(cfg_e, dq, out=fr.empty(0))
    el, sts = _timed_stages(fr, cfg_e, dq, out, args.steps, "64x64 graphs")
    res["graph_replay"] = {"value": dof * args.steps / el, "gmres_iters": sts[-1]["gmres_iters"]}
    if prec == capi.PREC_FP64:
        for key, pv in (("precision_fp32_factors", capi.PREC_FP32),
                        ("precision_bf16_mfma_factors", capi.PREC_FP32_BF16),
                        ("precision_bf16_storage", capi.PREC_BF16_STORE)):
            print("[bench] 64x64 preconditioner variant " + key, file=sys.stderr, flush=True)
            cfgv = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=pv)
            fr.solve_stage(cfgv, dq, out=out)
            el, sts = _timed_stages(fr, cfgv, dq, out, args.steps, key)
            stv = sts[-1]
            vv = dof * args.steps / el
            v_ap = torch.randn_like(dq)
            y_ap = fr.empty(0)
            t_ap = _events_time(lambda: fr.ej_solve(0, v_ap, out=y_ap), 50)
            res[key] = {"value": vv, "speedup_vs_fp64": vv / res["value"], "t_setup_s": stv["t_setup"],
                        "ptc_iters": stv["ptc_iters"], "gmres_iters": stv["gmres_iters"], "rel_res": stv["rel_res"],
                        "fine_ej_apply_us": t_ap * 1e6}
    # the FP64 factors again for the kernel rates
    fr.solve_stage(cfg, dq, out=out)
    print("[bench] 64x64 kernel rates", file=sys.stderr, flush=True)
    res["kernels"] = kernel_rates(fr, wl, dq)
    fr.close()
    torch.cuda.empty_cache()
    return wl, res


def padapt():
    """p-adaptive FR (Sec. 3.3) on the 32 x 32 vortical mesh: the first ROW
    stage on the ring degree map (degrees 1..4, nested p{4-2} pMG) beside
    the uniform p = 4 stage on the same mesh, field and step; residual launch
    times of both; one adaptation cycle (indicator, degree update, L2
    projection of the state, new degree map).  The same pair on a 128 x 128
    mesh (keys suffixed _128), where the launches are no longer a few
    workgroups each."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    out = {}
    for key, uni, n in (("p_adaptive", False, 32), ("uniform_p4", True, 32),
                        ("p_adaptive_128", False, 128), ("uniform_p4_128", True, 128)):
        wl = W.make_padapt_workload(n=(n, n), uniform=uni)
        deg = wl.extra["deg"]
        fr = capi.FR.from_padapt(wl, deg, nlevels=2, gap=2) if not uni else capi.FR.from_workload(wl, levels=[4, 2])
        dq = fr.to_dev(wl.dq)
        dof = int(wl.nv * np.sum((deg.astype(np.int64) + 1) ** 2))
        cfg = capi.stage_config_for(wl, precond=capi.PRECOND_PMG)
        y = fr.empty(0)
        fr.solve_stage(cfg, dq, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            _, st = fr.solve_stage(cfg, dq, out=y)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        r = fr.empty(0)
        t_res = _events_time(lambda: fr.residual(0, dq, out=r), 50)
        out[key] = {"dof": dof, "degrees": np.bincount(deg, minlength=5).tolist(), "stage_s": el,
                    "dof_per_s": dof / el, "gmres_iters": st["gmres_iters"], "true_rel_res": st["true_rel_res"],
                    "t_setup_s": st["t_setup"], "residual_us": t_res * 1e6}
        if not uni and n == 32:
            d_deg = torch.as_tensor(deg, device=fr.device)

            def cycle():
                eta = fr.pa_indicator(0, dq)
                new = fr.pa_adapt(eta, d_deg, p_max=4)
                fr.pa_project(d_deg, 4, dq, new, 4)
                return new

            new = cycle()
            torch.cuda.synchronize()
            t_dev = _events_time(cycle, 20)
            nd = new.cpu().numpy()
            # host cost of installing a degree map (lists, buffers, tables): the
            # current map again, since the context's level degrees are fixed
            t0 = time.perf_counter()
            fr.set_degrees(deg, 2)
            t_set = time.perf_counter() - t0
            out[key]["adapt_cycle"] = {"indicator_adapt_project_us": t_dev * 1e6, "set_degrees_ms": t_set * 1e3,
                                       "raised": int(np.sum(nd > deg)), "lowered": int(np.sum(nd < deg)),
                                       "new_degrees": np.bincount(nd, minlength=5).tolist()}
        fr.close()
        torch.cuda.empty_cache()
    out["workload"] = ("2D NS FR periodic 32x32 and 128x128, Ma 0.1, Re 1000, vortical field |u'| <= 0.05; degrees "
                       "in rings (4 at the centre down to 1) vs p = 4 everywhere; first ROW stage at dt = 100 dt_exp, "
                       "FGMRES(30), pMG p{4-2} (nested, order gap 2), EJ smoothers, FP64, recomputed residual 1e-8")
    out["time_ratio_uniform_over_adaptive"] = out["uniform_p4"]["stage_s"] / out["p_adaptive"]["stage_s"]
    out["time_ratio_uniform_over_adaptive_128"] = out["uniform_p4_128"]["stage_s"] / out["p_adaptive_128"]["stage_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full-stage", action="store_true",
                    help="also run the oracle's complete 64x64 stage (about a minute of one host core)")
    ap.add_argument("--no-extras", action="store_true", help="the headline stage and the roofline only")
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--only-kernel", default=None, choices=["ej_apply", "ej_factor", "residual", "jvp", "stage", "step"],
                    help="profiling driver: set up the workload's state, launch one kernel family --reps times "
                         "and a 256 MiB device copy (counter calibration), print nothing else")
    ap.add_argument("--workload", default="vortical2d", choices=["vortical2d", "tgv3d", "padapt2d"],
                    help="workload of the --only-kernel driver")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--coarse-smoother", default="ej", choices=["ej", "mbnk"],
                    help="coarsest-level smoother of the --only-kernel stage driver")
    ap.add_argument("--tableau", default="esdirk3", choices=["esdirk2", "row2", "esdirk3", "row3", "esdirk4", "row4"],
                    help="time-step scheme of the --only-kernel step driver")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (N > 1 is not supported)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_09733_amd import capi

    if args.only_kernel:
        only_kernel(args)
        return
    prec = PRECISIONS[args.precision]
    wl, head = headline(args, prec)
    st = head.pop("stats")
    result = {
        "metric": "DOF/s per ESDIRK/ROW stage solve to 1e-8 rel residual",
        "value": head.pop("value"),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == capi.PREC_FP64 else "f64 (EJ factors %s)" % args.precision,
        "data": "synthetic",
        "config": {
            "workload": "3D NS FR periodic 32^3 hex, p=3 (10,485,760 DOF), Taylor-Green vortex + seeded noise, "
                        "Ma 0.1, Re 1600; first ROW stage (gamma 0.25) at dt = 100 dt_exp by FGMRES(30) with "
                        "pMG p{3-2} n{2-2} (EJ smoothers, blocks 320^2 / 135^2, FP64), stopped when the "
                        "recomputed ||R - A_h Y|| <= 1e-8 ||R|| (one-sided FD product, eps 1e-6)",
            "dof": head.pop("dof"), "setup_included": True,
        },
    }
    result.update(head)
    if not args.no_extras:
        print("[bench] 64x64 vortical stage and its variants", file=sys.stderr, flush=True)
        _, result["vortical2d"] = vortical2d_extras(args, prec)
        print("[bench] kernel rates, 3D workload", file=sys.stderr, flush=True)
        result["kernels_3d"] = kernel_rates_3d()
        print("[bench] full time steps", file=sys.stderr, flush=True)
        result["time_step"] = time_steps()
        print("[bench] p-hierarchies and the pMG nonlinear solver", file=sys.stderr, flush=True)
        result["hierarchies"] = hierarchies()
        print("[bench] p-adaptive stage", file=sys.stderr, flush=True)
        result["p_adaptive"] = padapt()
        print("[bench] coarse smoothers", file=sys.stderr, flush=True)
        result["smoothers"] = smoothers()
        print("[bench] learned coarse correction: harvest, train, A/B", file=sys.stderr, flush=True)
        from paper_2202_09733_amd import workloads as W
        result["learned_coarse"] = learned_ab(W.vortical_64x64_p4())
        print("[bench] learned coarse correction on the 32^3 mesh: harvest, train, A/B", file=sys.stderr, flush=True)
        result["learned_coarse_3d"] = learned_3d()
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline (bounded sample of the 32^3 stage)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(wl, st)
    if args.cpu_full_stage:
        print("[bench] oracle: the complete 64x64 stage", file=sys.stderr, flush=True)
        result["cpu_full_stage_vortical2d"] = cpu_full_stage_2d()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
