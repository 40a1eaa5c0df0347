"""Benchmark: DOF/s of one implicit stage solve to 1e-8 relative nonlinear
residual on one MI355X, plus the residual/JVP/EJ kernel rates.

Workload (default): 2D Navier-Stokes FR on the 64x64 y-stretched periodic
mesh (aspect ratio 1-100), p = 4 (409,600 DOF), Ma 1e-3, one ESDIRK3 stage at
dt = 1000 dt_exp solved by PTC + JFNK + FGMRES(30) with the nonlinear pMG
p{4-2} preconditioner (n{2-2}, EJ smoothing on both levels), FP64.
One step = one full stage solve, including the per-time-step preconditioner
set-up (EJ formation and inversion on both levels) at the start.

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


def measured_traffic():
    """HBM bytes per fine-level FP64 k_ej_apply launch from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None if the kernel source has
    changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_ej_apply_vortical64.md")
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


def stage_3d(steps=1):
    """The first ROW stage of the 3D workload (32^3 hexes, p{3-2}, 10,485,760
    DOF, fine EJ blocks 320 x 320) with the preconditioner in FP64 and in the
    BF16-MFMA / BF16-storage form: DOF/s including the set-up, after one
    warm-up stage each."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
    wl = W.tgv_32cubed_p3()
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    out = {}
    for key, prec in (("fp64", capi.PREC_FP64), ("bf16_storage", capi.PREC_BF16_STORE)):
        cfg = capi.stage_config_for(wl, precision=prec)
        Y = fr.empty(0)
        fr.solve_stage(cfg, dq, out=Y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = fr.solve_stage(cfg, dq, out=Y)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        v_ap = torch.randn_like(dq)
        t_ap = _events_time(lambda: fr.ej_solve(0, v_ap, out=Y), 5)
        out[key] = {"dof_per_s": wl.dof() / el, "s_per_stage": el, "t_setup_s": st["t_setup"],
                    "t_solve_s": st["t_solve"], "gmres_iters": st["gmres_iters"], "rel_res": st["rel_res"],
                    "true_rel_res": st["true_rel_res"], "fine_ej_apply_ms": t_ap * 1e3}
    out["bf16_storage"]["speedup_vs_fp64"] = out["bf16_storage"]["dof_per_s"] / out["fp64"]["dof_per_s"]
    out["workload"] = ("3D NS FR periodic 32^3 p=3 (10,485,760 DOF) TGV, Ma 0.1, Re 1600, first ROW stage "
                       "gamma 0.25 at dt = 100 dt_exp, FGMRES(30) to 1e-8, pMG p{3-2} n{2-2}, EJ blocks 320^2 / 135^2")
    fr.close()
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


def fr_prec(fr):
    return getattr(fr, "_last_prec", 0)


def cpu_baseline(wl, st, n_sample_iters=3):
    """The oracle (plain FP64 C + numpy, one thread) on a bounded sample of
    the same stage: its preconditioner set-up run in full (EJ blocks of both
    levels by parity-coloured differencing, block LU), then the first
    n_sample_iters FGMRES iterations of the first pseudo-time step (nonlinear
    pMG preconditioner + FD JVP + Gram-Schmidt), timed; extrapolated to the
    GPU stage's PTC and FGMRES iteration counts."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t_begin = time.perf_counter()
        L0 = oracle.Level(**wl.level_kwargs(wl.p0))
        L1 = oracle.Level(**wl.level_kwargs(wl.p1))
        dq = wl.dq
        sigma_A = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
        sigma_S = 1.0 / wl.dt + sigma_A
        t0 = time.perf_counter()
        M, pm = oracle._setup_precond(L0, L1, dq, "pmg", sigma_A, sigma_A, sigma_S, {})
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        rq = L0.residual(dq)
        b = dq + (wl.a_ii * wl.dt) * rq
        F = (dq - b) / (wl.a_ii * wl.dt) - rq
        t_ptc = time.perf_counter() - t0  # one residual + stage function per pseudo-time step
        pm.set_point(dq, rq)
        A = lambda v: oracle.jvp(L0, dq, rq, v, sigma_A)
        t0 = time.perf_counter()
        _, ks = oracle.fgmres(A, M, -F, m=30, tol=1e-30, max_restarts=0, max_iters=n_sample_iters)
        t_iter = (time.perf_counter() - t0) / max(1, ks.iters)
    total = t_setup + st["ptc_iters"] * t_ptc + st["gmres_iters"] * t_iter
    dof = wl.dof()
    return dict(value=dof / total, unit="DOF/s", cores=1, kind="oracle",
                sample=("oracle run on the 64x64 vortical stage: preconditioner set-up in full (coloured EJ formation "
                        "and block LU on both levels, %.1f s) and the first %d preconditioned FGMRES iterations "
                        "(%.3f s each), one thread; extrapolated to the GPU stage's %d PTC steps and %d FGMRES "
                        "iterations = %.1f s of oracle time; measuring took %.1f s")
                % (t_setup, ks.iters, t_iter, st["ptc_iters"], st["gmres_iters"], total,
                   time.perf_counter() - t_begin),
                seconds_extrapolated=total)


def only_kernel(args):
    """Profiling driver: build the chosen workload's state, launch one kernel
    family --reps times, then a plain 256 MiB device copy whose counter
    readings calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    from paper_2202_09733_amd import capi
    from paper_2202_09733_amd import workloads as W
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the EJ-only comparison and kernel rates")
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--only-kernel", default=None, choices=["ej_apply", "ej_factor", "residual", "jvp", "stage", "step"],
                    help="profiling driver: set up the workload's state, launch one kernel family --reps times "
                         "and a 256 MiB device copy (counter calibration), print nothing else")
    ap.add_argument("--workload", default="vortical2d", choices=["vortical2d", "tgv3d"],
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
    from paper_2202_09733_amd import workloads as W

    if args.only_kernel:
        only_kernel(args)
        return
    wl = W.vortical_64x64_p4()
    fr = capi.FR.from_workload(wl)
    prec = PRECISIONS[args.precision]
    fr._last_prec = prec
    dq = fr.to_dev(wl.dq)
    cfg = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=prec)
    out = fr.empty(0)
    print("[bench] warmup %d stage solve(s)" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        _, st = fr.solve_stage(cfg, dq, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        _, st = fr.solve_stage(cfg, dq, out=out)
        stats.append(st)
        print("[bench] step %d: %.3f s (setup %.3f s), %d PTC, %d FGMRES, rel. residual %.2e"
              % (i, st["t_total"], st["t_setup"], st["ptc_iters"], st["gmres_iters"], st["rel_res"]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dof = wl.dof()
    elapsed = t1 - t0
    st = stats[-1]
    solve_only = float(np.mean([s["t_solve"] for s in stats]))
    setup = float(np.mean([s["t_setup"] for s in stats]))
    result = {
        "metric": "DOF/s per ESDIRK/ROW stage solve to 1e-8 rel residual",
        "value": dof * args.steps / elapsed,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == capi.PREC_FP64 else "f64 (EJ factors %s)" % args.precision,
        "data": "synthetic",
        "config": {
            "workload": "2D NS FR 64x64 y-stretched (AR 1-100), p=4 (409,600 DOF), Ma 1e-3, ESDIRK3 "
                        "stage at dt=1000 dt_exp, PTC+JFNK+FGMRES(30), pMG p{4-2} n{2-2} EJ smoothers",
            "dof": dof, "setup_included": True,
        },
        "stage": {
            "dof_per_s_without_setup": dof / solve_only, "t_setup_s": setup, "t_solve_s": solve_only,
            "ptc_iters": st["ptc_iters"], "gmres_iters": st["gmres_iters"],
            "gmres_per_newton": st["gmres_per_newton"], "rel_res": st["rel_res"],
            "n_R_fine": st["n_R_fine"], "n_R_coarse": st["n_R_coarse"],
            "n_ej_fine": st["n_ej_fine"], "n_ej_coarse": st["n_ej_coarse"],
        },
    }
    if not args.no_extras:
        print("[bench] plain-EJ comparison stage", file=sys.stderr, flush=True)
        cfg_ej = capi.stage_config_for(wl, precond=capi.PRECOND_EJ, precision=prec)
        _, st_ej = fr.solve_stage(cfg_ej, dq, out=fr.empty(0), raise_on_noconv=False)
        result["plain_ej"] = {k: st_ej[k] for k in ("ptc_iters", "gmres_iters", "rel_res", "t_total", "t_setup",
                                                      "converged")}
        result["plain_ej"]["dof_per_s"] = dof / st_ej["t_total"]
        # the same stage with each Arnoldi step replayed as a captured HIP graph
        print("[bench] graph-replay comparison stage", file=sys.stderr, flush=True)
        cfg_e = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=prec, graphs=1)
        fr.solve_stage(cfg_e, dq, out=fr.empty(0))
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.steps):
            _, ste = fr.solve_stage(cfg_e, dq, out=fr.empty(0))
        torch.cuda.synchronize()
        result["graph_replay"] = {"value": dof * args.steps / (time.perf_counter() - ta),
                                  "gmres_iters": ste["gmres_iters"],
                                  "note": "same stage, each Arnoldi step replayed as a captured HIP graph instead "
                                          "of host-launched kernels"}
        if prec == capi.PREC_FP64:
            for key, pv, note in [
                    ("precision_fp32_factors", capi.PREC_FP32,
                     "EJ inverses: FP64 Gauss-Jordan, stored FP32 on both levels; R, JVP, FGMRES, stage update FP64"),
                    ("precision_bf16_mfma_factors", capi.PREC_FP32_BF16,
                     "EJ inverses: blocked Gauss-Jordan with BF16-MFMA (hi/lo, FP32 accumulate) panel updates, "
                     "stored FP32; R, JVP, FGMRES, stage update FP64"),
                    ("precision_bf16_storage", capi.PREC_BF16_STORE,
                     "EJ inverses: as precision_bf16_mfma_factors, stored BF16 (FP64 accumulation in the apply); "
                     "R, JVP, FGMRES, stage update FP64")]:
                print("[bench] preconditioner variant " + key, file=sys.stderr, flush=True)
                cfgv = capi.stage_config_for(wl, precond=capi.PRECOND_PMG, precision=pv)
                fr.solve_stage(cfgv, dq, out=fr.empty(0))
                torch.cuda.synchronize()
                ta = time.perf_counter()
                stv = None
                for _ in range(args.steps):
                    _, stv = fr.solve_stage(cfgv, dq, out=fr.empty(0))
                torch.cuda.synchronize()
                vv = dof * args.steps / (time.perf_counter() - ta)
                # the fine apply with this variant's stored inverse
                v_ap = torch.randn_like(dq)
                y_ap = fr.empty(0)
                t_ap = _events_time(lambda: fr.ej_solve(0, v_ap, out=y_ap), 50)
                result[key] = {
                    "value": vv, "speedup_vs_fp64": vv / result["value"],
                    "dof_per_s_without_setup": dof / stv["t_solve"], "t_setup_s": stv["t_setup"],
                    "ptc_iters": stv["ptc_iters"], "gmres_iters": stv["gmres_iters"], "rel_res": stv["rel_res"],
                    "fine_ej_apply_us": t_ap * 1e6, "note": note}
        # re-create the pMG factors for the kernel-rate measurements
        fr.solve_stage(cfg, dq, out=out)
        print("[bench] kernel rates", file=sys.stderr, flush=True)
        rates = kernel_rates(fr, wl, dq)
        print("[bench] kernel rates, 3D workload", file=sys.stderr, flush=True)
        rates.update(kernel_rates_3d())
        print("[bench] 3D ROW stage", file=sys.stderr, flush=True)
        result["stage_3d"] = stage_3d()
        print("[bench] full time steps, ESDIRK3 and ROW3", file=sys.stderr, flush=True)
        result["time_step"] = time_steps()
        print("[bench] p-hierarchies and the pMG nonlinear solver", file=sys.stderr, flush=True)
        result["hierarchies"] = hierarchies()
        print("[bench] coarse smoothers", file=sys.stderr, flush=True)
        result["smoothers"] = smoothers()
        print("[bench] learned coarse correction: harvest, train, A/B", file=sys.stderr, flush=True)
        result["learned_coarse"] = learned_ab(wl)
        result["kernels"] = rates
        dom = rates["ej_apply_fine"]
        result["roofline"] = {
            "kernel": "k_ej_apply (fine level, n_b=100, FP64 inverse blocks)",
            "bound": "hbm", "achieved": dom["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["GBps"] / HBM_PEAK_GBS, "traffic": measured_traffic(),
        }
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(wl, st)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
