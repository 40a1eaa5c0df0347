"""Multi-level pMG on the GPU: the three-level FAS V-cycle against the
oracle's (oracle/multilevel.py), stage solves with p{4-2-1}, and pMG as the
standalone nonlinear stage solver against the oracle's, with hierarchies
down to p = 0 (p{3-1-0}, p{3-2-1-0})."""
import numpy as np
import pytest

from paper_2202_09733_amd import capi
from paper_2202_09733_amd import workloads as W
from gpu_util import announce, rel, require_gpu

pytestmark = pytest.mark.gpu


def test_pmg_apply_three_levels_parity(orc):
    require_gpu()
    announce("pmg apply p{4-2-1}")
    from oracle import multilevel as ML
    wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    ps = (4, 2, 1)
    fr = capi.FR.from_workload(wl, levels=list(ps))
    levels = [orc.Level(**wl.level_kwargs(p)) for p in ps]
    sigA = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    sigS = 1.0 / wl.dt + sigA
    facs = ML.hierarchy_factors(levels, wl.dq, sigS)
    n = (2, 3, 4)
    pm = ML.MultiPMG(levels, facs, ML.MultiPMGParams(sigma_D=sigA, n=n))
    rq = levels[0].residual(wl.dq)
    pm.set_point(wl.dq, rq)
    rng = np.random.default_rng(6)
    X = rng.standard_normal(levels[0].shape)
    X /= np.linalg.norm(X)
    Y_ref = pm.apply(X)
    q1 = orc.restrict(wl.dq, 2, 5, 3)
    q2 = orc.restrict(q1, 2, 3, 2)
    fr.ej_factor(0, fr.to_dev(wl.dq), sigS)
    fr.ej_factor(1, fr.to_dev(q1), sigS)
    fr.ej_factor(2, fr.to_dev(q2), sigS)
    fr.pmg_set_point(fr.to_dev(wl.dq), fr.to_dev(rq))
    Y = fr.pmg_apply(fr.to_dev(X), sigA, n0=n[0], n1=n[1], n2=n[2]).cpu().numpy()
    e3 = rel(Y, Y_ref)
    # the two-level cycle of the same context equals the two-level oracle
    pm2 = orc.PMG(levels[0], levels[1], facs[0], facs[1], orc.PMGParams(sigma_D=sigA, n0=2, n1=3))
    pm2.set_point(wl.dq, rq)
    Y2 = fr.pmg_apply(fr.to_dev(X), sigA, n0=2, n1=3, levels=2).cpu().numpy()
    e2 = rel(Y2, pm2.apply(X))
    print("p{4-2-1} cycle vs oracle %.2e; p{4-2} cycle of the same context vs oracle %.2e; "
          "three- vs two-level difference %.2e" % (e3, e2, rel(Y, Y2)))
    # independently FD-formed blocks on each side (see the EJ bar)
    assert e3 <= 1e-6 and e2 <= 1e-6
    assert rel(Y, Y2) > 1e-4  # the third level changes the cycle


def test_stage_three_levels_vortical64(orc):
    """The 64x64 vortical stage with the p{4-2-1} preconditioner reaches 1e-8 in the
    oracle's F."""
    require_gpu()
    announce("stage vortical 64x64 p{4-2-1}")
    wl = W.vortical_64x64_p4()
    fr = capi.FR.from_workload(wl, levels=[4, 2, 1])
    q, st = fr.solve_stage(capi.stage_config_for(wl), fr.to_dev(wl.dq))
    q2, st2 = fr.solve_stage(capi.stage_config_for(wl, pmg_levels=2), fr.to_dev(wl.dq))
    print("vortical 64x64: p{4-2-1} %d PTC / %d FGMRES (%.3f s); p{4-2} %d / %d (%.3f s)"
          % (st["ptc_iters"], st["gmres_iters"], st["t_total"], st2["ptc_iters"], st2["gmres_iters"],
             st2["t_total"]))
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    R0 = L0.residual(wl.dq)
    b = wl.dq + wl.a_ii * wl.dt * R0
    qh = q.cpu().numpy()
    F = (qh - b) / (wl.a_ii * wl.dt) - L0.residual(qh)
    assert st["converged"] == 1 and np.linalg.norm(F) / np.linalg.norm(2 * R0) <= 1.5e-8


@pytest.mark.parametrize("ps", [(2, 1), (3, 2, 1), (3, 1, 0), (3, 2, 1, 0)])
def test_pmg_nonlinear_solver_parity(orc, ps):
    require_gpu()
    announce("pMG nonlinear solver p%s" % (ps,))
    from oracle import multilevel as ML
    wl = W.make_bump_workload(n=(8, 8), p0=ps[0], p1=ps[1], dt_factor=3.0)
    fr = capi.FR.from_workload(wl, levels=list(ps))
    n = tuple([2] * (len(ps) - 1) + [4])
    cfg = capi.stage_config_for(wl, solver=capi.SOLVER_PMG, tol=1e-10, max_ptc=200, n0=n[0], n1=n[1],
                                n2=n[2] if len(n) > 2 else 2, n3=n[3] if len(n) > 3 else 2)
    q, st = fr.solve_stage(cfg, fr.to_dev(wl.dq))
    levels = [orc.Level(**wl.level_kwargs(p)) for p in ps]
    q_ref, so = ML.pmg_nonlinear_stage(levels, wl.dq, wl.dt, wl.a_ii, n=n, tol=1e-10, max_vcycles=200)
    upd = np.linalg.norm(q_ref - wl.dq)
    d = np.linalg.norm(q.cpu().numpy() - q_ref) / upd
    print("pMG nonlinear solver p%s: GPU %d V-cycles, oracle %d; |q - q_ref| / |update| = %.2e"
          % (ps, st["ptc_iters"], so.vcycles, d))
    assert st["converged"] == 1 and so.converged and st["gmres_iters"] == 0
    assert abs(st["ptc_iters"] - so.vcycles) <= 1
    assert d <= 1e-8


def test_pmg_nonlinear_solver_refresh_parity(orc):
    """Smoothers re-formed at the current iterate every 3 V-cycles, against
    the oracle's same schedule."""
    require_gpu()
    announce("pMG nonlinear solver with smoother refresh")
    from oracle import multilevel as ML
    wl = W.make_bump_workload(n=(8, 8), p0=3, p1=1, dt_factor=3.0)
    ps = (3, 1)
    fr = capi.FR.from_workload(wl, levels=list(ps))
    cfg = capi.stage_config_for(wl, solver=capi.SOLVER_PMG, tol=1e-10, max_ptc=200, n0=2, n1=4,
                                smoother_refresh=3)
    q, st = fr.solve_stage(cfg, fr.to_dev(wl.dq))
    levels = [orc.Level(**wl.level_kwargs(p)) for p in ps]
    q_ref, so = ML.pmg_nonlinear_stage(levels, wl.dq, wl.dt, wl.a_ii, n=(2, 4), tol=1e-10, max_vcycles=200,
                                       refresh=3)
    q0, s0 = ML.pmg_nonlinear_stage(levels, wl.dq, wl.dt, wl.a_ii, n=(2, 4), tol=1e-10, max_vcycles=200)
    d = np.linalg.norm(q.cpu().numpy() - q_ref) / np.linalg.norm(q_ref - wl.dq)
    print("refresh every 3: GPU %d V-cycles, oracle %d (without refresh %d); |q - q_ref| / |update| = %.2e"
          % (st["ptc_iters"], so.vcycles, s0.vcycles, d))
    assert st["converged"] == 1 and so.converged
    assert abs(st["ptc_iters"] - so.vcycles) <= 1
    assert d <= 1e-8
