"""Degenerate cases of the method on the GPU and the host-side argument
checks of the boundary: a stage, a time step and the preconditioner at a
steady state (R(q^n) = 0) return exact zeros without iterating; rejected
arguments raise before any kernel is launched."""
import numpy as np
import pytest

from paper_2202_09733_amd import capi
from paper_2202_09733_amd import workloads as W
from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


def _freestream(n=(8, 8), p0=2, p1=1):
    wl = W.make_bump_workload(n=n, p0=p0, p1=p1, Ma=0.1, dt_factor=10.0, seed=3)
    fr = capi.FR.from_workload(wl)
    return wl, fr, fr.to_dev(np.zeros(fr.shape(0)))


@pytest.mark.parametrize("case", ["esdirk_jfnk", "esdirk_pmg_solver", "esdirk_mbnk", "row"])
def test_stage_at_steady_state_is_exact(case):
    """F(q^n) = -2 R(q^n) = 0: converged at once, the stage state (ESDIRK) or
    increment (ROW) exactly q^n = 0."""
    require_gpu()
    announce("stage at the freestream: " + case)
    wl, fr, z = _freestream()
    kw = {"esdirk_jfnk": {}, "esdirk_pmg_solver": dict(solver=capi.SOLVER_PMG),
          "esdirk_mbnk": dict(coarse_smoother=capi.SMOOTHER_MBNK),
          "row": dict(scheme=capi.SCHEME_ROW)}[case]
    out, st = fr.solve_stage(capi.stage_config_for(wl, **kw), z)
    assert st["converged"] == 1 and st["gmres_iters"] == 0 and st["ptc_iters"] == 0
    assert not np.any(out.cpu().numpy())


@pytest.mark.parametrize("tableau", [capi.TAB_ESDIRK2, capi.TAB_ROW2, capi.TAB_ESDIRK3, capi.TAB_ROW3,
                                     capi.TAB_ESDIRK4, capi.TAB_ROW4])
def test_time_step_at_steady_state_is_exact(tableau):
    require_gpu()
    announce("time step at the freestream, tableau %d" % tableau)
    wl, fr, z = _freestream()
    out, st = fr.time_step(capi.stage_config_for(wl), z, tableau=tableau)
    assert st["gmres_iters"] == 0 and not np.any(out.cpu().numpy())


@pytest.mark.parametrize("coarse", [capi.COARSE_EJ, capi.COARSE_MBNK])
def test_preconditioner_of_zero_is_zero(coarse):
    """X = 0: every sweep sees G = 0 exactly (R(q + 0 v) reproduces R(q)
    bitwise), so Y = 0 exactly, with the scale falling back to 1."""
    require_gpu()
    announce("pmg apply of zero, coarse mode %d" % coarse)
    wl, fr, _ = _freestream()
    dq = fr.to_dev(wl.dq)
    sigA = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    sigS = 1.0 / wl.dt + sigA
    fr.ej_factor(0, dq, sigS)
    q1 = fr.restrict(0, dq)
    if coarse == capi.COARSE_MBNK:
        fr.mbnk_factor(1, q1, sigS)
    else:
        fr.ej_factor(1, q1, sigS)
    rq = fr.residual(0, dq)
    fr.pmg_set_point(dq, rq)
    y = fr.pmg_apply(fr.to_dev(np.zeros(fr.shape(0))), sigA, coarse_mode=coarse).cpu().numpy()
    assert not np.any(y)


def test_boundary_rejects_bad_arguments():
    """Host-side checks: each of these returns FR_EINVAL before launching
    anything, and the context stays usable."""
    require_gpu()
    announce("argument checks")
    # MBNK needs even element counts >= 4 per axis and blocks of <= 136 unknowns
    wl = W.make_bump_workload(n=(5, 4), p0=2, p1=1, Ma=0.1, seed=3)
    fr = capi.FR.from_workload(wl)
    with pytest.raises(capi.FRError) as ex:
        fr.mbnk_factor(1, fr.to_dev(np.zeros(fr.shape(1))), 10.0)
    assert ex.value.code == capi.FR_EINVAL
    # no factorisation yet: the MBNK calls and the MBNK coarse mode refuse
    with pytest.raises(capi.FRError):
        fr.mbnk_matvec(fr.to_dev(np.zeros(fr.shape(1))))
    wl = W.make_tgv_workload(n=(4, 4, 4), p0=3, p1=2)
    fr3 = capi.FR.from_workload(wl)
    with pytest.raises(capi.FRError) as ex:
        fr3.mbnk_factor(0, fr3.to_dev(np.zeros(fr3.shape(0))), 10.0)  # 320 unknowns per block
    assert ex.value.code == capi.FR_EINVAL
    # degree out of range
    with pytest.raises(capi.FRError):
        capi.FR(3, (2, 2, 2), [np.ones(2)] * 3, [4, 1], 1.4, 1e-3, 0.72, 0.1, W.reference_state(3, 0.1)[0])
    # GMRES iterations per MBNK sweep are capped at 8
    wl, fr, z = _freestream()
    fr.mbnk_factor(1, fr.to_dev(np.zeros(fr.shape(1))), 10.0)
    with pytest.raises(capi.FRError) as ex:
        fr.mbnk_solve(fr.to_dev(np.zeros(fr.shape(1))), maxit=9)
    assert ex.value.code == capi.FR_EINVAL
    # the context still works after the refusals
    assert not np.any(fr.mbnk_solve(fr.to_dev(np.zeros(fr.shape(1)))).cpu().numpy())


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_state_is_reported(bad):
    """A NaN or Inf in the state reaches the EJ factorisation as a non-finite
    pivot: ej_factor, the stage solve (both schemes) and the time step return
    FR_ENONFINITE, and the context still solves a finite stage afterwards."""
    require_gpu()
    announce("non-finite state (%r)" % bad)
    wl = W.make_bump_workload(n=(8, 8), p0=2, p1=1, Ma=0.1, dt_factor=10.0, seed=3)
    fr = capi.FR.from_workload(wl)
    dq = wl.dq.copy()
    dq[1, 3, 5] = bad
    d_bad = fr.to_dev(dq)
    with pytest.raises(capi.FRError) as ex:
        fr.ej_factor(0, d_bad, 10.0)
    assert ex.value.code == capi.FR_ENONFINITE
    for scheme in (capi.SCHEME_ESDIRK, capi.SCHEME_ROW):
        with pytest.raises(capi.FRError) as ex:
            fr.solve_stage(capi.stage_config_for(wl, scheme=scheme), d_bad)
        assert ex.value.code == capi.FR_ENONFINITE
    with pytest.raises(capi.FRError) as ex:
        fr.time_step(capi.stage_config_for(wl), d_bad, tableau=capi.TAB_ROW2)
    assert ex.value.code == capi.FR_ENONFINITE
    q, st = fr.solve_stage(capi.stage_config_for(wl), fr.to_dev(wl.dq))
    assert st["converged"] == 1 and np.all(np.isfinite(q.cpu().numpy()))


@pytest.mark.parametrize("p,precision", [(1, capi.PREC_FP64), (2, capi.PREC_FP64), (4, capi.PREC_FP64),
                                         (4, capi.PREC_BF16_STORE)])
def test_zero_pivot_is_reported(orc, p, precision):
    """At rest (u = 0) without viscosity or penalty and with sigma = 0, a
    density perturbation changes no flux, so every block has an exactly zero
    column (the oracle's blocks show it and its LU reports the zero pivot):
    ej_factor returns FR_ESINGULAR, in the LDS (p = 1, 2) and the blocked
    (p = 4) Gauss-Jordan."""
    require_gpu()
    announce("zero pivot p=%d precision %d" % (p, precision))
    qinf, _ = W.reference_state(2, 0.1, u_dir=(0.0, 0.0, 0.0), speed=0.0)
    h = [np.full(4, 0.25), np.full(4, 0.25)]
    L = orc.Level(dim=2, n=(4, 4), h=h, p=p, gamma=1.4, mu=0.0, Pr=0.72, tau=0.0, qinf=qinf)
    B = L.ej_blocks(np.zeros(L.shape), 0.0)
    assert np.any(np.all(B[0] == 0.0, axis=0))
    assert orc.lu_factor(B)[2] != 0
    fr = capi.FR(2, (4, 4), h, [p], 1.4, 0.0, 0.72, 0.0, qinf)
    with pytest.raises(capi.FRError) as ex:
        fr.ej_factor(0, fr.to_dev(np.zeros(L.shape)), 0.0, precision)
    assert ex.value.code == capi.FR_ESINGULAR
    # a non-zero shift makes the same blocks regular
    fr.ej_factor(0, fr.to_dev(np.zeros(L.shape)), 10.0, precision)


def test_iteration_caps_are_reported():
    """One pseudo-time step (ESDIRK), one Krylov iteration without restarts
    (ROW), one V-cycle (pMG nonlinear solver) and a time step with one
    pseudo-time step per stage: FR_ENOCONV, with the statistics of the work
    done."""
    require_gpu()
    announce("iteration caps")
    wl = W.make_bump_workload(n=(8, 8), p0=2, p1=1, Ma=0.1, dt_factor=10.0, seed=3)
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    _, st = fr.solve_stage(capi.stage_config_for(wl, max_ptc=1), dq, raise_on_noconv=False)
    assert st["rc"] == capi.FR_ENOCONV and st["converged"] == 0 and st["ptc_iters"] == 1
    _, st = fr.solve_stage(capi.stage_config_for(wl, scheme=capi.SCHEME_ROW, m=1, max_restarts=0), dq,
                           raise_on_noconv=False)
    assert st["rc"] == capi.FR_ENOCONV and st["converged"] == 0 and st["gmres_iters"] == 1
    _, st = fr.solve_stage(capi.stage_config_for(wl, solver=capi.SOLVER_PMG, max_ptc=1), dq,
                           raise_on_noconv=False)
    assert st["rc"] == capi.FR_ENOCONV and st["ptc_iters"] == 1
    _, st = fr.time_step(capi.stage_config_for(wl, max_ptc=1), dq, tableau=capi.TAB_ESDIRK2,
                         raise_on_noconv=False)
    assert st["rc"] == capi.FR_ENOCONV
    with pytest.raises(capi.FRError) as ex:
        fr.solve_stage(capi.stage_config_for(wl, max_ptc=1), dq)
    assert ex.value.code == capi.FR_ENOCONV
