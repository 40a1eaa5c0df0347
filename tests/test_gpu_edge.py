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
    # MBNK needs even element counts >= 4 per axis and blocks of <= 128 unknowns
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
        fr3.mbnk_factor(1, fr3.to_dev(np.zeros(fr3.shape(1))), 10.0)  # 135 unknowns per block
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
