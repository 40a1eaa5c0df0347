"""Precision form: element-Jacobi inverses stored in FP32 inside the FP64
Krylov solve (FP64 FD JVP, FP64 orthogonalisation, FP64 stage update).  Each
result's error against the FP64 path / oracle is stated; the stage must still
reach 1e-8 in the FP64 nonlinear residual."""
import numpy as np
import pytest

from paper_2202_09733_amd import capi
from paper_2202_09733_amd import workloads as W
from gpu_util import announce, rel, require_gpu

pytestmark = pytest.mark.gpu


def test_fp32_inverse_and_solve_error(orc):
    require_gpu()
    announce("fp32 EJ storage error, vortical 8x8")
    wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    fr = capi.FR.from_workload(wl)
    sig = 2.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    dq = fr.to_dev(wl.dq)
    rng = np.random.default_rng(3)
    x = fr.to_dev(rng.standard_normal(fr.shape(0)))
    fr.ej_factor(0, dq, sig, capi.PREC_FP64)
    inv64 = fr.ej_inverse(0)
    y64 = fr.ej_solve(0, x).cpu().numpy()
    fr.ej_factor(0, dq, sig, capi.PREC_FP32)
    inv32 = fr.ej_inverse(0)
    y32 = fr.ej_solve(0, x).cpu().numpy()
    e_inv = rel(inv32, inv64)
    e_y = rel(y32, y64)
    print("fp32 storage: inverse rel err %.2e, solve rel err %.2e" % (e_inv, e_y))
    # rounding each entry to FP32 bounds the inverse error by 2^-24 entrywise
    assert e_inv <= 2 ** -24 * 1.01
    assert e_y <= 1e-5


def test_fp32_stage_converges_vortical64_full(orc):
    require_gpu()
    announce("stage vortical 64x64 with FP32 EJ storage")
    wl = W.vortical_64x64_p4()
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    q64, s64 = fr.solve_stage(capi.stage_config_for(wl, precision=capi.PREC_FP64), dq)
    q32, s32 = fr.solve_stage(capi.stage_config_for(wl, precision=capi.PREC_FP32), dq)
    assert s32["converged"] == 1 and s32["rel_res"] <= 1e-8
    q32 = q32.cpu().numpy()
    q64 = q64.cpu().numpy()
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    R0 = L0.residual(wl.dq)
    b = wl.dq + wl.a_ii * wl.dt * R0
    F = (q32 - b) / (wl.a_ii * wl.dt) - L0.residual(q32)
    assert np.linalg.norm(F) / np.linalg.norm(2 * R0) <= 1.5e-8
    e_state = np.linalg.norm(q32 - q64) / np.linalg.norm(q64 - wl.dq)
    print("fp32 vs fp64 stage: iterations %d/%d vs %d/%d; state difference %.2e of the stage update"
          % (s32["ptc_iters"], s32["gmres_iters"], s64["ptc_iters"], s64["gmres_iters"], e_state))
    assert e_state <= 1e-5


@pytest.mark.parametrize("dim", [2, 3])
def test_bf16_mfma_factor_error(orc, dim):
    """Blocked Gauss-Jordan with the panel updates on BF16 MFMA (hi/lo split,
    FP32 accumulation): the inverse against the FP64 inverse of the same
    blocks; the error is stated and bounded by the 16-bit effective mantissa
    times the block condition number."""
    require_gpu()
    announce("bf16-mfma EJ factor error dim=%d" % dim)
    if dim == 2:
        wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    else:
        wl = W.make_tgv_workload(n=(2, 2, 2))
    fr = capi.FR.from_workload(wl)
    sig = 2.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    dq = fr.to_dev(wl.dq)
    fr.ej_factor(0, dq, sig, capi.PREC_FP64)
    inv64 = fr.ej_inverse(0)
    fr.ej_factor(0, dq, sig, capi.PREC_FP32_BF16)
    invb = fr.ej_inverse(0)
    cond = max(np.linalg.cond(np.linalg.inv(inv64[k])) for k in range(0, inv64.shape[0], max(1, inv64.shape[0] // 8)))
    e = rel(invb, inv64)
    print("bf16x3-MFMA inverse: rel err %.2e (block cond up to %.1e)" % (e, cond))
    assert e <= 2.0 ** -15 * cond


def test_bf16_mfma_stage_converges_vortical64(orc):
    require_gpu()
    announce("stage vortical 64x64 with BF16-MFMA EJ factors")
    wl = W.vortical_64x64_p4()
    fr = capi.FR.from_workload(wl)
    q, st = fr.solve_stage(capi.stage_config_for(wl, precision=capi.PREC_FP32_BF16), fr.to_dev(wl.dq))
    assert st["converged"] == 1
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    R0 = L0.residual(wl.dq)
    b = wl.dq + wl.a_ii * wl.dt * R0
    qh = q.cpu().numpy()
    F = (qh - b) / (wl.a_ii * wl.dt) - L0.residual(qh)
    print("bf16-mfma factors: %d PTC / %d FGMRES, setup %.4f s" % (st["ptc_iters"], st["gmres_iters"], st["t_setup"]))
    assert np.linalg.norm(F) / np.linalg.norm(2 * R0) <= 1.5e-8


def test_bf16_storage_stage_converges_vortical64(orc):
    """EJ inverses stored in BF16 (applied with FP64 accumulation): the stage
    still reaches 1e-8 in the oracle's FP64 F; iteration counts stated."""
    require_gpu()
    announce("stage vortical 64x64 with BF16-stored EJ inverses")
    wl = W.vortical_64x64_p4()
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    sig = 2.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    fr.ej_factor(0, dq, sig, capi.PREC_FP64)
    inv64 = fr.ej_inverse(0)
    fr.ej_factor(0, dq, sig, capi.PREC_BF16_STORE)
    e = rel(fr.ej_inverse(0), inv64)
    q, st = fr.solve_stage(capi.stage_config_for(wl, precision=capi.PREC_BF16_STORE), dq)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    R0 = L0.residual(wl.dq)
    b = wl.dq + wl.a_ii * wl.dt * R0
    qh = q.cpu().numpy()
    F = (qh - b) / (wl.a_ii * wl.dt) - L0.residual(qh)
    print("bf16 storage: inverse rel err %.2e; %d PTC / %d FGMRES" % (e, st["ptc_iters"], st["gmres_iters"]))
    assert e <= 2.0 ** -8
    assert st["converged"] == 1 and np.linalg.norm(F) / np.linalg.norm(2 * R0) <= 1.5e-8
