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


def _oracle_blocks(orc, wl, sig):
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    B = L0.ej_blocks(wl.dq, sig)
    return L0, B, orc.lu_factor(B)


def _oracle_inverse(B):
    """Inverses of the oracle's blocks (row-major, as FR.ej_inverse returns them)."""
    return np.stack([np.linalg.inv(b) for b in B])


def test_fp32_inverse_and_solve_error(orc):
    """FP32-stored inverses and their solve against the oracle's FP64 blocks
    (their inverse, and the oracle's LU solve).  The bar is the triangle
    inequality: FP32 rounding of each stored entry (2^-24) plus the measured
    FP64 agreement of the two sides' independently FD-formed blocks."""
    require_gpu()
    announce("fp32 EJ storage error, vortical 8x8")
    wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    fr = capi.FR.from_workload(wl)
    sig = 2.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    L0, B, fac = _oracle_blocks(orc, wl, sig)
    invO = _oracle_inverse(B)
    dq = fr.to_dev(wl.dq)
    rng = np.random.default_rng(3)
    xh = rng.standard_normal(fr.shape(0))
    x = fr.to_dev(xh)
    yO = orc.lu_solve(fac, xh)
    fr.ej_factor(0, dq, sig, capi.PREC_FP64)
    inv64 = fr.ej_inverse(0)
    y64 = fr.ej_solve(0, x).cpu().numpy()
    fr.ej_factor(0, dq, sig, capi.PREC_FP32)
    inv32 = fr.ej_inverse(0)
    y32 = fr.ej_solve(0, x).cpu().numpy()
    e64_inv, e64_y = rel(inv64, invO), rel(y64, yO)
    e32_inv, e32_y = rel(inv32, invO), rel(y32, yO)
    print("vs the oracle: FP64 inverse %.2e, solve %.2e; FP32 inverse %.2e, solve %.2e; FP32 vs GPU FP64 %.2e"
          % (e64_inv, e64_y, e32_inv, e32_y, rel(inv32, inv64)))
    # rounding each entry to FP32 bounds the storage error by 2^-24 entrywise
    assert rel(inv32, inv64) <= 2 ** -24 * 1.01
    assert e32_inv <= 2 ** -24 * 1.01 + e64_inv
    assert e32_y <= 1e-5


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
    FP32 accumulation), stored in FP32 and in BF16: the inverse and the solve
    against the oracle's FP64 blocks and LU solve.  Bars: 16 effective
    mantissa bits times the block condition number (FP32 storage), 2^-8 per
    stored entry (BF16 storage), each plus the measured FP64 agreement of the
    two sides' blocks."""
    require_gpu()
    announce("bf16-mfma EJ factor error dim=%d" % dim)
    if dim == 2:
        wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    else:
        wl = W.make_tgv_workload(n=(2, 2, 2))
    fr = capi.FR.from_workload(wl)
    sig = 2.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    L0, B, fac = _oracle_blocks(orc, wl, sig)
    invO = _oracle_inverse(B)
    dq = fr.to_dev(wl.dq)
    rng = np.random.default_rng(4)
    xh = rng.standard_normal(fr.shape(0))
    x = fr.to_dev(xh)
    yO = orc.lu_solve(fac, xh)
    fr.ej_factor(0, dq, sig, capi.PREC_FP64)
    e64 = rel(fr.ej_inverse(0), invO)
    cond = max(np.linalg.cond(B[k]) for k in range(0, B.shape[0], max(1, B.shape[0] // 8)))
    out = {}
    for prec in (capi.PREC_FP32_BF16, capi.PREC_BF16_STORE):
        fr.ej_factor(0, dq, sig, prec)
        out[prec] = (rel(fr.ej_inverse(0), invO), rel(fr.ej_solve(0, x).cpu().numpy(), yO))
    print("vs the oracle (block cond up to %.1e): FP64 inverse %.2e; BF16-MFMA/FP32 inverse %.2e, solve %.2e; "
          "BF16 storage inverse %.2e, solve %.2e" % (cond, e64, *out[capi.PREC_FP32_BF16], *out[capi.PREC_BF16_STORE]))
    assert out[capi.PREC_FP32_BF16][0] <= 2.0 ** -15 * cond + e64
    assert out[capi.PREC_BF16_STORE][0] <= 2.0 ** -8 + e64


@pytest.mark.parametrize("precision", [capi.PREC_FP64, capi.PREC_FP32, capi.PREC_FP32_BF16, capi.PREC_BF16_STORE])
def test_precision_form_pmg_apply_error(orc, precision):
    """One pmg_precond_apply output Y of each precision form against the
    oracle's FP64 V-cycle (p{4-2}, n{2-2}, both levels' EJ factors in that
    precision on the GPU): the error of the preconditioner result is stated;
    the bars (FP64 1e-6, FP32 storage 1e-4, BF16-MFMA factorisation 1e-2,
    BF16 storage 5e-2) sit above the storage precision times the largest
    block condition number, which is printed with the error."""
    require_gpu()
    announce("precision-form pmg apply, precision %d" % precision)
    wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    fr = capi.FR.from_workload(wl)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    sigA = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    sigS = 1.0 / wl.dt + sigA
    q1 = orc.restrict(wl.dq, 2, wl.p0 + 1, wl.p1 + 1)
    pm = orc.PMG(L0, L1, orc.lu_factor(L0.ej_blocks(wl.dq, sigS)), orc.lu_factor(L1.ej_blocks(q1, sigS)),
                 orc.PMGParams(sigma_D=sigA))
    rq = L0.residual(wl.dq)
    pm.set_point(wl.dq, rq)
    rng = np.random.default_rng(5)
    X = rng.standard_normal(L0.shape)
    X /= np.linalg.norm(X)
    Y_ref = pm.apply(X)
    d_q = fr.to_dev(wl.dq)
    fr.ej_factor(0, d_q, sigS, precision)
    fr.ej_factor(1, fr.to_dev(q1), sigS, precision)
    fr.pmg_set_point(d_q, fr.to_dev(rq))
    Y = fr.pmg_apply(fr.to_dev(X), sigA).cpu().numpy()
    e = rel(Y, Y_ref)
    B0 = L0.ej_blocks(wl.dq, sigS)
    cond = max(np.linalg.cond(B0[k]) for k in range(0, B0.shape[0], 8))
    print("precision %d: pmg_precond_apply vs the FP64 oracle %.2e (fine block cond up to %.1e)"
          % (precision, e, cond))
    bar = {capi.PREC_FP64: 1e-6, capi.PREC_FP32: 1e-4, capi.PREC_FP32_BF16: 1e-2,
           capi.PREC_BF16_STORE: 5e-2}[precision]
    assert e <= bar


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
