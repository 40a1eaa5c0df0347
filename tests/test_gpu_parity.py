"""GPU parity: every ABI call of the HIP library against the FP64 CPU oracle
on the same seeded inputs.  Sizes span several workgroup tiles with ragged
tails; the 8x8 bump and 64x64 vortical meshes are also checked at full size.

Bars (normwise relative error unless stated):
  * residual R: 1e-10 (both sides FP64, deviation form, no cancellation
    against p_inf);
  * JVP: 1e-10 when the step changes R by much more than its rounding; at the
    production step eps = 1e-6 the bar is derived from the measured R
    difference d_R: 10 * 2 d_R ||R|| / ||R(q + h v) - R(q)||, the rounding of
    the two residuals amplified by the finite difference;
  * EJ blocks (FD of R with step 1e-7 max(1, |q|)): the same derivation with
    the block step;
  * transfers: 1e-14.
"""
import numpy as np
import pytest

from paper_2202_09733_amd import capi
from paper_2202_09733_amd import workloads as W
from gpu_util import announce, rel, require_gpu

pytestmark = pytest.mark.gpu

U = 2.2e-16


def _mesh(dim, n, levels, Ma, seed, stretch=False):
    rng = np.random.default_rng(seed)
    if stretch:
        h = [rng.uniform(0.01, 0.2, n[a]) for a in range(dim)]
    else:
        h = [np.full(n[a], 1.0 / n[a]) for a in range(dim)]
    qinf, _ = W.reference_state(dim, Ma, u_dir=(0.8, 0.6, 0.0))
    return dict(dim=dim, n=n, h=h, gamma=1.4, mu=2e-3, Pr=0.72, tau=0.1, qinf=qinf), rng


def _pair(orc, spec, levels):
    fr = capi.FR(spec["dim"], spec["n"], spec["h"], levels, spec["gamma"], spec["mu"], spec["Pr"], spec["tau"],
                 spec["qinf"])
    ol = [orc.Level(p=p, **spec) for p in levels]
    return fr, ol


RES_CASES = [
    (2, (12, 10), 1, 0.3), (2, (8, 6), 2, 1e-3), (2, (6, 4), 3, 0.1), (2, (6, 4), 4, 1e-3),
    (3, (4, 4, 2), 2, 0.1), (3, (3, 2, 2), 3, 0.3), (3, (2, 2, 2), 1, 0.2),
    (2, (12, 10), 0, 0.3), (3, (3, 4, 2), 0, 0.1),
]


@pytest.mark.parametrize("dim,n,p,Ma", RES_CASES)
def test_residual_parity(orc, dim, n, p, Ma):
    require_gpu()
    announce("residual dim=%d n=%s p=%d Ma=%g" % (dim, n, p, Ma))
    spec, rng = _mesh(dim, n, [p], Ma, seed=100 + p, stretch=True)
    fr, (ol,) = _pair(orc, spec, [p])
    dq = W.random_state(ol.shape, rng, spec["qinf"], amp=0.02)
    r_ref = ol.residual(dq)
    r = fr.residual(0, fr.to_dev(dq)).cpu().numpy()
    assert rel(r, r_ref) <= 1e-10
    # freestream: exactly zero
    z = fr.residual(0, fr.to_dev(np.zeros(ol.shape))).cpu().numpy()
    assert np.all(z == 0.0)
    # run-to-run bitwise reproducible
    r2 = fr.residual(0, fr.to_dev(dq)).cpu().numpy()
    assert np.array_equal(r, r2)


@pytest.mark.parametrize("which", ["bumps_8x8_p2", "vortical_64x64_p4"])
def test_residual_parity_full_size(orc, which):
    require_gpu()
    announce("residual full size " + which)
    wl = getattr(W, which)()
    fr = capi.FR.from_workload(wl)
    ol = orc.Level(**wl.level_kwargs(wl.p0))
    r_ref = ol.residual(wl.dq)
    r = fr.residual(0, fr.to_dev(wl.dq)).cpu().numpy()
    assert rel(r, r_ref) <= 1e-10
    # coarse level at the restricted state
    ol1 = orc.Level(**wl.level_kwargs(wl.p1))
    q1 = orc.restrict(wl.dq, wl.dim, wl.p0 + 1, wl.p1 + 1)
    r1 = fr.residual(1, fr.to_dev(q1)).cpu().numpy()
    assert rel(r1, ol1.residual(q1)) <= 1e-10


def test_residual_sampled_3d_config(orc):
    """3D 32^3 p=3 Taylor-Green state: full-size GPU residual; the oracle's
    residual is evaluated on the same state and compared on every entry."""
    require_gpu()
    announce("residual full size TGV 32^3 p=3")
    wl = W.tgv_32cubed_p3()
    fr = capi.FR.from_workload(wl)
    ol = orc.Level(**wl.level_kwargs(wl.p0))
    r = fr.residual(0, fr.to_dev(wl.dq)).cpu().numpy()
    r_ref = ol.residual(wl.dq)
    assert rel(r, r_ref) <= 1e-10


@pytest.mark.parametrize("dim,n,p0,p1", [(2, (6, 4), 4, 2), (2, (8, 6), 2, 1), (3, (4, 2, 2), 3, 2), (2, (6, 4), 3, 0),
                                          (3, (4, 2, 2), 1, 0)])
def test_transfer_parity(orc, dim, n, p0, p1):
    require_gpu()
    announce("transfer dim=%d p%d->p%d" % (dim, p0, p1))
    spec, rng = _mesh(dim, n, [p0, p1], 0.2, seed=7)
    fr, (o0, o1) = _pair(orc, spec, [p0, p1])
    x = rng.standard_normal(o0.shape)
    y = fr.restrict(0, fr.to_dev(x)).cpu().numpy()
    assert rel(y, orc.restrict(x, dim, p0 + 1, p1 + 1)) <= 1e-14
    z = rng.standard_normal(o1.shape)
    w = fr.prolong(1, fr.to_dev(z)).cpu().numpy()
    assert rel(w, orc.prolong(z, dim, p0 + 1, p1 + 1)) <= 1e-14


@pytest.mark.parametrize("dim,n,p,Ma", [(2, (6, 4), 4, 1e-3), (2, (8, 6), 2, 0.1), (3, (3, 2, 2), 3, 0.2),
                                        (2, (8, 6), 0, 0.1)])
def test_jvp_parity(orc, dim, n, p, Ma):
    require_gpu()
    announce("jvp dim=%d p=%d Ma=%g" % (dim, p, Ma))
    spec, rng = _mesh(dim, n, [p], Ma, seed=200 + p, stretch=True)
    fr, (ol,) = _pair(orc, spec, [p])
    dq = W.random_state(ol.shape, rng, spec["qinf"], amp=0.02)
    v = rng.standard_normal(ol.shape)
    v /= np.linalg.norm(v)
    rq = ol.residual(dq)
    d_q, d_rq, d_v = fr.to_dev(dq), fr.to_dev(rq), fr.to_dev(v)
    r_gpu = fr.residual(0, d_q).cpu().numpy()
    dR = rel(r_gpu, rq)
    sigma = 123.0
    for eps, mode, central in [(1e-2, capi.EPS_ABSOLUTE, False), (1e-6, capi.EPS_NORMALIZED, False),
                               (1e-6, capi.EPS_SCALED, False), (1e-2, capi.EPS_ABSOLUTE, True),
                               (1e-6, capi.EPS_SCALED, True)]:
        w_ref = orc.jvp(ol, dq, rq, v, sigma, eps=eps, mode=mode, central=central)
        gmode = mode | (capi.FD_CENTRAL if central else 0)
        w = fr.jvp(0, d_q, d_rq, d_v, sigma, eps=eps, eps_mode=gmode).cpu().numpy()
        h = orc.fd_step(v, eps, mode, dq)
        # the difference of the two residuals the product divides (norm), and
        # the rounding of each, amplified by that division
        dRv = h * np.linalg.norm(sigma * v - w_ref) * (2.0 if central else 1.0)
        bar = max(1e-10, 10 * 2 * max(dR, U) * np.linalg.norm(rq) / dRv)
        assert rel(w, w_ref) <= bar, (eps, central, rel(w, w_ref), bar)


@pytest.mark.parametrize("which", ["vortical_64x64_p4", "tgv_32cubed_p3"])
def test_jvp_parity_full_size(orc, which):
    """The production FD JVP (SCALED step, eps = 1e-6) at full size, 409,600
    and 10,485,760 unknowns, element by element against the oracle on the
    same state and direction: normwise bar as in test_jvp_parity, and the
    largest entry error relative to the largest entry."""
    require_gpu()
    announce("jvp full size " + which)
    wl = getattr(W, which)()
    fr = capi.FR.from_workload(wl)
    ol = orc.Level(**wl.level_kwargs(wl.p0))
    rng = np.random.default_rng(77)
    v = rng.standard_normal(ol.shape)
    v /= np.linalg.norm(v)
    rq = ol.residual(wl.dq)
    sigma = 1.0 / (wl.a_ii * wl.dt)
    w_ref = orc.jvp(ol, wl.dq, rq, v, sigma, eps=1e-6, mode=orc.EPS_SCALED)
    d_q = fr.to_dev(wl.dq)
    dR = rel(fr.residual(0, d_q).cpu().numpy(), rq)
    w = fr.jvp(0, d_q, fr.to_dev(rq), fr.to_dev(v), sigma, eps=1e-6, eps_mode=capi.EPS_SCALED).cpu().numpy()
    h = orc.fd_step(v, 1e-6, orc.EPS_SCALED, wl.dq)
    dRv = h * np.linalg.norm(sigma * v - w_ref)   # ||R(q + h v) - R(q)||
    bar = max(1e-10, 10 * 2 * max(dR, U) * np.linalg.norm(rq) / dRv)
    e = rel(w, w_ref)
    e_max = np.abs(w - w_ref).max() / np.abs(w_ref).max()
    print("%s: JVP rel err %.2e (bar %.2e), max entry err %.2e of max |w|; residual rel err %.2e"
          % (which, e, bar, e_max, dR))
    assert e <= bar and e_max <= 10 * bar


@pytest.mark.parametrize("dim,n,p,sigma", [(2, (4, 4), 2, 50.0), (2, (4, 2), 4, 5e3), (3, (2, 2, 2), 2, 20.0),
                                           (3, (2, 2, 2), 3, 40.0), (2, (6, 4), 0, 30.0), (3, (2, 2, 2), 0, 20.0)])
def test_ej_blocks_and_solve_parity(orc, dim, n, p, sigma):
    require_gpu()
    announce("ej dim=%d p=%d" % (dim, p))
    spec, rng = _mesh(dim, n, [p], 0.1, seed=300 + p, stretch=True)
    fr, (ol,) = _pair(orc, spec, [p])
    dq = W.random_state(ol.shape, rng, spec["qinf"], amp=0.02)
    B = ol.ej_blocks(dq, sigma)
    fr.ej_factor(0, fr.to_dev(dq), sigma, capi.PREC_FP64)
    Binv = fr.ej_inverse(0)
    # rounding of R amplified by the block step 1e-7 max(1, |q|)
    rq = ol.residual(dq)
    dR = rel(fr.residual(0, fr.to_dev(dq)).cpu().numpy(), rq)
    hmin = 1e-7
    bar_blk = max(1e-10, 10 * 2 * max(dR, U) * np.abs(rq).max() / hmin / np.abs(B).max())
    for k in range(ol.Ne):
        Bk_gpu = np.linalg.inv(Binv[k])
        assert rel(Bk_gpu, B[k]) <= bar_blk + 1e-12 * np.linalg.cond(B[k])
    fac = orc.lu_factor(B)
    x = rng.standard_normal(ol.shape)
    y_ref = orc.lu_solve(fac, x)
    y = fr.ej_solve(0, fr.to_dev(x)).cpu().numpy()
    cond = max(np.linalg.cond(B[k]) for k in range(ol.Ne))
    assert rel(y, y_ref) <= (bar_blk + 1e-14) * cond * 10


def test_ej_solve_is_exact_inverse_of_gpu_blocks(orc):
    """The stored inverse times the (GPU-formed) block is the identity."""
    require_gpu()
    spec, rng = _mesh(2, (4, 4), [3], 0.1, seed=17)
    fr, (ol,) = _pair(orc, spec, [3])
    dq = W.random_state(ol.shape, rng, spec["qinf"], amp=0.02)
    fr.ej_factor(0, fr.to_dev(dq), 80.0, capi.PREC_FP64)
    Binv = fr.ej_inverse(0)
    B = ol.ej_blocks(dq, 80.0)
    for k in range(ol.Ne):
        E = Binv[k] @ B[k] - np.eye(ol.nb)
        assert np.abs(E).max() < 1e-6


def test_pmg_apply_parity(orc):
    require_gpu()
    announce("pmg apply p{4-2}")
    wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    fr = capi.FR.from_workload(wl)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    sigA = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    sigS = 1.0 / wl.dt + sigA
    fac0 = orc.lu_factor(L0.ej_blocks(wl.dq, sigS))
    q1 = orc.restrict(wl.dq, 2, 5, 3)
    fac1 = orc.lu_factor(L1.ej_blocks(q1, sigS))
    pm = orc.PMG(L0, L1, fac0, fac1, orc.PMGParams(sigma_D=sigA))
    rq = L0.residual(wl.dq)
    pm.set_point(wl.dq, rq)
    rng = np.random.default_rng(5)
    X = rng.standard_normal(L0.shape)
    X /= np.linalg.norm(X)
    Y_ref = pm.apply(X)
    d_q = fr.to_dev(wl.dq)
    fr.ej_factor(0, d_q, sigS)
    fr.ej_factor(1, fr.to_dev(q1), sigS)
    d_rq = fr.to_dev(rq)
    fr.pmg_set_point(d_q, d_rq)
    Y = fr.pmg_apply(fr.to_dev(X), sigA).cpu().numpy()
    # the two sides use independently FD-formed blocks (see the EJ bar)
    assert rel(Y, Y_ref) <= 1e-6
    # one sweep, no coarse level: exactly the EJ solve with the same factors
    Y1 = fr.pmg_apply(fr.to_dev(X), sigA, n0=1, coarse_mode=capi.COARSE_NONE,
                      scale_mode=capi.SCALE_LITERAL).cpu().numpy()
    Y1e = fr.ej_solve(0, fr.to_dev(X)).cpu().numpy()
    assert np.array_equal(Y1, Y1e)


def _oracle_F(orc, wl, q):
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    R0 = L0.residual(wl.dq)
    b = wl.dq + wl.a_ii * wl.dt * R0
    F0 = -2 * R0
    F = (q - b) / (wl.a_ii * wl.dt) - L0.residual(q)
    return np.linalg.norm(F) / np.linalg.norm(F0)


@pytest.mark.parametrize("precond", [capi.PRECOND_PMG, capi.PRECOND_EJ])
def test_stage_bumps8_matches_oracle(orc, precond):
    require_gpu()
    announce("stage bumps 8x8 precond=%d" % precond)
    wl = W.bumps_8x8_p2()
    fr = capi.FR.from_workload(wl)
    cfg = capi.stage_config_for(wl, precond=precond)
    q, st = fr.solve_stage(cfg, fr.to_dev(wl.dq))
    q = q.cpu().numpy()
    assert st["converged"] == 1 and st["rel_res"] <= 1e-8
    # the oracle's own F at the GPU state meets the tolerance
    assert _oracle_F(orc, wl, q) <= 1.5e-8
    # and the oracle's stage solve converges to the same state
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    q_ref, so = orc.esdirk_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, precond="pmg" if precond else "ej",
                                 eta=cfg.eta)
    assert so.converged
    assert np.linalg.norm(q - q_ref) <= 1e-6 * np.linalg.norm(q_ref - wl.dq)
    print("gpu ptc/gmres", st["ptc_iters"], st["gmres_iters"], "oracle", so.ptc_iters, so.gmres_iters)


def test_stage_vortical64_full_size(orc):
    """Full 64x64 vortical stage on the GPU (pMG p{4-2}); the oracle's residual at
    the GPU's final state confirms ||F|| <= 1e-8 ||F(q^n)||."""
    require_gpu()
    announce("stage vortical 64x64 full size pMG")
    wl = W.vortical_64x64_p4()
    fr = capi.FR.from_workload(wl)
    q, st = fr.solve_stage(capi.stage_config_for(wl), fr.to_dev(wl.dq))
    print(st)
    assert st["converged"] == 1
    assert _oracle_F(orc, wl, q.cpu().numpy()) <= 1.5e-8
    # per-phase times of the Arnoldi steps (HIP events) fit inside the solve
    phases = st["t_precond"] + st["t_jvp"] + st["t_ortho"]
    print("phases: preconditioner %.4f s, FD product %.4f s, orthogonalisation %.4f s of %.4f s"
          % (st["t_precond"], st["t_jvp"], st["t_ortho"], st["t_solve"]))
    assert min(st["t_precond"], st["t_jvp"], st["t_ortho"]) > 0 and phases <= st["t_solve"]


@pytest.mark.parametrize("tol,verify", [(1e-10, 0), (1e-8, 1)])
def test_row_stage_tiny_matches_oracle(orc, tol, verify):
    """A ROW stage stopped on the Krylov estimate at 1e-10 (below the
    recomputed residual's rounding floor on this mesh), and on the
    recomputed residual at 1e-8: GPU against the oracle."""
    require_gpu()
    announce("row stage tiny, tol %g, verify %d" % (tol, verify))
    wl = W.make_bump_workload(n=(4, 4), p0=2, p1=1, Ma=0.2, dt_factor=10.0, seed=13, scheme="row", amp=5e-2)
    fr = capi.FR.from_workload(wl)
    Y, st = fr.solve_stage(capi.stage_config_for(wl, tol=tol, verify=verify), fr.to_dev(wl.dq))
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    Y_ref, so = orc.row_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, tol=tol, verify=bool(verify))
    assert st["converged"] == 1 and so.converged
    if verify:
        assert st["true_rel_res"] <= tol
    e = rel(Y.cpu().numpy(), Y_ref)
    print("row stage tiny: GPU %d FGMRES, oracle %d; rel. difference %.2e" % (st["gmres_iters"], so.gmres_iters, e))
    assert e <= (1e-7 if not verify else 1e-6)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_row_stage_short_cycles_matches_oracle(orc, m):
    """FGMRES(m) with m = 2, 3, 5: many restarts, so cycles end both on
    the basis limit and on convergence right after a step launched ahead of
    the host's check.  The GPU takes the oracle's restart count and
    solution."""
    require_gpu()
    announce("row stage tiny, m %d" % m)
    wl = W.make_bump_workload(n=(4, 4), p0=2, p1=1, Ma=0.2, dt_factor=10.0, seed=13, scheme="row", amp=5e-2)
    fr = capi.FR.from_workload(wl)
    Y, st = fr.solve_stage(capi.stage_config_for(wl, tol=1e-8, verify=1, m=m, max_restarts=200),
                           fr.to_dev(wl.dq))
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    Y_ref, so = orc.row_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, m=m, max_restarts=200, tol=1e-8, verify=True)
    assert st["converged"] == 1 and so.converged
    assert st["true_rel_res"] <= 1e-8
    e = rel(Y.cpu().numpy(), Y_ref)
    print("m %d: GPU %d FGMRES / %d restarts, oracle %d; rel. difference %.2e"
          % (m, st["gmres_iters"], st["restarts"], so.gmres_iters, e))
    assert abs(st["gmres_iters"] - so.gmres_iters) <= 1
    assert e <= 1e-6


@pytest.fixture(scope="module")
def tgv32_oracle_rhs(orc):
    wl = W.tgv_32cubed_p3()
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    return wl, L0, L0.residual(wl.dq)


@pytest.mark.parametrize("precision", [capi.PREC_FP64, capi.PREC_FP32, capi.PREC_BF16_STORE])
@pytest.mark.parametrize("central", [False, True])
def test_row_stage_tgv32_full_size(orc, tgv32_oracle_rhs, precision, central):
    """3D 32^3 p=3 first ROW stage with pMG p{3-2} (fine blocks 320 x 320,
    blocked Gauss-Jordan) with the EJ inverses in FP64, FP32, or from the
    BF16-MFMA factorisation stored in BF16, and the one-sided (the paper's)
    or the central FD product.  The stage is solved when the residual of the
    FD operator recomputed at the solution, ||R - A_h Y||, meets 1e-8 of ||R||
    (the FD operator is linear only to its truncation error, ~1e-7 relative
    here, so the Krylov estimate alone stops early and FGMRES continues from
    the recomputed residual); the oracle recomputes it at the GPU solution."""
    require_gpu()
    announce("row stage TGV 32^3 full size, precision %d, central %d" % (precision, central))
    wl, L0, R0 = tgv32_oracle_rhs
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    mode = capi.EPS_SCALED | (capi.FD_CENTRAL if central else 0)
    Y, st = fr.solve_stage(capi.stage_config_for(wl, precision=precision, eps_mode=mode), dq)
    print({k: st[k] for k in ("gmres_iters", "restarts", "rel_res", "true_rel_res", "t_setup", "t_solve")})
    assert st["converged"] == 1 and st["true_rel_res"] <= 1e-8
    Y = Y.cpu().numpy()
    fr.close()
    sigma = 1.0 / (wl.a_ii * wl.dt)
    AY = orc.jvp(L0, wl.dq, R0, Y, sigma, eps=1e-6, mode=orc.EPS_SCALED, central=central)
    true_orc = np.linalg.norm(R0 - AY) / np.linalg.norm(R0)
    print("oracle FD residual at the GPU solution %.3e, GPU %.3e" % (true_orc, st["true_rel_res"]))
    assert true_orc <= 1.1e-8
    assert abs(true_orc - st["true_rel_res"]) <= 0.1 * true_orc


@pytest.mark.parametrize("case", ["esdirk_vortical64", "row_3d"])
def test_graph_replay_matches_eager(orc, case):
    """Arnoldi steps captured as HIP graphs and replayed (many replays per
    stage, with host synchronisations and host-launched work between them,
    over two consecutive stage solves that reuse the cached graphs) give
    bitwise the same stage, iteration counts and operation counts as the
    host-launched kernels."""
    require_gpu()
    announce("graph replay vs eager: %s" % case)
    if case == "esdirk_vortical64":
        wl = W.vortical_64x64_p4()
    else:
        wl = W.make_tgv_workload(n=(8, 8, 8))
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    q_e, s_e = fr.solve_stage(capi.stage_config_for(wl), dq)
    q_e = q_e.cpu().numpy()
    for rep in range(2):
        q_g, s_g = fr.solve_stage(capi.stage_config_for(wl, graphs=1), dq)
        assert np.array_equal(q_g.cpu().numpy(), q_e), rep
        for k in ("ptc_iters", "gmres_iters", "n_R_fine", "n_R_coarse", "n_ej_fine", "n_ej_coarse"):
            assert s_g[k] == s_e[k], (rep, k, s_g[k], s_e[k])
    print("%s: %d FGMRES iterations; eager %.4f s, graphs %.4f s (solve part)" % (
        case, s_g["gmres_iters"], s_e["t_solve"], s_g["t_solve"]))
