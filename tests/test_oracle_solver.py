"""Pins of the oracle's Jacobian-vector product, element-Jacobi blocks, block
LU, flexible GMRES, nonlinear p-multigrid preconditioner and stage solves,
against dense linear algebra on tiny meshes (numpy/scipy), brute-force
Jacobians and closed forms."""
import numpy as np
import pytest
import scipy.linalg

from paper_2202_09733_amd import workloads as W


def _tiny(orc, dim=2, n=(4, 4), p=1, Ma=0.3, seed=0, amp=0.05):
    qinf, _ = W.reference_state(dim, Ma, u_dir=(0.8, 0.6, 0.0))
    rng = np.random.default_rng(seed)
    h = [rng.uniform(0.1, 0.3, n[a]) for a in range(dim)]
    L = orc.Level(dim=dim, n=n, h=h, p=p, gamma=1.4, mu=1e-2, Pr=0.72, tau=0.1, qinf=qinf)
    dq = W.random_state(L.shape, rng, qinf, amp=amp)
    return L, dq, rng


def dense_jacobian(L, dq, rel=1e-6):
    """Central-difference Jacobian of R, one column per DOF."""
    N = L.N
    J = np.zeros((N, N))
    x = dq.reshape(-1)
    for j in range(N):
        h = rel * max(1.0, abs(x[j]))
        e = np.zeros(N)
        e[j] = h
        J[:, j] = (L.residual((x + e).reshape(L.shape)) - L.residual((x - e).reshape(L.shape))).reshape(-1) / (2 * h)
    return J


@pytest.fixture(scope="module")
def tiny2d(orc):
    L, dq, rng = _tiny(orc)
    return L, dq, dense_jacobian(L, dq)


def test_jvp_matches_dense_jacobian(orc, tiny2d):
    L, dq, J = tiny2d
    rq = L.residual(dq)
    v = np.random.default_rng(1).standard_normal(L.shape)
    sigma = 3.7
    ref = sigma * v.reshape(-1) - J @ v.reshape(-1)
    errs = []
    for eps in [1e-4, 1e-5, 1e-6]:
        w = orc.jvp(L, dq, rq, v, sigma, eps=eps, mode=orc.EPS_NORMALIZED)
        errs.append(np.linalg.norm(w.reshape(-1) - ref) / np.linalg.norm(ref))
    # one-sided difference: error O(h), falling with eps until rounding
    assert errs[0] < 1e-4 and errs[1] < errs[0] and errs[2] < 1e-6


def _ej_blocks_naive(L, dq, sigma):
    """Per element and per column, exactly as the definition states."""
    r0 = L.residual(dq)
    B = np.zeros((L.Ne, L.nb, L.nb))
    for k in range(L.Ne):
        for j in range(L.nb):
            jv, ji = divmod(j, L.Np)
            qp = dq.copy()
            hj = 1e-7 * max(1.0, abs(L.qinf[jv] + dq[jv, ji, k]))
            qp[jv, ji, k] = dq[jv, ji, k] + hj
            ha = qp[jv, ji, k] - dq[jv, ji, k]
            rp = L.residual(qp)
            col = -(rp[:, :, k] - r0[:, :, k]).reshape(-1) / ha
            col[j] += sigma
            B[k, :, j] = col
    return B


def test_ej_colouring_is_bitwise_the_definition(orc):
    L, dq, _ = _tiny(orc, n=(4, 2), p=1)
    B = L.ej_blocks(dq, 2.5)
    assert np.array_equal(B, _ej_blocks_naive(L, dq, 2.5))


def test_ej_blocks_are_diagonal_blocks_of_dense_jacobian(orc, tiny2d):
    L, dq, J = tiny2d
    sigma = 11.0
    B = L.ej_blocks(dq, sigma)
    # dense index of (v, i, k) is (v*Np + i)*Ne + k
    for k in range(L.Ne):
        idx = np.arange(L.nb) * L.Ne + k
        ref = sigma * np.eye(L.nb) - J[np.ix_(idx, idx)]
        assert np.allclose(B[k], ref, rtol=0, atol=2e-5 * np.abs(ref).max())


def test_ej_blocks_3d(orc):
    L, dq, _ = _tiny(orc, dim=3, n=(2, 2, 2), p=1)
    J = dense_jacobian(L, dq)
    B = L.ej_blocks(dq, 0.0)
    for k in [0, 3, 7]:
        idx = np.arange(L.nb) * L.Ne + k
        assert np.allclose(B[k], -J[np.ix_(idx, idx)], rtol=0, atol=2e-5 * np.abs(J).max())


def test_lu_against_lapack(orc):
    rng = np.random.default_rng(2)
    B = rng.standard_normal((7, 20, 20)) + 3 * np.eye(20)
    B[3, :, 0] = 0.0
    B[3, 5, 0] = 1e-3           # forces a pivot search
    LU, piv, st = orc.lu_factor(B)
    assert st == 0
    for k in range(7):
        lu_ref, piv_ref = scipy.linalg.lu_factor(B[k])
        assert np.array_equal(piv[k], piv_ref)
        assert np.allclose(LU[k], lu_ref, rtol=0, atol=1e-13 * np.abs(B[k]).max())
        # P A = L U reconstruction
        Lm = np.tril(LU[k], -1) + np.eye(20)
        Um = np.triu(LU[k])
        PA = B[k].copy()
        for c in range(20):
            PA[[c, piv[k][c]]] = PA[[piv[k][c], c]]
        assert np.linalg.norm(PA - Lm @ Um) <= 1e-14 * np.linalg.norm(B[k]) * 20
    x = rng.standard_normal((20, 7))            # state layout: entry j of block k at [j, k]
    y = orc.lu_solve((LU, piv), x)
    for k in range(7):
        assert np.allclose(y[:, k], np.linalg.solve(B[k], x[:, k]), rtol=1e-12, atol=1e-12)


def test_lu_reports_singular_block(orc):
    B = np.eye(4)[None].repeat(2, axis=0)
    B[1] = 0.0
    _, _, st = orc.lu_factor(B)
    assert st == -4


def test_fgmres_dense(orc):
    rng = np.random.default_rng(4)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, st = orc.fgmres(lambda v: A @ v, lambda v: v, b, m=30, tol=1e-12, max_restarts=20)
    assert st.converged
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-10)
    # the residual estimate never increases within the run
    h = np.array(st.history)
    assert np.all(np.diff(h[:31]) <= 1e-12 * h[0])
    # a variable (flexible) preconditioner still converges to the same solution
    D = np.diag(1.0 / np.diag(A))
    cnt = [0]

    def M(v):
        cnt[0] += 1
        return D @ v * (1.0 + 0.1 * (cnt[0] % 3))
    x2, st2 = orc.fgmres(lambda v: A @ v, M, b, m=30, tol=1e-12, max_restarts=20)
    assert st2.converged and np.allclose(x2, np.linalg.solve(A, b), rtol=1e-10, atol=1e-10)


def test_fgmres_restart_recomputes_true_residual(orc):
    rng = np.random.default_rng(6)
    n = 80
    A = np.diag(np.linspace(1, 100, n)) + 0.01 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, st = orc.fgmres(lambda v: A @ v, lambda v: v, b, m=5, tol=1e-10, max_restarts=500)
    assert st.converged and st.restarts > 0
    assert np.linalg.norm(b - A @ x) <= 1.01e-10 * np.linalg.norm(b)


class _LinearLevel:
    """A Level whose residual is the linear map R(q) = J q."""

    def __init__(self, base, J):
        self.__dict__.update({k: getattr(base, k) for k in ("dim", "p", "P", "nv", "Np", "Ne", "nb", "N")})
        self.J = J

    @property
    def shape(self):
        return (self.nv, self.Np, self.Ne)

    def residual(self, q):
        return (self.J @ q.reshape(-1)).reshape(self.shape)


def _blocks_of(M, L, sigma):
    B = np.zeros((L.Ne, L.nb, L.nb))
    for k in range(L.Ne):
        idx = np.arange(L.nb) * L.Ne + k
        B[k] = sigma * np.eye(L.nb) - M[np.ix_(idx, idx)]
    return B


def _state_matrix(Md, L):
    """Per-element, per-variable dense operator (points x points) lifted to
    the state layout (v, i, k) -> (v*Np + i)*Ne + k."""
    n0, n1 = Md.shape
    out = np.zeros((L[1].nv * n0 * L[1].Ne, L[0].nv * n1 * L[0].Ne))
    Ne, nv = L[0].Ne, L[0].nv
    for v in range(nv):
        for k in range(Ne):
            rows = (v * n0 + np.arange(n0)) * Ne + k
            cols = (v * n1 + np.arange(n1)) * Ne + k
            out[np.ix_(rows, cols)] = Md
    return out


@pytest.mark.parametrize("n0,n1", [(2, 2), (1, 3), (3, 1)])
def test_pmg_linear_is_closed_form_two_grid(orc, n0, n1):
    """With a linear R the nonlinear pMG is the two-grid operator
    K0 X, d = X - A0 Y, Y += Pi K1 Gamma d, Y += K0 (X - A0 Y)."""
    fine, dq, _ = _tiny(orc, n=(4, 4), p=2, seed=3)
    coarse = orc.Level(dim=2, n=(4, 4), h=fine.h, p=1, gamma=1.4, mu=1e-2, Pr=0.72, tau=0.1, qinf=fine.qinf)
    rng = np.random.default_rng(8)
    J0 = dense_jacobian(fine, dq)
    J1 = dense_jacobian(coarse, orc.restrict(dq, 2, 3, 2))
    sigma_D, sigma_S = 40.0, 55.0
    F, C = _LinearLevel(fine, J0), _LinearLevel(coarse, J1)
    fac0 = orc.lu_factor(_blocks_of(J0, fine, sigma_S))
    fac1 = orc.lu_factor(_blocks_of(J1, coarse, sigma_S))
    for mode in (orc.SCALE_LITERAL, orc.SCALE_NORMALIZED):
        pm = orc.PMG(F, C, fac0, fac1, orc.PMGParams(sigma_D=sigma_D, n0=n0, n1=n1, scale_mode=mode))
        pm.set_point(np.zeros(fine.shape), np.zeros(fine.shape))
        X = rng.standard_normal(fine.shape)
        Y = pm.apply(X).reshape(-1)
        # closed form with dense matrices
        N0, N1 = fine.N, coarse.N
        A0 = sigma_D * np.eye(N0) - J0
        A1 = sigma_D * np.eye(N1) - J1
        B0 = np.zeros((N0, N0))
        for k in range(fine.Ne):
            idx = np.arange(fine.nb) * fine.Ne + k
            B0[np.ix_(idx, idx)] = _blocks_of(J0, fine, sigma_S)[k]
        B1 = np.zeros((N1, N1))
        for k in range(coarse.Ne):
            idx = np.arange(coarse.nb) * coarse.Ne + k
            B1[np.ix_(idx, idx)] = _blocks_of(J1, coarse, sigma_S)[k]
        B0i, B1i = np.linalg.inv(B0), np.linalg.inv(B1)

        def K(n, A, Bi):
            S = np.zeros_like(A)
            T = np.eye(A.shape[0])
            for _ in range(n):
                S += T @ Bi
                T = T @ (np.eye(A.shape[0]) - Bi @ A)
            return S
        K0, K1 = K(n0, A0, B0i), K(n1, A1, B1i)
        G1, P1 = orc.transfer1d(3, 2)
        Gam = _state_matrix(np.kron(G1, G1), (fine, coarse))
        Pi = _state_matrix(np.kron(P1, P1), (coarse, fine))
        x = X.reshape(-1)
        Yp = K0 @ x
        d = x - A0 @ Yp
        Yc = Yp + Pi @ (K1 @ (Gam @ d))
        Yref = Yc + K0 @ (x - A0 @ Yc)
        assert np.allclose(Y, Yref, rtol=0, atol=1e-12 * np.abs(Yref).max())


def test_pmg_one_sweep_is_element_jacobi(orc):
    """One pseudo-time step from Y = 0 recovers the EJ preconditioner (Sec. 3.2)."""
    fine, dq, rng = _tiny(orc, n=(4, 4), p=2, seed=5)
    sigma = 30.0
    fac = orc.lu_factor(fine.ej_blocks(dq, sigma))
    X = rng.standard_normal(fine.shape)
    for mode, rtol in ((orc.SCALE_LITERAL, 0.0), (orc.SCALE_NORMALIZED, 1e-13)):
        pm = orc.PMG(fine, None, fac, None, orc.PMGParams(sigma_D=sigma, n0=1, n1=0, coarse=False,
                                                          scale_mode=mode))
        pm.set_point(dq, fine.residual(dq))
        ref = orc.lu_solve(fac, X)
        assert np.allclose(pm.apply(X), ref, rtol=0, atol=rtol * np.abs(ref).max())


def test_pmg_nonlinear_close_to_linearisation(orc):
    """For Navier-Stokes, P(cX)/c - P(X) = O(c) in literal scaling."""
    fine, dq, rng = _tiny(orc, n=(4, 4), p=2, seed=6)
    coarse = orc.Level(dim=2, n=(4, 4), h=fine.h, p=1, gamma=1.4, mu=1e-2, Pr=0.72, tau=0.1, qinf=fine.qinf)
    sigma = 50.0
    fac0 = orc.lu_factor(fine.ej_blocks(dq, sigma + 10))
    fac1 = orc.lu_factor(coarse.ej_blocks(orc.restrict(dq, 2, 3, 2), sigma + 10))
    pm = orc.PMG(fine, coarse, fac0, fac1, orc.PMGParams(sigma_D=sigma, scale_mode=orc.SCALE_LITERAL))
    pm.set_point(dq, fine.residual(dq))
    X = rng.standard_normal(fine.shape) * 1e-3
    Y1 = pm.apply(X)
    d = []
    for c in (2.0, 4.0, 8.0):
        d.append(np.linalg.norm(pm.apply(c * X) / c - Y1))
    assert d[0] < d[1] < d[2]
    assert 1.5 < d[2] / d[1] < 3.0


def _dense_newton_stage(L, dq_n, dt, g, J_of, tol=1e-13):
    R0 = L.residual(dq_n)
    b = dq_n + g * dt * R0
    q = dq_n.copy()
    for _ in range(30):
        F = ((q - b) / (g * dt) - L.residual(q)).reshape(-1)
        if np.linalg.norm(F) < tol * np.linalg.norm(2 * R0):
            break
        A = np.eye(L.N) / (g * dt) - J_of(q)
        q = q - np.linalg.solve(A, F).reshape(L.shape)
    return q


@pytest.mark.parametrize("precond", ["ej", "pmg"])
def test_esdirk_stage_equals_dense_newton(orc, precond):
    wl = W.make_bump_workload(n=(4, 4), p0=2, p1=1, Ma=0.2, dt_factor=10.0, seed=12, amp=5e-2)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    q, st = orc.esdirk_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, precond=precond,
                             eta=0.01 if precond == "ej" else 0.1, tol=1e-11)
    assert st.converged
    # F(q^n) = -2 R(q^n)
    assert abs(st.res0 - 2 * np.linalg.norm(L0.residual(wl.dq))) <= 1e-12 * st.res0
    qref = _dense_newton_stage(L0, wl.dq, wl.dt, wl.a_ii, lambda q: dense_jacobian(L0, q))
    assert np.linalg.norm(q - qref) <= 1e-9 * np.linalg.norm(qref - wl.dq) + 1e-12 * np.linalg.norm(qref)


def test_row_stage_equals_dense_solve(orc):
    wl = W.make_bump_workload(n=(4, 4), p0=2, p1=1, Ma=0.2, dt_factor=10.0, seed=13, scheme="row", amp=5e-2)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    Y, st = orc.row_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, precond="pmg", tol=1e-10)
    # the FD operator is linear only up to O(h) and rounding: the true
    # residual sits within a small factor of the Krylov estimate
    assert st.rel_res <= 5e-10
    J = dense_jacobian(L0, wl.dq)
    Yref = np.linalg.solve(np.eye(L0.N) / (wl.a_ii * wl.dt) - J, L0.residual(wl.dq).reshape(-1))
    assert np.linalg.norm(Y.reshape(-1) - Yref) <= 1e-6 * np.linalg.norm(Yref)


def test_pmg_beats_ej_on_stiff_case(orc):
    """Shape check of the paper's claim (pMG cuts GMRES iterations vs EJ):
    low Mach, stretched mesh, large time step."""
    wl = W.make_vortical_workload(n=(8, 8), dt_factor=1000.0)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    _, s_ej = orc.esdirk_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, precond="ej", eta=0.01)
    _, s_pm = orc.esdirk_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, precond="pmg", eta=0.1)
    assert s_ej.converged and s_pm.converged
    assert s_pm.gmres_iters * 2 < s_ej.gmres_iters


def test_central_jvp_is_second_order(orc, tiny2d):
    """The central FD product converges to the dense Jacobian at second
    order in the step (error falls ~100x per decade of eps, against ~10x for
    the one-sided product), and is odd in the step: the product along -v is
    minus the product along v, exactly."""
    L, dq, J = tiny2d
    rq = L.residual(dq)
    v = np.random.default_rng(2).standard_normal(L.shape)
    sigma = 3.7
    ref = sigma * v.reshape(-1) - J @ v.reshape(-1)
    err = {}
    for central in (False, True):
        err[central] = []
        for eps in [1e-2, 1e-3]:
            w = orc.jvp(L, dq, rq, v, sigma, eps=eps, mode=orc.EPS_NORMALIZED, central=central)
            err[central].append(np.linalg.norm(w.reshape(-1) - ref) / np.linalg.norm(ref))
    one, cen = err[False], err[True]
    assert 5 < one[0] / one[1] < 20
    assert cen[0] / cen[1] > 50
    assert cen[1] < 1e-2 * one[1]
    wp = orc.jvp(L, dq, rq, v, 0.0, eps=1e-4, mode=orc.EPS_NORMALIZED, central=True)
    wm = orc.jvp(L, dq, rq, -v, 0.0, eps=1e-4, mode=orc.EPS_NORMALIZED, central=True)
    assert np.array_equal(wp, -wm)


def test_row_stage_meets_its_recomputed_residual(orc):
    """The ROW stage stops on the residual of the FD operator recomputed at
    its solution (one-sided and central products alike).  The central
    product is linear to O(h^2), so its stage needs no extra cycle and lands
    closer to numpy.linalg.solve(sigma I - J, R) than the one-sided stage
    (whose FD operator is linear only to O(h))."""
    L, dq, _ = _tiny(orc, p=1, amp=0.2)
    L1 = None
    dt, g = 0.05, 0.25
    sigma = 1.0 / (g * dt)
    R0 = L.residual(dq)
    J = dense_jacobian(L, dq)
    Yx = np.linalg.solve(sigma * np.eye(L.N) - J, R0.reshape(-1))
    out = {}
    for central in (False, True):
        Y, st = orc.row_stage(L, L1, dq, dt, g, precond="ej", tol=1e-9, central=central)
        A = lambda v: orc.jvp(L, dq, R0, v, sigma, eps=1e-6, mode=orc.EPS_SCALED, central=central)
        true = np.linalg.norm(R0 - A(Y)) / np.linalg.norm(R0)
        assert st.converged and true <= 1e-9 and abs(true - st.rel_res) <= 1e-3 * true
        out[central] = (st.gmres_iters, np.linalg.norm(Y.reshape(-1) - Yx) / np.linalg.norm(Yx))
    assert out[True][0] <= out[False][0]
    assert out[True][1] < 0.1 * out[False][1]
    # below the rounding floor of the recomputed residual (~1e-10 here) the
    # stage stops once a further cycle no longer halves it, converged on its
    # estimate, and reports the floor
    _, st = orc.row_stage(L, L1, dq, dt, g, precond="ej", tol=1e-11)
    assert st.converged and 1e-11 < st.rel_res < 1e-9 and st.gmres_iters < 60


def test_fgmres_verify_restarts_until_the_true_residual_meets_tol():
    """An operator that is linear up to a small non-additive part (as a
    finite-difference product is): the plain estimate-based stop leaves a
    true residual above the tolerance, verify=True continues from the true
    residual until it meets the tolerance; with a linear operator verify
    changes nothing."""
    import oracle as orc
    rng = np.random.default_rng(3)
    n = 60
    Amat = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    C = rng.standard_normal((n, n)) / np.sqrt(n)

    def A_nonlin(v):   # positively homogeneous, non-additive at ~1e-6
        nv = np.linalg.norm(v)
        return Amat @ v + (1e-6 * C @ (v * v) / nv if nv > 0 else 0.0)
    M = lambda v: v / 4.0
    x0, s0 = orc.fgmres(A_nonlin, M, b, m=40, tol=1e-10)
    x1, s1 = orc.fgmres(A_nonlin, M, b, m=40, tol=1e-10, verify=True)
    t0 = np.linalg.norm(b - A_nonlin(x0)) / np.linalg.norm(b)
    t1 = np.linalg.norm(b - A_nonlin(x1)) / np.linalg.norm(b)
    assert s0.converged and t0 > 1e-9
    assert s1.converged and t1 <= 1e-10 and s1.restarts >= 1
    xl0, _ = orc.fgmres(lambda v: Amat @ v, M, b, m=40, tol=1e-10)
    xl1, sl1 = orc.fgmres(lambda v: Amat @ v, M, b, m=40, tol=1e-10, verify=True)
    assert sl1.restarts == 0 and np.array_equal(xl0, xl1)
