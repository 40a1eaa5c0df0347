"""Pins of the oracle's full time steps (the ESDIRK2/3/4 and ROW2/3/4
tableaux, the step drivers).  The tableaux are derived inside the oracle from
(a subset of) the order conditions or typed from their publication; here they
are checked against what fixes them independently of that: every order
condition up to the scheme's order (rooted trees for Runge-Kutta, the
Rosenbrock table of Hairer & Wanner IV.7), measured convergence orders against
exact solutions of linear (matrix exponential) and nonlinear (closed form)
ODEs, the linear stability function at infinity, on the imaginary axis and in
the left half-plane, and the published coefficients of Kennedy & Carpenter's
ESDIRK3(2)4L[2]SA (which the order-3 conditions with c3 = 3/5 single out) and
ESDIRK2(1)3L[2]SA (b1 = b2 = sqrt(2)/4)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import stepping as S


def _orders(stepper, f, jac, y0, exact, T=1.0, Ns=(10, 20, 40, 80)):
    errs = []
    for N in Ns:
        y = y0.copy()
        h = T / N
        for _ in range(N):
            y = stepper(f, jac, y, h)
        errs.append(np.linalg.norm(y - exact(T)))
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)], errs


def _linear_problem():
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((6, 6))
    L = -(Q @ Q.T) - 0.5 * np.eye(6) + 0.3 * (Q - Q.T)
    y0 = rng.standard_normal(6)
    return (lambda y: L @ y), (lambda y: L), y0, (lambda t: scipy.linalg.expm(L * t) @ y0)


def _nonlinear_problem():
    # u' = -u + v^2, v' = -2 v:  v = v0 e^{-2t},  u = (u0 + v0^2/3) e^{-t} - (v0^2/3) e^{-4t};
    # w' = -w^2: w = w0 / (1 + w0 t)
    u0, v0, w0 = 0.7, 1.3, 0.9
    f = lambda y: np.array([-y[0] + y[1] ** 2, -2.0 * y[1], -y[2] ** 2])
    jac = lambda y: np.array([[-1.0, 2.0 * y[1], 0.0], [0.0, -2.0, 0.0], [0.0, 0.0, -2.0 * y[2]]])
    exact = lambda t: np.array([(u0 + v0 ** 2 / 3.0) * np.exp(-t) - (v0 ** 2 / 3.0) * np.exp(-4.0 * t),
                                v0 * np.exp(-2.0 * t), w0 / (1.0 + w0 * t)])
    return f, jac, np.array([u0, v0, w0]), exact


def test_lstable_gamma():
    g = S.lstable_gamma()
    assert abs(6 * g ** 3 - 18 * g ** 2 + 9 * g - 1) < 1e-14
    assert abs(g - 0.43586652150845899942) < 1e-15


def test_esdirk3_matches_published_coefficients():
    t = S.esdirk3_tableau()
    pub_b = [0.187641024346724, -0.595297473576955, 0.971789927721772, 0.435866521508459]
    assert np.allclose(t.b, pub_b, atol=2e-15)
    assert np.allclose(t.c, [0.0, 0.871733043016918, 0.6, 1.0], atol=2e-15)
    assert np.allclose(t.A[3], t.b)


ORDER = {"esdirk2": 2, "row2": 2, "esdirk3": 3, "row3": 3, "esdirk4": 4, "row4": 4}


def _stepper(scheme, tab=None):
    if scheme.startswith("esdirk"):
        tab = tab or S.ESDIRK_TABLEAUX[scheme]()
        return lambda f, j, y, h: S.esdirk_step_ode(f, j, y, h, tab)
    tab = tab or S.ROW_TABLEAUX[scheme]()
    return lambda f, j, y, h: S.row_step_ode(f, j, y, h, tab)


@pytest.mark.parametrize("scheme", list(ORDER))
@pytest.mark.parametrize("problem", ["linear", "nonlinear"])
def test_convergence_order(scheme, problem):
    f, jac, y0, exact = _linear_problem() if problem == "linear" else _nonlinear_problem()
    p = ORDER[scheme]
    # the order-4 schemes reach their asymptotic rate later: one halving more
    Ns = (20, 40, 80, 160) if p == 4 else (10, 20, 40, 80)
    orders, errs = _orders(_stepper(scheme), f, jac, y0, exact, Ns=Ns)
    assert min(orders[1:]) > p - 0.15, (orders, errs)
    assert max(orders) < p + 0.3, (orders, errs)


def _rk_conditions(A, b, p):
    """Residuals of the Runge-Kutta order conditions for every rooted tree
    with at most p (<= 4) vertices: sum b Phi(tree) = 1/gamma(tree)."""
    c = A.sum(axis=1)
    Ac, Ac2 = A @ c, A @ (c * c)
    r = [b.sum() - 1.0, b @ c - 0.5]
    if p >= 3:
        r += [b @ (c * c) - 1.0 / 3.0, b @ Ac - 1.0 / 6.0]
    if p >= 4:
        r += [b @ c ** 3 - 0.25, b @ (c * Ac) - 1.0 / 8.0, b @ Ac2 - 1.0 / 12.0, b @ (A @ Ac) - 1.0 / 24.0]
    return np.array(r)


def _row_conditions(t, p):
    """Residuals of the Rosenbrock order conditions up to order p (<= 4)
    (Hairer & Wanner, Table IV.7.1) with beta = alpha + Gamma off the
    diagonal."""
    g, b, al = t.gamma, t.b, t.alpha
    beta = np.tril(t.alpha + t.Gam, -1)
    bp, ai = beta.sum(axis=1), al.sum(axis=1)
    r = [b.sum() - 1.0, b @ bp - (0.5 - g)]
    if p >= 3:
        r += [b @ ai ** 2 - 1.0 / 3.0, b @ (beta @ bp) - (1.0 / 6.0 - g + g * g)]
    if p >= 4:
        r += [b @ ai ** 3 - 0.25, (b * ai) @ (al @ bp) - (1.0 / 8.0 - g / 3.0),
              b @ (beta @ ai ** 2) - (1.0 / 12.0 - g / 3.0),
              b @ (beta @ (beta @ bp)) - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g ** 3)]
    return np.array(r)


@pytest.mark.parametrize("scheme", list(ORDER))
def test_order_conditions(scheme):
    """Every condition up to the scheme's order holds to rounding; the
    structural choices hold exactly (explicit first stage, one diagonal,
    stiff accuracy for ESDIRK; lower-triangular Gamma with one diagonal for
    ROW); the next order's conditions do not all hold."""
    p = ORDER[scheme]
    if scheme.startswith("esdirk"):
        t = S.ESDIRK_TABLEAUX[scheme]()
        assert not np.any(t.A[0]) and np.all(np.diag(t.A)[1:] == t.gamma)
        assert np.array_equal(t.A[-1], t.b) and not np.any(np.triu(t.A, 1))
        res, nxt = _rk_conditions(t.A, t.b, p), _rk_conditions(t.A, t.b, min(p + 1, 4))
    else:
        t = S.ROW_TABLEAUX[scheme]()
        assert np.all(np.diag(t.Gam) == t.gamma) and not np.any(np.triu(t.Gam, 1))
        assert not np.any(np.triu(t.alpha))
        res, nxt = _row_conditions(t, p), _row_conditions(t, min(p + 1, 4))
    assert np.max(np.abs(res)) < 1e-14, res
    if p < 4:
        assert np.max(np.abs(nxt)) > 1e-3, nxt


def test_diagonals():
    """gamma of each pair from its own characterisation: g^2 - 2g + 1/2 = 0
    (order 2), the cubic (order 3), L_4(1/g) = 0 (order 4)."""
    g2, g4 = S.gamma2(), S.gamma4()
    assert abs(g2 * g2 - 2.0 * g2 + 0.5) < 4e-16 and 0.0 < g2 < 0.5
    x = 1.0 / g4
    assert abs((x ** 4 - 16 * x ** 3 + 72 * x ** 2 - 96 * x + 24) / 24.0) < 1e-13
    assert abs(g4 - 0.5728160624821349) < 1e-15
    assert S.esdirk4_tableau().gamma == 0.25


def test_esdirk2_matches_published_coefficients():
    t = S.esdirk2_tableau()
    assert np.allclose(t.b, [np.sqrt(2.0) / 4.0, np.sqrt(2.0) / 4.0, 1.0 - np.sqrt(2.0) / 2.0], atol=1e-15)
    assert np.allclose(t.c, [0.0, 2.0 - np.sqrt(2.0), 1.0], atol=1e-15)


def test_esdirk4_abscissae():
    t = S.esdirk4_tableau()
    assert np.allclose(t.c, [0.0, 0.5, 83.0 / 250.0, 31.0 / 50.0, 17.0 / 20.0, 1.0], atol=1e-15)


def test_planted_row_error_drops_the_order():
    """A perturbed ROW coefficient still passes a linear test's leading terms
    only through the stability function; the nonlinear problem must see it."""
    f, jac, y0, exact = _nonlinear_problem()
    tab = S.row3_tableau()
    tab.cm = tab.cm.copy()
    tab.cm[2, 1] *= 1.05
    orders, _ = _orders(_stepper("row3", tab), f, jac, y0, exact)
    assert orders[-1] < 2.5


@pytest.mark.parametrize("scheme", ["esdirk4", "row4"])
def test_planted_order4_error_drops_the_order(scheme):
    """One perturbed coefficient of the order-4 schemes (a fourth-order tree's
    weight) shows as a lower measured order on the nonlinear problem."""
    f, jac, y0, exact = _nonlinear_problem()
    if scheme == "esdirk4":
        tab = S.esdirk4_tableau()
        tab.A = tab.A.copy()
        tab.A[4, 3] *= 1.02
        tab.A[4, 0] -= 0.02 * S.esdirk4_tableau().A[4, 3]  # keep c_5
    else:
        tab = S.row4_tableau()
        tab.cm = tab.cm.copy()
        tab.cm[3, 2] *= 1.02
    orders, _ = _orders(_stepper(scheme, tab), f, jac, y0, exact)
    assert orders[-1] < 3.6, orders


@pytest.mark.parametrize("scheme", list(ORDER))
def test_l_stability(scheme):
    if scheme.startswith("esdirk"):
        t = S.ESDIRK_TABLEAUX[scheme]()
        A, b = t.A, t.b
    else:
        t = S.ROW_TABLEAUX[scheme]()
        A, b = t.alpha + t.Gam, t.b
    assert abs(S.stability(-1e9, A, b)) < 1e-6
    ys = np.concatenate([np.logspace(-3, 5, 400), -np.logspace(-3, 5, 400)])
    assert max(abs(S.stability(1j * y, A, b)) for y in ys) <= 1.0 + 1e-12
    xs = -np.logspace(-3, 5, 60)
    assert max(abs(S.stability(x + 1j * y, A, b)) for x in xs for y in ys[::20]) <= 1.0 + 1e-12


@pytest.mark.parametrize("order", [2, 3, 4])
def test_fr_steps_small_dt_consistency(orc, order):
    """On an FR system with a tiny time step both full steps of each pair
    agree with the Taylor expansion q + dt R + dt^2/2 J R to third order in
    dt, and with each other."""
    from paper_2202_09733_amd import workloads as W
    wl = W.make_bump_workload(name="tiny", n=(4, 4), p0=2, p1=1, dt_factor=1.0)
    fine = orc.Level(**wl.level_kwargs(wl.p0))
    coarse = orc.Level(**wl.level_kwargs(wl.p1))
    q = wl.dq
    R = fine.residual(q)
    dt = 1e-3 * float(np.linalg.norm(q)) / float(np.linalg.norm(R))
    h = 1e-7 * (1.0 + np.linalg.norm(q)) / np.linalg.norm(R)
    JR = (fine.residual(q + h * R) - R) / h
    taylor = q + dt * R + 0.5 * dt * dt * JR
    et = S.ESDIRK_TABLEAUX["esdirk%d" % order]()
    rt = S.ROW_TABLEAUX["row%d" % order]()
    qe, se = S.esdirk_step(fine, coarse, q, dt, tab=et, tol=1e-12, eta=1e-3)
    qr, sr = S.row_step(fine, coarse, q, dt, tab=rt, tol=1e-12)
    assert se.converged and sr.converged
    assert len(se.stages) == len(et.b) - 1 and len(sr.stages) == len(rt.b)
    step = np.linalg.norm(dt * R)
    assert np.linalg.norm(qe - taylor) <= 1e-3 * step
    assert np.linalg.norm(qr - taylor) <= 1e-3 * step
    assert np.linalg.norm(qe - qr) <= 1e-4 * step
