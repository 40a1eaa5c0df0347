"""Pins of the oracle's full time steps (ESDIRK3 and ROW3 tableaux, the step
drivers).  The tableaux are derived inside the oracle from order conditions;
here they are checked against what fixes them independently of that
derivation: measured convergence orders against exact solutions of linear
(matrix exponential) and nonlinear (closed form) ODEs, the linear stability
function at infinity and on the imaginary axis, and the published
coefficients of the four-stage L-stable ESDIRK with c3 = 3/5 (Kennedy &
Carpenter's ESDIRK3(2)4L[2]SA, which the same conditions single out)."""
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


@pytest.mark.parametrize("scheme", ["esdirk3", "row3"])
@pytest.mark.parametrize("problem", ["linear", "nonlinear"])
def test_convergence_order_3(scheme, problem):
    f, jac, y0, exact = _linear_problem() if problem == "linear" else _nonlinear_problem()
    if scheme == "esdirk3":
        tab = S.esdirk3_tableau()
        stepper = lambda f, j, y, h: S.esdirk_step_ode(f, j, y, h, tab)
    else:
        tab = S.row3_tableau()
        stepper = lambda f, j, y, h: S.row_step_ode(f, j, y, h, tab)
    orders, errs = _orders(stepper, f, jac, y0, exact)
    assert min(orders[1:]) > 2.85, (orders, errs)
    assert max(orders) < 3.3, (orders, errs)


def test_planted_row_error_drops_the_order():
    """A perturbed ROW coefficient still passes a linear test's leading terms
    only through the stability function; the nonlinear problem must see it."""
    f, jac, y0, exact = _nonlinear_problem()
    tab = S.row3_tableau()
    tab.cm = tab.cm.copy()
    tab.cm[2, 1] *= 1.05
    stepper = lambda f, j, y, h: S.row_step_ode(f, j, y, h, tab)
    orders, _ = _orders(stepper, f, jac, y0, exact)
    assert orders[-1] < 2.5


@pytest.mark.parametrize("scheme", ["esdirk3", "row3"])
def test_l_stability(scheme):
    if scheme == "esdirk3":
        t = S.esdirk3_tableau()
        A, b = t.A, t.b
    else:
        t = S.row3_tableau()
        A, b = t.alpha + t.Gam, t.b
    assert abs(S.stability(-1e9, A, b)) < 1e-6
    ys = np.concatenate([np.logspace(-3, 5, 400), -np.logspace(-3, 5, 400)])
    assert max(abs(S.stability(1j * y, A, b)) for y in ys) <= 1.0 + 1e-12
    xs = -np.logspace(-3, 5, 60)
    assert max(abs(S.stability(x + 1j * y, A, b)) for x in xs for y in ys[::20]) <= 1.0 + 1e-12


def test_fr_steps_small_dt_consistency(orc):
    """On an FR system with a tiny time step both full steps agree with the
    Taylor expansion q + dt R + dt^2/2 J R to third order in dt, and with
    each other."""
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
    qe, se = S.esdirk_step(fine, coarse, q, dt, tol=1e-12, eta=1e-3)
    qr, sr = S.row_step(fine, coarse, q, dt, tol=1e-12)
    assert se.converged and sr.converged
    step = np.linalg.norm(dt * R)
    assert np.linalg.norm(qe - taylor) <= 1e-3 * step
    assert np.linalg.norm(qr - taylor) <= 1e-3 * step
    assert np.linalg.norm(qe - qr) <= 1e-4 * step
