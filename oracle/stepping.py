"""Full implicit time steps for the oracle: every stage of an ESDIRK scheme
and of a Rosenbrock-Wanner (ROW) scheme, with the preconditioner formed once
per time step.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``: only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
may use it).

The paper integrates in time with ESDIRK schemes (Sec. 2.1, Eq. (ESDIRK2) and
the stage equations around it) and with ROW schemes (Sec. 2.1, Eq.
(Rosenbrock_General)), and forms the preconditioner at the start of each
physical time step (Sec. 2.2).  It names its tableaux without printing them,
so the oracle builds its own (Hairer & Wanner, Solving ODEs II, Sec. IV.6
and IV.7), in pairs that share the diagonal gamma (hence the shift
1/(gamma dt) and the preconditioner):

* order 2 (the paper's ESDIRK2 / ROW2 comparison of Sec. 4.2), gamma =
  1 - 1/sqrt(2) (L-stability of two implicit stages of order 2):
  - ESDIRK2: three stages, explicit first stage, stiffly accurate,
    c = (0, 2 gamma, 1), b from the two order-2 conditions (Kennedy &
    Carpenter's ESDIRK2(1)3L[2]SA);
  - ROW2: two stages, alpha_21 = 1, b = (1/2, 1/2), beta_21 from the
    remaining order-2 condition.
* order 3, gamma = the root in (0.4, 0.5) of 6 g^3 - 18 g^2 + 9 g - 1:
  - ESDIRK3: four stages, explicit first stage, stiffly accurate,
    c = (0, 2 gamma, 3/5, 1), the rest from the four order-3 conditions;
  - ROW3: three stages, alpha_21 = alpha_31 = 1, alpha_32 = 0 (stages 2 and
    3 evaluate R at the same state), b = (2/3, 1/6, 1/6), beta_31 =
    beta_21; beta_21 and beta_32 from the two remaining order conditions.
* order 4 (the ESDIRK4 / ROW4 comparison of Sec. 4.3):
  - ESDIRK4: the six-stage ESDIRK of Bijl et al. (2002), i.e. the implicit
    tableau of Kennedy & Carpenter's ARK4(3)6L[2]SA, gamma = 1/4, with its
    published rational coefficients;
  - ROW4: four stages, gamma = 0.5728160624821349 (1/x with x the second
    root of the Laguerre polynomial L_4: L-stability at s = p = 4),
    Shampine's alpha (alpha_21 = 1, alpha_31 = alpha_41 = 12/25,
    alpha_32 = alpha_42 = 3/25, alpha_43 = 0: stages 3 and 4 evaluate R at
    the same state) and b = (8/27, 1/8, 0, 125/216), gamma_31 = 0, and the
    other beta_ij from the order-4 conditions.

ROW schemes are used in the transformed form of the paper's
Eq. (Rosenbrock_General):
    (I/(gamma dt) - J) Y_i = R(q^n + sum_j a_ij Y_j) + (1/dt) sum_j c_ij Y_j,
    q^{n+1} = q^n + sum_i m_i Y_i,
with a = alpha Gamma^{-1}, c = diag(1/gamma) - Gamma^{-1}, m = b Gamma^{-1}.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from . import EPS_SCALED, StageStats, _setup_precond, fgmres, jvp


def lstable_gamma() -> float:
    """Root in (0.4, 0.5) of 6 g^3 - 18 g^2 + 9 g - 1: the diagonal that makes
    a three-implicit-stage order-3 scheme L-stable."""
    r = np.roots([6.0, -18.0, 9.0, -1.0])
    r = [x.real for x in r if abs(x.imag) < 1e-12 and 0.4 < x.real < 0.5]
    g = r[0]
    for _ in range(3):  # Newton polish
        g -= (6 * g ** 3 - 18 * g ** 2 + 9 * g - 1) / (18 * g ** 2 - 36 * g + 9)
    return float(g)


@dataclass
class ESDIRKTableau:
    A: np.ndarray  # (s, s), first row zero, a_ii = gamma for i >= 1
    b: np.ndarray
    c: np.ndarray
    gamma: float


def esdirk3_tableau() -> ESDIRKTableau:
    """ESDIRK3 from the order conditions sum b = 1, sum b c = 1/2,
    sum b c^2 = 1/3, sum b A c = 1/6 with b = last row of A (stiffly
    accurate), c = (0, 2 gamma, 3/5, 1)."""
    g = lstable_gamma()
    c2, c3 = 2.0 * g, 0.6
    # b4 = g, c4 = 1: b2 c2 + b3 c3 = 1/2 - g and b2 c2^2 + b3 c3^2 = 1/3 - g
    b2, b3 = np.linalg.solve(np.array([[c2, c3], [c2 * c2, c3 * c3]]), np.array([0.5 - g, 1.0 / 3.0 - g]))
    b1 = 1.0 - b2 - b3 - g
    # sum_i b_i sum_j a_ij c_j = b2 (g c2) + b3 (a32 c2 + g c3) + g (b2 c2 + b3 c3 + g) = 1/6
    a32 = (1.0 / 6.0 - b2 * g * c2 - b3 * g * c3 - g * (b2 * c2 + b3 * c3 + g)) / (b3 * c2)
    a31 = c3 - g - a32
    A = np.array([[0.0, 0.0, 0.0, 0.0],
                  [g, g, 0.0, 0.0],
                  [a31, a32, g, 0.0],
                  [b1, b2, b3, g]])
    return ESDIRKTableau(A=A, b=A[3].copy(), c=A.sum(axis=1), gamma=g)


@dataclass
class ROWTableau:
    alpha: np.ndarray  # (s, s) strictly lower
    Gam: np.ndarray    # (s, s) lower, diagonal gamma
    b: np.ndarray
    gamma: float
    a: np.ndarray = field(default=None)  # transformed: alpha Gam^{-1}
    cm: np.ndarray = field(default=None)  # transformed: diag(1/gamma) - Gam^{-1}
    m: np.ndarray = field(default=None)  # transformed: b Gam^{-1}


def _row(alpha: np.ndarray, Gam: np.ndarray, b: np.ndarray, g: float) -> ROWTableau:
    """A ROW tableau with its transformed coefficients a = alpha Gamma^{-1},
    c = diag(1/gamma) - Gamma^{-1}, m = b Gamma^{-1}."""
    Gi = scipy.linalg.solve_triangular(Gam, np.eye(len(b)), lower=True)
    t = ROWTableau(alpha=alpha, Gam=Gam, b=b, gamma=g)
    t.a = alpha @ Gi
    t.cm = np.diag(1.0 / np.diag(Gam)) - Gi
    t.m = b @ Gi
    return t


def row3_tableau() -> ROWTableau:
    """ROW3 from the Rosenbrock order conditions with beta_ij = alpha_ij +
    gamma_ij, beta_i' = sum_j beta_ij: sum b = 1, sum b beta' = 1/2 - gamma,
    sum b alpha_i^2 = 1/3, sum b_i beta_ij beta_j' = 1/6 - gamma + gamma^2."""
    g = lstable_gamma()
    b = np.array([2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0])
    alpha = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    # with beta31 = beta21 = x, beta32 = y:
    #   b2 x + b3 (x + y) = 1/2 - g   ->  2x + y = 3 - 6g
    #   b3 y x = 1/6 - g + g^2         ->  x y = 1 - 6g + 6g^2
    s_ = 3.0 - 6.0 * g
    p_ = 1.0 - 6.0 * g + 6.0 * g * g
    x = (s_ + np.sqrt(s_ * s_ - 8.0 * p_)) / 4.0
    y = s_ - 2.0 * x
    Gam = np.array([[g, 0.0, 0.0], [x - 1.0, g, 0.0], [x - 1.0, y, g]])
    return _row(alpha, Gam, b, g)


def gamma2() -> float:
    """1 - 1/sqrt(2): the root in (0, 1) of g^2 - 2 g + 1/2, which makes two
    implicit stages of order 2 L-stable."""
    return 1.0 - 1.0 / np.sqrt(2.0)


def esdirk2_tableau() -> ESDIRKTableau:
    """ESDIRK2: c = (0, 2 gamma, 1), stiffly accurate, b from sum b = 1 and
    sum b c = 1/2 with b_3 = gamma, c_3 = 1."""
    g = gamma2()
    b2 = (0.5 - g) / (2.0 * g)
    b1 = 1.0 - b2 - g
    A = np.array([[0.0, 0.0, 0.0], [g, g, 0.0], [b1, b2, g]])
    return ESDIRKTableau(A=A, b=A[2].copy(), c=A.sum(axis=1), gamma=g)


def row2_tableau() -> ROWTableau:
    """ROW2: alpha_21 = 1, b = (1/2, 1/2); sum b beta' = 1/2 - gamma gives
    beta_21 = 1 - 2 gamma, so gamma_21 = beta_21 - alpha_21 = -2 gamma."""
    g = gamma2()
    alpha = np.array([[0.0, 0.0], [1.0, 0.0]])
    Gam = np.array([[g, 0.0], [-2.0 * g, g]])
    return _row(alpha, Gam, np.array([0.5, 0.5]), g)


def esdirk4_tableau() -> ESDIRKTableau:
    """ESDIRK4: gamma = 1/4, c = (0, 1/2, 83/250, 31/50, 17/20, 1), stiffly
    accurate; the published rational coefficients of the implicit tableau of
    Kennedy & Carpenter's ARK4(3)6L[2]SA (the ESDIRK4 of Bijl et al.)."""
    g = 0.25
    A = np.zeros((6, 6))
    A[1, :2] = [g, g]
    A[2, :3] = [8611.0 / 62500.0, -1743.0 / 31250.0, g]
    A[3, :4] = [5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, g]
    A[4, :5] = [15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0,
                2285395.0 / 8070912.0, g]
    A[5, :] = [82889.0 / 524892.0, 0.0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, g]
    return ESDIRKTableau(A=A, b=A[5].copy(), c=A.sum(axis=1), gamma=g)


def gamma4() -> float:
    """1/x with x the second-smallest root of the Laguerre polynomial
    L_4(x) = (x^4 - 16 x^3 + 72 x^2 - 96 x + 24)/24: the diagonal that makes
    four stages of order 4 L-stable (and A-stable)."""
    c = [1.0, -16.0, 72.0, -96.0, 24.0]
    x = sorted(r.real for r in np.roots(c))[1]
    for _ in range(3):  # Newton polish
        x -= np.polyval(c, x) / np.polyval([4.0, -48.0, 144.0, -96.0], x)
    return float(1.0 / x)


def row4_tableau() -> ROWTableau:
    """ROW4 from the eight order-4 Rosenbrock conditions (Hairer & Wanner,
    Table IV.7.1) with alpha and b fixed as in Shampine's method and
    gamma_31 = 0.  With alpha_1 = 0, alpha_2 = 1, alpha_3 = alpha_4 = 3/5 and
    b_3 = 0 the conditions on beta reduce to
      b4 alpha_3 alpha_32 beta_21 = 1/8 - g/3,
      b4 beta_43 beta_32 beta_21 = 1/24 - g/2 + 3g^2/2 - g^3,
      b4 (beta_42 beta_21 + beta_43 beta_3') = 1/6 - g + g^2,
      b4 (beta_42 alpha_2^2 + beta_43 alpha_3^2) = 1/12 - g/3,
      b2 beta_21 + b4 beta_4' = 1/2 - g,
    solved in this order."""
    g = gamma4()
    b = np.array([8.0 / 27.0, 1.0 / 8.0, 0.0, 125.0 / 216.0])
    a31, a32 = 12.0 / 25.0, 3.0 / 25.0
    a3 = a31 + a32
    alpha = np.array([[0.0, 0.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0], [a31, a32, 0.0, 0.0], [a31, a32, 0.0, 0.0]])
    b2, b4 = b[1], b[3]
    B21 = (1.0 / 8.0 - g / 3.0) / (b4 * a3 * a32)
    P8 = (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g ** 3) / (b4 * B21)  # beta_43 beta_32
    Q4 = (1.0 / 6.0 - g + g * g) / b4
    S7 = (1.0 / 12.0 - g / 3.0) / b4
    T2 = (0.5 - g - b2 * B21) / b4  # beta_4'
    B31 = a31  # gamma_31 = 0
    # beta_42 = S7 - a3^2 beta_43; Q4 = beta_42 B21 + beta_43 B31 + P8
    B43 = (Q4 - P8 - S7 * B21) / (B31 - a3 * a3 * B21)
    B32 = P8 / B43
    B42 = S7 - a3 * a3 * B43
    B41 = T2 - B42 - B43
    beta = np.array([[0.0, 0.0, 0.0, 0.0], [B21, 0.0, 0.0, 0.0], [B31, B32, 0.0, 0.0], [B41, B42, B43, 0.0]])
    Gam = beta - alpha + g * np.eye(4)
    return _row(alpha, Gam, b, g)


ESDIRK_TABLEAUX = {"esdirk2": esdirk2_tableau, "esdirk3": esdirk3_tableau, "esdirk4": esdirk4_tableau}
ROW_TABLEAUX = {"row2": row2_tableau, "row3": row3_tableau, "row4": row4_tableau}


def stability(z: complex, A: np.ndarray, b: np.ndarray) -> complex:
    """Stability function R(z) = 1 + z b^T (I - z A)^{-1} 1 of a Runge-Kutta
    tableau (for a ROW scheme pass beta = alpha + Gamma)."""
    s = len(b)
    return 1.0 + z * (b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s)))


# ---------------------------------------------------------------------------
# steps of a small ODE system y' = f(y) with dense linear algebra (the pins)
# ---------------------------------------------------------------------------

def esdirk_step_ode(f, jac, y, h, tab: ESDIRKTableau, newton_tol=1e-13, max_newton=50):
    """One ESDIRK step: Y_1 = y, Y_i = y + h sum_{j<i} a_ij f(Y_j) + h a_ii f(Y_i)
    by Newton's method with the exact Jacobian; y_new = Y_s."""
    k = [f(y)]
    Yi = y
    for i in range(1, len(tab.b)):
        rhs = y + h * sum(tab.A[i, j] * k[j] for j in range(i))
        Yi = Yi.copy()
        for _ in range(max_newton):
            F = Yi - rhs - h * tab.A[i, i] * f(Yi)
            d = np.linalg.solve(np.eye(len(y)) - h * tab.A[i, i] * jac(Yi), -F)
            Yi = Yi + d
            if np.linalg.norm(d) <= newton_tol * (1.0 + np.linalg.norm(Yi)):
                break
        k.append(f(Yi))
    return Yi


def row_step_ode(f, jac, y, h, tab: ROWTableau):
    """One ROW step in the transformed form with J = jac(y)."""
    J = jac(y)
    n = len(y)
    U = []
    for i in range(len(tab.b)):
        w = y + sum(tab.a[i, j] * U[j] for j in range(i))
        r = f(w) + sum(tab.cm[i, j] / h * U[j] for j in range(i))
        U.append(np.linalg.solve(np.eye(n) / (h * tab.gamma) - J, r))
    return y + sum(tab.m[i] * U[i] for i in range(len(tab.b)))


# ---------------------------------------------------------------------------
# full time steps of the FR system with the paper's solvers
# ---------------------------------------------------------------------------

@dataclass
class StepStats:
    stages: list = field(default_factory=list)
    gmres_iters: int = 0
    converged: bool = True


def esdirk_step(fine, coarse, dq_n, dt, tab: ESDIRKTableau | None = None, precond="pmg", eta=0.1, m=30,
                max_restarts=20, tol=1e-8, max_ptc=100, eps=1e-6, eps_mode=EPS_SCALED, dtau=None, pmg_kw=None):
    """One ESDIRK time step of dq/dt = R(q) (Sec. 2.1): stage 1 is q^n; stage
    i solves F_i(q) = (q - b_i)/(a_ii dt) - R(q) = 0 with
    b_i = q^n + dt sum_{j<i} a_ij R(q_j), by pseudo-transient continuation
    with inexact Newton and preconditioned FGMRES (Sec. 2.2), starting from
    q_{i-1}, until ||F_i|| <= tol ||F_i(q_{i-1})||.  The preconditioner is
    formed once at q^n (Sec. 2.2); the pMG linearisation point follows the
    Newton iterate.  Stiffly accurate: q^{n+1} = q_s."""
    tab = tab or esdirk3_tableau()
    pmg_kw = dict(pmg_kw or {})
    g = tab.gamma
    dtau = dt if dtau is None else dtau
    sigma_A = 1.0 / dtau + 1.0 / (g * dt)
    sigma_S = 1.0 / dtau + sigma_A
    M, pm = _setup_precond(fine, coarse, dq_n, precond, sigma_A, sigma_A, sigma_S, pmg_kw)
    Rs = [fine.residual(dq_n)]
    q = dq_n.copy()
    rq = Rs[0]
    out = StepStats()
    for i in range(1, len(tab.b)):
        b = dq_n + dt * sum(tab.A[i, j] * Rs[j] for j in range(i))
        a_ii = tab.A[i, i]
        st = StageStats()
        F = (q - b) / (a_ii * dt) - rq
        f0 = float(np.linalg.norm(F))
        st.res0 = f0
        fn = f0
        while fn > tol * f0 and st.ptc_iters < max_ptc:
            if pm is not None:
                pm.set_point(q, rq)
            A = lambda v, q=q, rq=rq: jvp(fine, q, rq, v, sigma_A, eps, eps_mode)
            dx, ks = fgmres(A, M, -F, m=m, tol=eta, max_restarts=max_restarts)
            st.gmres_iters += ks.iters
            q = q + dx
            rq = fine.residual(q)
            F = (q - b) / (a_ii * dt) - rq
            fn = float(np.linalg.norm(F))
            st.ptc_iters += 1
            if not np.isfinite(fn):
                break
        st.res = fn
        st.rel_res = fn / f0 if f0 > 0 else 0.0
        st.converged = bool(fn <= tol * f0)
        out.stages.append(st)
        out.gmres_iters += st.gmres_iters
        out.converged = out.converged and st.converged
        Rs.append(rq)
    return q, out


def row_step(fine, coarse, dq_n, dt, tab: ROWTableau | None = None, precond="pmg", m=30, max_restarts=50,
             tol=1e-8, eps=1e-6, eps_mode=EPS_SCALED, pmg_kw=None, verify=True):
    """One ROW time step (Sec. 2.1 Eq. (Rosenbrock_General), transformed
    form): for each stage i, (I/(gamma dt) - J) Y_i = R(q^n + sum_j a_ij Y_j)
    + (1/dt) sum_j c_ij Y_j with J the FD Jacobian at q^n, solved by FGMRES
    to tol relative to its right-hand side (verify=True: the recomputed
    residual decides; False: the Krylov estimate);
    q^{n+1} = q^n + sum m_i Y_i.  The
    preconditioner is formed once at q^n and linearised there (Sec. 3.2, ROW
    form: pseudo-time terms dropped, dtau* = dt)."""
    tab = tab or row3_tableau()
    pmg_kw = dict(pmg_kw or {})
    sigma = 1.0 / (tab.gamma * dt)
    sigma_S = 1.0 / dt + sigma
    M, pm = _setup_precond(fine, coarse, dq_n, precond, sigma, sigma, sigma_S, pmg_kw)
    R0 = fine.residual(dq_n)
    if pm is not None:
        pm.set_point(dq_n, R0)
    A = lambda v: jvp(fine, dq_n, R0, v, sigma, eps, eps_mode)
    U = []
    out = StepStats()
    for i in range(len(tab.b)):
        if i == 0:
            Ri = R0
        else:
            Ri = fine.residual(dq_n + sum(tab.a[i, j] * U[j] for j in range(i)))
        rhs = Ri + sum(tab.cm[i, j] / dt * U[j] for j in range(i))
        Y, ks = fgmres(A, M, rhs, m=m, tol=tol, max_restarts=max_restarts, verify=verify)
        st = StageStats()
        st.gmres_iters = ks.iters
        st.converged = bool(ks.converged)
        st.res0 = float(np.linalg.norm(rhs))
        out.stages.append(st)
        out.gmres_iters += ks.iters
        out.converged = out.converged and st.converged
        U.append(Y)
    return dq_n + sum(tab.m[i] * U[i] for i in range(len(tab.b))), out
