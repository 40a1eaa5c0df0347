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
so the oracle derives its own from the order conditions (Hairer & Wanner,
Solving ODEs II, Sec. IV.6 and IV.7):

* ESDIRK3: four stages, explicit first stage, stiffly accurate, order 3,
  diagonal gamma = the root in (0.4, 0.5) of 6 g^3 - 18 g^2 + 9 g - 1
  (L-stability), abscissae c = (0, 2 gamma, 3/5, 1).  The remaining
  coefficients follow from the four order-3 conditions.
* ROW3: three stages, order 3, L-stable, the same gamma (so both schemes
  share the shift 1/(gamma dt) and the same preconditioner), alpha_21 =
  alpha_31 = 1, alpha_32 = 0 (stages 2 and 3 evaluate R at the same state),
  b = (2/3, 1/6, 1/6), beta_31 = beta_21; beta_21 and beta_32 follow from
  the two remaining order conditions.  Used in the transformed form of the
  paper's Eq. (Rosenbrock_General):
      (I/(gamma dt) - J) Y_i = R(q^n + sum_j a_ij Y_j) + (1/dt) sum_j c_ij Y_j,
      q^{n+1} = q^n + sum_i m_i Y_i.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

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
    Gi = np.linalg.inv(Gam)
    t = ROWTableau(alpha=alpha, Gam=Gam, b=b, gamma=g)
    t.a = alpha @ Gi
    t.cm = np.diag(1.0 / np.diag(Gam)) - Gi
    t.m = b @ Gi
    return t


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
             tol=1e-8, eps=1e-6, eps_mode=EPS_SCALED, pmg_kw=None):
    """One ROW time step (Sec. 2.1 Eq. (Rosenbrock_General), transformed
    form): for each stage i, (I/(gamma dt) - J) Y_i = R(q^n + sum_j a_ij Y_j)
    + (1/dt) sum_j c_ij Y_j with J the FD Jacobian at q^n, solved by FGMRES
    to tol relative to its right-hand side; q^{n+1} = q^n + sum m_i Y_i.  The
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
        Y, ks = fgmres(A, M, rhs, m=m, tol=tol, max_restarts=max_restarts)
        st = StageStats()
        st.gmres_iters = ks.iters
        st.converged = bool(ks.converged)
        st.res0 = float(np.linalg.norm(rhs))
        out.stages.append(st)
        out.gmres_iters += ks.iters
        out.converged = out.converged and st.converged
        U.append(Y)
    return dq_n + sum(tab.m[i] * U[i] for i in range(len(tab.b))), out
