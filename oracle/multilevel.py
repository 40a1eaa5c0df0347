"""Multi-level nonlinear p-multigrid for the oracle: the FAS V-cycle over a
p-hierarchy of any depth (p{3-2-1}, p{4-2-1}, ...), used as the preconditioner
and as a standalone nonlinear solver of an ESDIRK stage.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).

Sec. 3.1 describes the V-cycle on two levels (pre-smoothing, defect,
restriction, coarse FAS forcing, coarse smoothing, prolongation of the coarse
change, post-smoothing) and uses deeper hierarchies (p{3-1-0},
p{3-2-1-0} for the nonlinear solver, p{3-2-1} for the preconditioner,
Tabs. 2, 5 and 6) with sweeps n{n0-n1-...}.  The deeper cycle applies the
two-level step recursively: on every level but the coarsest, n_l sweeps
before and after the correction from the level below; n_{L-1} sweeps on the
coarsest.  Each level's equation is
    G_l(Y) = sigma_D Y - [R_l(q_l + Y) - R_l(q_l)] - S_l = 0,
q_l the restricted linearisation point, S_0 = X and S_{l+1} =
G_{l+1}(Gamma Y_l; 0) + Gamma d_l (FAS forcing), smoothed by the element-Jacobi
pseudo-time step Y <- Y - B_l^{-1} G_l(Y) with blocks frozen at the start of
the time step.  With two levels this is exactly ``oracle.PMG``.

As a nonlinear solver (Sec. 3.1, the pMG baseline of Tab. 2/4): each
iteration applies one V-cycle to X = -F(q) with sigma_D = 1/(a_ii dt) and
literal scaling, so that G_0(Y) = 0 is F(q + Y) = 0, and sets q <- q + Y.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import (EPS_SCALED, SCALE_LITERAL, SCALE_NORMALIZED, SCALE_SCALED, StageStats, fgmres, jvp, lu_factor,
               level_prolong, level_restrict, lu_solve)
from . import mbnk as MB


@dataclass
class MultiPMGParams:
    sigma_D: float
    n: tuple                # sweeps per level; n[L-1] on the coarsest level
    scale_mode: int = SCALE_SCALED
    eps_p: float = 1e-6


class MultiPMG:
    """levels: Level objects, finest first; facs: LU factors of each level's
    blocks B_l = sigma_S I - dR_l/dq.  coarse_ilu: when given (an
    ``mbnk.ILU0`` of the coarsest level's assembled sigma_S I - J), the
    coarsest level smooths with MBNK sweeps instead of EJ sweeps."""

    def __init__(self, levels, facs, prm: MultiPMGParams, coarse_ilu=None):
        assert len(levels) == len(facs) == len(prm.n) and len(levels) >= 1
        self.levels, self.facs, self.prm, self.coarse_ilu = levels, facs, prm, coarse_ilu

    def _smooth_step(self, l, G):
        if self.coarse_ilu is not None and l == len(self.levels) - 1 and l > 0:
            return MB.mbnk_sweep(self.coarse_ilu, G)
        return lu_solve(self.facs[l], G)

    def set_point(self, dq: np.ndarray, rq: np.ndarray):
        self.q = [dq]
        self.r = [rq]
        for l in range(1, len(self.levels)):
            a, b = self.levels[l - 1], self.levels[l]
            ql = level_restrict(a, b, self.q[-1])
            self.q.append(ql)
            self.r.append(b.residual(ql))

    def _G(self, l, Y, S):
        return self.prm.sigma_D * Y - (self.levels[l].residual(self.q[l] + Y) - self.r[l]) - S

    def _cycle(self, l, S, Y0, G0):
        """Smooth G_l(Y) = 0 from Y0, where G_l(Y0) = G0, with the correction
        from the levels below in between."""
        n = self.prm.n[l]
        Y = Y0.copy()
        for it in range(n):
            G = G0 if it == 0 else self._G(l, Y, S)
            Y = Y - self._smooth_step(l, G)
        if l == len(self.levels) - 1:
            return Y
        a, b = self.levels[l], self.levels[l + 1]
        d = -self._G(l, Y, S)
        Z0 = level_restrict(a, b, Y)
        dc = level_restrict(a, b, d)
        S1 = self._G(l + 1, Z0, 0.0) + dc
        Z = self._cycle(l + 1, S1, Z0, -dc)
        Y = Y + level_prolong(a, b, Z - Z0)
        for it in range(n):
            Y = Y - lu_solve(self.facs[l], self._G(l, Y, S))
        return Y

    def apply(self, X: np.ndarray) -> np.ndarray:
        p = self.prm
        s = 1.0
        if p.scale_mode in (SCALE_NORMALIZED, SCALE_SCALED):
            xn = float(np.linalg.norm(X))
            size = 1.0 + float(np.linalg.norm(self.q[0])) if p.scale_mode == SCALE_SCALED else 1.0
            s = p.eps_p * p.sigma_D * size / xn if xn > 0 else 1.0
        Xs = s * X
        Y = self._cycle(0, Xs, np.zeros_like(X), -Xs)
        return Y / s


def hierarchy_factors(levels, dq_n, sigma_S):
    """Blocks of every level at the restricted q^n (Sec. 2.2: formed once per
    time step)."""
    facs, q = [], dq_n
    for l, L in enumerate(levels):
        if l > 0:
            a = levels[l - 1]
            q = level_restrict(a, L, q)
        facs.append(lu_factor(L.ej_blocks(q, sigma_S)))
    return facs


@dataclass
class NLStats:
    vcycles: int = 0
    res0: float = float("nan")
    res: float = float("nan")
    rel_res: float = float("nan")
    converged: bool = False


def coarse_mbnk(levels, dq_n, sigma_S):
    """ILU0 of the coarsest level's assembled sigma_S I - J at the restricted q^n."""
    q = dq_n
    for l in range(1, len(levels)):
        a, b = levels[l - 1], levels[l]
        q = level_restrict(a, b, q)
    return MB.ilu0(MB.assemble(levels[-1], q, sigma_S))


def esdirk_stage_ml(levels, dq_n, dt, a_ii, n=None, coarse="ej", eta=0.1, m=30, max_restarts=20, tol=1e-8,
                    max_ptc=100, eps=1e-6, eps_mode=EPS_SCALED, dtau=None):
    """The second ESDIRK stage as ``oracle.esdirk_stage`` (PTC + inexact Newton +
    FGMRES) with the multi-level pMG preconditioner; coarse = "ej" or "mbnk"
    (the coarsest level's smoother)."""
    dtau = dt if dtau is None else dtau
    n = tuple(n) if n is not None else tuple([2] * len(levels))
    sigma_A = 1.0 / dtau + 1.0 / (a_ii * dt)
    sigma_S = 1.0 / dtau + sigma_A
    facs = hierarchy_factors(levels, dq_n, sigma_S)
    ilu = coarse_mbnk(levels, dq_n, sigma_S) if coarse == "mbnk" else None
    pm = MultiPMG(levels, facs, MultiPMGParams(sigma_D=sigma_A, n=n), coarse_ilu=ilu)
    fine = levels[0]
    R0 = fine.residual(dq_n)
    b = dq_n + (a_ii * dt) * R0
    q, rq = dq_n.copy(), R0
    F = (q - b) / (a_ii * dt) - rq
    st = StageStats()
    f0 = float(np.linalg.norm(F))
    st.res0 = f0
    fn = f0
    while fn > tol * f0 and st.ptc_iters < max_ptc:
        pm.set_point(q, rq)
        A = lambda v, q=q, rq=rq: jvp(fine, q, rq, v, sigma_A, eps, eps_mode)
        dx, ks = fgmres(A, pm.apply, -F, m=m, tol=eta, max_restarts=max_restarts)
        st.gmres_iters += ks.iters
        st.gmres_per_newton.append(ks.iters)
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
    return q, st


def pmg_nonlinear_stage(levels, dq_n, dt, a_ii, a_i1=None, n=None, dtau=None, tol=1e-8, max_vcycles=500,
                        coarse="ej", refresh=0):
    """Second ESDIRK stage q = q^n + dt (a_i1 R(q^n) + a_ii R(q)) solved by
    pMG as the nonlinear solver: V-cycles on F(q + Y) = 0, smoothers with the
    pseudo-time shift sigma_S = 1/dtau + 1/(a_ii dt), blocks formed at q^n,
    until ||F|| <= tol ||F(q^n)||; coarse = "ej" or "mbnk" (the coarsest
    level's smoother).  refresh > 0 re-forms the smoothers at the current
    iterate every `refresh` V-cycles (Sec. 4.2.2 updates them every 20
    pseudo-time iterations for this solver)."""
    a_i1 = a_ii if a_i1 is None else a_i1
    dtau = dt if dtau is None else dtau
    n = tuple(n) if n is not None else tuple([2] * (len(levels) - 1) + [2])
    sigma = 1.0 / (a_ii * dt)
    sigma_S = 1.0 / dtau + sigma
    prm = MultiPMGParams(sigma_D=sigma, n=n, scale_mode=SCALE_LITERAL)

    def smoothers(q):
        facs = hierarchy_factors(levels, q, sigma_S)
        ilu = coarse_mbnk(levels, q, sigma_S) if coarse == "mbnk" else None
        return MultiPMG(levels, facs, prm, coarse_ilu=ilu)

    pm = smoothers(dq_n)
    fine = levels[0]
    R0 = fine.residual(dq_n)
    b = dq_n + (a_i1 * dt) * R0
    q, rq = dq_n.copy(), R0
    F = (q - b) / (a_ii * dt) - rq
    st = NLStats(res0=float(np.linalg.norm(F)))
    fn = st.res0
    while fn > tol * st.res0 and st.vcycles < max_vcycles:
        if refresh > 0 and st.vcycles > 0 and st.vcycles % refresh == 0:
            pm = smoothers(q)
        pm.set_point(q, rq)
        q = q + pm.apply(-F)
        rq = fine.residual(q)
        F = (q - b) / (a_ii * dt) - rq
        fn = float(np.linalg.norm(F))
        st.vcycles += 1
        if not np.isfinite(fn):
            break
    st.res = fn
    st.rel_res = fn / st.res0 if st.res0 > 0 else 0.0
    st.converged = bool(fn <= tol * st.res0)
    return q, st
