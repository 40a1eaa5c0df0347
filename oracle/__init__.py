"""Plain FP64 CPU oracle for the p-multigrid preconditioned JFNK stage solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the GPU path in ``paper_2202_09733_amd``: the residual, the EJ
blocks and the block LU are the C file ``fr_oracle.c`` next to this one
(built with gcc -O2 -ffp-contract=off), everything above them is numpy below.

Paper: Wang, Trojak, Witherden, Jameson, "Nonlinear p-multigrid preconditioner
for implicit time integration of compressible Navier-Stokes equations",
arXiv 2202.09733.  Each function names the passage it follows.

State vectors are deviations dq = q - q_inf from the reference state, laid out
[nvar][npts][nelem]; see ``fr_oracle.c``.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
except where its docstring says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fr_oracle.c")
_SO = os.path.join(_HERE, "_fr_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile fr_oracle.c into a shared library next to it."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.or_residual.argtypes = [ctypes.c_void_p, dp, dp]
        L.or_residual.restype = ctypes.c_int
        L.or_ej_blocks.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_double, dp]
        L.or_ej_blocks.restype = ctypes.c_int
        L.or_lu_factor_batch.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip]
        L.or_lu_factor_batch.restype = ctypes.c_int
        L.or_lu_solve_batch.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip, dp, dp]
        L.or_lu_solve_batch.restype = None
        L.or_ops1d.argtypes = [ctypes.c_int, dp]
        L.or_transfer1d.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.or_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.or_inviscid_dflux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, dp]
        L.or_roe_dflux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, dp, dp]
        L.or_viscous_flux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class _MeshC(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("P", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("h", ctypes.POINTER(ctypes.c_double) * 3),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("Pr", ctypes.c_double),
                ("tau", ctypes.c_double), ("qinf", ctypes.c_double * 5)]


# ---------------------------------------------------------------------------
# 1D operators and transfers
# ---------------------------------------------------------------------------

def ops1d(P: int) -> dict:
    """Nodes, weights, D, end interpolants and correction derivatives."""
    out = np.zeros(P * P + 6 * P)
    lib().or_ops1d(P, _dp(out))
    o = {}
    o["xi"] = out[0:P].copy()
    o["w"] = out[P:2 * P].copy()
    o["D"] = out[2 * P:2 * P + P * P].reshape(P, P).copy()
    s = 2 * P + P * P
    o["bm"] = out[s:s + P].copy()
    o["bp"] = out[s + P:s + 2 * P].copy()
    o["gLd"] = out[s + 2 * P:s + 3 * P].copy()
    o["gRd"] = out[s + 3 * P:s + 4 * P].copy()
    return o


def transfer1d(P0: int, P1: int):
    """1D restriction (P1 x P0) and prolongation (P0 x P1) by L2 projection,
    Sec. 3.1 Eqs. (projection), (prolongation)."""
    G = np.zeros(P1 * P0)
    Pi = np.zeros(P0 * P1)
    lib().or_transfer1d(P0, P1, _dp(G), _dp(Pi))
    return G.reshape(P1, P0), Pi.reshape(P0, P1)


def _kron_d(M: np.ndarray, dim: int) -> np.ndarray:
    out = M
    for _ in range(dim - 1):
        out = np.kron(M, out)
    return out


def restrict(x: np.ndarray, dim: int, P0: int, P1: int) -> np.ndarray:
    """Apply Gamma = Gamma_1 (x) ... (x) Gamma_1 per element and variable."""
    G, _ = transfer1d(P0, P1)
    Gd = _kron_d(G, dim)
    return np.ascontiguousarray(np.einsum("ij,vjk->vik", Gd, x))


def prolong(x: np.ndarray, dim: int, P0: int, P1: int) -> np.ndarray:
    """Apply Pi = Pi_1 (x) ... (x) Pi_1 per element and variable."""
    _, Pi = transfer1d(P0, P1)
    Pd = _kron_d(Pi, dim)
    return np.ascontiguousarray(np.einsum("ij,vjk->vik", Pd, x))


def level_restrict(fine, coarse, x: np.ndarray) -> np.ndarray:
    """Gamma from one level of a p-hierarchy to the next coarser one: the
    uniform transfer, or element by element on mixed-degree levels."""
    if hasattr(fine, "restrict_to"):
        return fine.restrict_to(coarse, x)
    return restrict(x, fine.dim, fine.P, coarse.P)


def level_prolong(fine, coarse, x: np.ndarray) -> np.ndarray:
    """Pi from a coarse level back to the finer one (see level_restrict)."""
    if hasattr(fine, "prolong_from"):
        return fine.prolong_from(coarse, x)
    return prolong(x, fine.dim, fine.P, coarse.P)


# ---------------------------------------------------------------------------
# One polynomial level of the FR discretisation
# ---------------------------------------------------------------------------

class Level:
    """FR operator R on one periodic mesh at one polynomial degree p."""

    def __init__(self, dim, n, h, p, gamma, mu, Pr, tau, qinf):
        self.dim, self.p, self.P = int(dim), int(p), int(p) + 1
        self.n = tuple(int(x) for x in n) + (1,) * (3 - len(n))
        self.h = [np.ascontiguousarray(np.asarray(h[a], dtype=np.float64)) for a in range(dim)]
        self.nv = dim + 2
        self.Np = self.P ** dim
        self.Ne = int(np.prod(self.n[:dim]))
        self.nb = self.nv * self.Np
        self.N = self.nv * self.Np * self.Ne
        self.gamma, self.mu, self.Pr, self.tau = gamma, mu, Pr, tau
        self.qinf = np.asarray(qinf, dtype=np.float64)
        m = _MeshC()
        m.dim, m.P = self.dim, self.P
        for a in range(3):
            m.n[a] = self.n[a]
        for a in range(dim):
            m.h[a] = _dp(self.h[a])
        m.gamma, m.mu, m.Pr, m.tau = gamma, mu, Pr, tau
        for v in range(self.nv):
            m.qinf[v] = self.qinf[v]
        self._m = m

    @property
    def shape(self):
        return (self.nv, self.Np, self.Ne)

    def residual(self, dq: np.ndarray) -> np.ndarray:
        """R(q) = -(div f)_h by FR (Sec. 2.1 Eq. (1); FR reading in fr_oracle.c)."""
        dq = np.ascontiguousarray(dq, dtype=np.float64).reshape(self.shape)
        r = np.empty(self.shape)
        rc = lib().or_residual(ctypes.byref(self._m), _dp(dq), _dp(r))
        if rc:
            raise MemoryError("or_residual failed: %d" % rc)
        return r

    def ej_blocks(self, dq: np.ndarray, sigma: float, r0: np.ndarray | None = None) -> np.ndarray:
        """Element-Jacobi blocks sigma I - dR_k/dq_k, [Ne][nb][nb] (Sec. 2.2)."""
        dq = np.ascontiguousarray(dq, dtype=np.float64).reshape(self.shape)
        if r0 is None:
            r0 = self.residual(dq)
        B = np.empty((self.Ne, self.nb, self.nb))
        rc = lib().or_ej_blocks(ctypes.byref(self._m), _dp(dq), _dp(np.ascontiguousarray(r0)),
                                float(sigma), _dp(B))
        if rc == -1:
            raise ValueError("EJ colouring needs an even element count per axis")
        if rc:
            raise MemoryError("or_ej_blocks failed: %d" % rc)
        return B


# ---------------------------------------------------------------------------
# Block LU (element-Jacobi factor / solve)
# ---------------------------------------------------------------------------

def lu_factor(B: np.ndarray):
    """Partial-pivoting LU of every block (getrf semantics).  Returns (LU, piv, status)."""
    LU = np.ascontiguousarray(B, dtype=np.float64).copy()
    nblk, n, _ = LU.shape
    piv = np.zeros((nblk, n), dtype=np.int32)
    st = lib().or_lu_factor_batch(nblk, n, _dp(LU), _ip(piv))
    return LU, piv, st


def lu_solve(fac, x: np.ndarray) -> np.ndarray:
    """y_k = B_k^{-1} x_k for every element block, state layout in and out."""
    LU, piv = fac[0], fac[1]
    nblk, n, _ = LU.shape
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().or_lu_solve_batch(nblk, n, _dp(LU), _ip(piv), _dp(x), _dp(y))
    return y


# ---------------------------------------------------------------------------
# Finite-difference Jacobian-vector product (Sec. 2.2)
# ---------------------------------------------------------------------------

EPS_ABSOLUTE, EPS_NORMALIZED, EPS_SCALED = 0, 1, 2


def fd_step(v: np.ndarray, eps: float, mode: int, dq: np.ndarray | None = None) -> float:
    """Step h of the FD matvec: ABSOLUTE h = eps; NORMALIZED h = eps / ||v||_2
    (the paper's fixed eps applied to the unit direction); SCALED
    h = eps (1 + ||dq||_2) / ||v||_2 (the paper's eps with Knoll-Keyes
    scaling by the size of the state deviation)."""
    if mode == EPS_ABSOLUTE:
        return eps
    nv = float(np.linalg.norm(v))
    if nv == 0.0:
        return eps
    if mode == EPS_SCALED:
        return eps * (1.0 + float(np.linalg.norm(dq))) / nv
    return eps / nv


def jvp(level: Level, dq, rq, v, shift, eps=1e-6, mode=EPS_SCALED, central=False):
    """w = shift v - (R(q + h v) - R(q)) / h  (Sec. 2.2, matrix-free product).
    central=True (not the paper's form): w = shift v - (R(q + h v) -
    R(q - h v)) / (2 h), second-order accurate in h (rq unused)."""
    h = fd_step(v, eps, mode, dq)
    if central:
        return shift * v - (level.residual(dq + h * v) - level.residual(dq - h * v)) / (2.0 * h)
    return shift * v - (level.residual(dq + h * v) - rq) / h


# ---------------------------------------------------------------------------
# Flexible GMRES (right preconditioned, CGS2, Givens)
# ---------------------------------------------------------------------------

@dataclass
class KrylovStats:
    iters: int = 0
    restarts: int = 0
    matvecs: int = 0
    precs: int = 0
    converged: bool = False
    breakdown: bool = False
    res_est: float = float("nan")
    history: list = field(default_factory=list)


def fgmres(A, M, b, m=30, tol=1e-8, max_restarts=20, max_iters=None, verify=False):
    """Solve A x = b from x0 = 0 with flexible GMRES(m) (Saad 1993), right
    preconditioning z_j = M(v_j), classical Gram-Schmidt with one
    re-orthogonalisation, Givens rotations for the least-squares problem.
    The paper's Krylov solver is GMRES (Sec. 2.2); the flexible form is needed
    because the p-multigrid preconditioner is nonlinear (Sec. 3.2).
    Converged when the residual estimate <= tol ||b||.  A restart recomputes
    the true residual b - A x.  verify=True: once the estimate meets the
    tolerance, the true residual b - A x is recomputed and decides; if it does
    not meet the tolerance a new cycle starts from it, as long as each such
    recomputation at least halves the previous one; when one does not, the
    solve ends there as converged on its estimate, and res_est holds the
    recomputed residual (for an operator that is linear only to the accuracy
    of a finite difference, the estimate and the true residual differ, and
    the latter has a floor)."""
    st = KrylovStats()
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    target = tol * bnorm
    st.history.append(bnorm)
    if bnorm == 0.0:
        st.converged = True
        st.res_est = 0.0
        return x, st
    r = b.copy()
    beta = bnorm
    prev_true = None
    while True:
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        jend = 0
        for j in range(m):
            z = M(V[j])
            st.precs += 1
            w = A(z)
            st.matvecs += 1
            Vm = np.stack(V)                       # (j+1, ...)
            Vf = Vm.reshape(len(V), -1)
            wf = w.reshape(-1)
            h1 = Vf @ wf
            wf = wf - Vf.T @ h1
            h2 = Vf @ wf
            wf = wf - Vf.T @ h2
            hcol = h1 + h2
            hn = float(np.linalg.norm(wf))
            H[:j + 1, j] = hcol
            H[j + 1, j] = hn
            Z.append(z)
            for i in range(j):                     # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            st.iters += 1
            jend = j + 1
            st.res_est = abs(g[j + 1])
            st.history.append(st.res_est)
            if hn == 0.0:
                st.breakdown = True
                break
            V.append((wf / hn).reshape(b.shape))
            if st.res_est <= target:
                break
            if max_iters is not None and st.iters >= max_iters:
                break
        y = scipy.linalg.solve_triangular(H[:jend, :jend], g[:jend], lower=False)
        for i in range(jend):
            x = x + y[i] * Z[i]
        est_done = st.res_est <= target or st.breakdown
        if est_done and (not verify or st.breakdown):
            st.converged = True
            return x, st
        if not est_done:
            if st.restarts >= max_restarts or (max_iters is not None and st.iters >= max_iters):
                return x, st
            st.restarts += 1
        r = b - A(x)
        st.matvecs += 1
        beta = float(np.linalg.norm(r))
        st.res_est = beta
        if beta <= target:
            st.converged = True
            return x, st
        if est_done:
            if prev_true is not None and beta > 0.5 * prev_true:
                st.converged = True        # the floor of the operator: the estimate met tol
                return x, st
            if st.restarts >= max_restarts:
                return x, st
            prev_true = beta
            st.restarts += 1


# ---------------------------------------------------------------------------
# Nonlinear p-multigrid preconditioner (Sec. 3.1 applied to Sec. 3.2)
# ---------------------------------------------------------------------------

SCALE_LITERAL, SCALE_NORMALIZED, SCALE_SCALED = 0, 1, 2


@dataclass
class PMGParams:
    sigma_D: float          # 1/dtau + 1/(a_ii dt) (ESDIRK) or 1/(a_ii dt) (ROW)
    n0: int = 2             # pre- and post-sweeps on p0
    n1: int = 2             # sweeps on p1
    scale_mode: int = SCALE_SCALED
    eps_p: float = 1e-6
    coarse: bool = True     # False: fine-level smoothing only (no coarse correction, no post-sweeps)
    learned: object = None  # mlp.LearnedCoarse: the coarse sweeps replaced by the learned correction


class PMG:
    """Two-level nonlinear pMG preconditioner Y ~ A^{-1} X.

    It solves 0 = X + R(q + Y) - R(q) - sigma_D Y (Sec. 3.2, the nonlinear
    preconditioner equation with q_hat = q + Y) by one FAS V-cycle
    (Sec. 3.1), smoothing with the element-Jacobi linearised pseudo-time step
    Y <- Y - B^{-1} G(Y), where G(Y) = sigma_D Y - [R(q+Y) - R(q)] - X and
    B = sigma_S I - dR_k/dq_k holds the blocks with sigma_S = 1/dtau* + sigma_D
    (the pseudo-time backward-Euler step, alpha = 1), frozen at the start of
    the time step (Sec. 2.2).  X is scaled by s before the cycle and Y by
    1/s after: LITERAL s = 1; NORMALIZED s = eps_p sigma_D / ||X||;
    SCALED s = eps_p sigma_D (1 + ||q||) / ||X||, so that Y is a small
    perturbation of the state in the same sense as the FD matvec step.

    With ``prm.learned`` (an ``mlp.LearnedCoarse``) the coarse sweeps are
    replaced by the learned correction (not in the paper): C1 = B1^{-1} Gamma d
    from the restricted defect d = -G(Y), the correction C = learned(C1), and
    Y <- Y + Pi C before the post-sweeps.

    fine/coarse: Level objects; fac0/fac1: LU factors of B on each level.
    """

    def __init__(self, fine: Level, coarse: Level | None, fac0, fac1, prm: PMGParams):
        self.fine, self.coarse, self.fac0, self.fac1, self.prm = fine, coarse, fac0, fac1, prm
        self.q = None

    def set_point(self, dq: np.ndarray, rq: np.ndarray):
        """Linearisation point: the current Newton iterate and R there."""
        self.q, self.rq = dq, rq
        if self.coarse is not None and self.prm.coarse:
            self.q1 = level_restrict(self.fine, self.coarse, dq)
            self.r1 = self.coarse.residual(self.q1)

    def _G(self, Y, X):
        p = self.prm
        return p.sigma_D * Y - (self.fine.residual(self.q + Y) - self.rq) - X

    def _G1(self, Z, S):
        p = self.prm
        return p.sigma_D * Z - (self.coarse.residual(self.q1 + Z) - self.r1) - S

    def apply(self, X: np.ndarray) -> np.ndarray:
        p = self.prm
        s = 1.0
        if p.scale_mode in (SCALE_NORMALIZED, SCALE_SCALED):
            xn = float(np.linalg.norm(X))
            size = 1.0 + float(np.linalg.norm(self.q)) if p.scale_mode == SCALE_SCALED else 1.0
            s = p.eps_p * p.sigma_D * size / xn if xn > 0 else 1.0
        Xs = s * X
        # pre-smoothing (the first sweep starts from Y = 0 where G = -X)
        Y = np.zeros_like(X)
        for it in range(p.n0):
            G = -Xs if it == 0 else self._G(Y, Xs)
            Y = Y - lu_solve(self.fac0, G)
        if self.coarse is None or not p.coarse:
            return Y / s
        # defect and restriction; FAS forcing S1 = F1(Gamma Y) + Gamma d
        d = -self._G(Y, Xs)
        if p.learned is not None:
            C1 = lu_solve(self.fac1, level_restrict(self.fine, self.coarse, d))
            Y = Y + level_prolong(self.fine, self.coarse, p.learned.correct(C1))
            for it in range(p.n0):
                Y = Y - lu_solve(self.fac0, self._G(Y, Xs))
            return Y / s
        Z0 = level_restrict(self.fine, self.coarse, Y)
        dc = level_restrict(self.fine, self.coarse, d)
        S1 = self._G1(Z0, 0.0) + dc
        Z = Z0.copy()
        for it in range(p.n1):
            Gc = -dc if it == 0 else self._G1(Z, S1)
            Z = Z - lu_solve(self.fac1, Gc)
        # prolongate the coarse change and post-smooth
        Y = Y + level_prolong(self.fine, self.coarse, Z - Z0)
        for it in range(p.n0):
            Y = Y - lu_solve(self.fac0, self._G(Y, Xs))
        return Y / s


# ---------------------------------------------------------------------------
# Stage solves
# ---------------------------------------------------------------------------

@dataclass
class StageStats:
    ptc_iters: int = 0
    gmres_iters: int = 0
    gmres_per_newton: list = field(default_factory=list)
    res0: float = float("nan")
    res: float = float("nan")
    rel_res: float = float("nan")
    converged: bool = False
    history: list = field(default_factory=list)


def _setup_precond(fine, coarse, dq_lin, kind, sigma_EJ, sigma_D, sigma_S, pmg_kw):
    """Blocks evaluated at the start of the time step (Sec. 2.2)."""
    if kind == "ej":
        fac = lu_factor(fine.ej_blocks(dq_lin, sigma_EJ))
        return lambda x: lu_solve(fac, x), None
    fac0 = lu_factor(fine.ej_blocks(dq_lin, sigma_S))
    fac1 = None
    use_coarse = pmg_kw.get("coarse", True)
    if coarse is not None and use_coarse:
        q1 = level_restrict(fine, coarse, dq_lin)
        fac1 = lu_factor(coarse.ej_blocks(q1, sigma_S))
    pm = PMG(fine, coarse, fac0, fac1, PMGParams(sigma_D=sigma_D, **pmg_kw))
    return pm.apply, pm


def esdirk_stage(fine: Level, coarse: Level | None, dq_n, dt, a_ii, a_i1=None, precond="pmg",
                 eta=0.1, m=30, max_restarts=20, tol=1e-8, max_ptc=100, eps=1e-6,
                 eps_mode=EPS_SCALED, dtau=None, pmg_kw=None):
    """Second stage of an ESDIRK scheme with explicit first stage
    (Sec. 2.1 Eq. (ESDIRK2)): q_2 = q^n + dt (a_21 R(q^n) + a_22 R(q_2)),
    solved by pseudo-transient continuation with inexact Newton
    (Sec. 2.2 Eqs. (SDIRK_newton), (pseudo_transient),
    (linearized_pseudo_transient_final)): each PTC step solves
    (I/dtau + I/(a_ii dt) - dR/dq) dq = -F(q) by FGMRES to relative tolerance
    eta with the FD matvec.  Stops when ||F|| <= tol ||F(q^n)||."""
    pmg_kw = dict(pmg_kw or {})
    a_i1 = a_ii if a_i1 is None else a_i1
    dtau = dt if dtau is None else dtau
    sigma_A = 1.0 / dtau + 1.0 / (a_ii * dt)
    sigma_S = 1.0 / dtau + sigma_A                  # dtau* = dtau
    st = StageStats()
    M, pm = _setup_precond(fine, coarse, dq_n, precond, sigma_A, sigma_A, sigma_S, pmg_kw)
    R0 = fine.residual(dq_n)
    b = dq_n + (a_i1 * dt) * R0
    q = dq_n.copy()
    rq = R0
    F = (q - b) / (a_ii * dt) - rq
    f0 = float(np.linalg.norm(F))
    st.res0 = f0
    st.history.append(f0)
    fn = f0
    while fn > tol * f0 and st.ptc_iters < max_ptc:
        if pm is not None:
            pm.set_point(q, rq)
        A = lambda v, q=q, rq=rq: jvp(fine, q, rq, v, sigma_A, eps, eps_mode)
        dx, ks = fgmres(A, M, -F, m=m, tol=eta, max_restarts=max_restarts)
        st.gmres_iters += ks.iters
        st.gmres_per_newton.append(ks.iters)
        q = q + dx
        rq = fine.residual(q)
        F = (q - b) / (a_ii * dt) - rq
        fn = float(np.linalg.norm(F))
        st.history.append(fn)
        st.ptc_iters += 1
        if not np.isfinite(fn):
            break
    st.res = fn
    st.rel_res = fn / f0 if f0 > 0 else 0.0
    st.converged = bool(fn <= tol * f0)
    return q, st


def row_stage(fine: Level, coarse: Level | None, dq_n, dt, a_ii, precond="pmg", m=30,
              max_restarts=50, tol=1e-8, eps=1e-6, eps_mode=EPS_SCALED, pmg_kw=None, central=False,
              verify=True):
    """First stage of a Rosenbrock-Wanner scheme (Sec. 2.1 Eq.
    (Rosenbrock_General) with i = 1): (I/(a_ii dt) - dR/dq(q^n)) Y = R(q^n),
    solved by FGMRES with the FD matvec to ||R(q^n) - A_h Y|| <= tol ||R(q^n)||
    (verify=True: the recomputed residual decides; verify=False: the Krylov
    estimate).
    The preconditioner is the ROW form of Sec. 3.2 (pseudo-time terms of the
    outer solver dropped; dtau* = dt).  central=True takes the central FD
    product (jvp) for the Krylov solve and the recomputed residual."""
    pmg_kw = dict(pmg_kw or {})
    sigma = 1.0 / (a_ii * dt)
    sigma_S = 1.0 / dt + sigma
    st = StageStats()
    M, pm = _setup_precond(fine, coarse, dq_n, precond, sigma, sigma, sigma_S, pmg_kw)
    R0 = fine.residual(dq_n)
    if pm is not None:
        pm.set_point(dq_n, R0)
    A = lambda v: jvp(fine, dq_n, R0, v, sigma, eps, eps_mode, central)
    Y, ks = fgmres(A, M, R0, m=m, tol=tol, max_restarts=max_restarts, verify=verify)
    st.gmres_iters = ks.iters
    st.gmres_per_newton.append(ks.iters)
    st.res0 = float(np.linalg.norm(R0))
    st.res = float(np.linalg.norm(R0 - A(Y)))
    st.rel_res = st.res / st.res0 if st.res0 > 0 else 0.0
    st.converged = bool(ks.converged)
    st.history = ks.history
    return Y, st
