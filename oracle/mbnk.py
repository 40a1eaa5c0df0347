"""Matrix-based Newton-Krylov (MBNK) smoother for the oracle: an assembled
coarse-level Jacobian, its block ILU0 factorisation and the smoothing sweep.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).

Sec. 3.2 names two smoothers for the pMG levels: element-Jacobi and MBNK,
for which GMRES runs to a relative tolerance of 1e-1 with at most five
iterations, preconditioned by ILU0 (per domain-decomposition block).  Where
the paper is silent this oracle reads it as:

* The MBNK sweep solves the same linearised pseudo-time step as the EJ sweep,
  A~ delta = G(Y), Y <- Y - delta, with A~ = sigma_S I - J instead of its
  block diagonal; the Krylov matvec uses the assembled A~.
* The assembled J keeps, for every element k, the blocks dR_k/dq_m for m = k
  and its 2 dim face neighbours, each by one-sided differences with the EJ
  step rule (1e-7 max(1, |q_j|)).  Through the LDG gradient R_k also depends
  on its edge-diagonal neighbours; those blocks are not assembled.
* ILU0 is taken in red-black element ordering (colour = parity of the
  coordinate sum; an even element count per periodic axis), which makes the
  factorisation and both triangular solves element-parallel.  With face
  neighbours only, red rows have no lower entries, so
      U_rr = A_rr,  L_br = A_br A_rr^{-1},
      U_bb = A_bb - sum_{r ~ b} A_br A_rr^{-1} A_rb   (ILU0 keeps the black
  diagonal blocks only), U_br = 0 rows beyond the pattern.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fgmres


def _coords(L, k):
    n0, n1 = L.n[0], L.n[1]
    return (k % n0, (k // n0) % n1, k // (n0 * n1))


def _index(L, c):
    return c[0] + L.n[0] * (c[1] + L.n[1] * c[2])


def face_neighbour(L, k, a, s):
    """Element across the face of k normal to axis a on side s = -1 / +1 (periodic)."""
    c = list(_coords(L, k))
    c[a] = (c[a] + s) % L.n[a]
    return _index(L, c)


def slot(a, s):
    """Neighbour slot of (axis a, side s): 2 a + (s > 0)."""
    return 2 * a + (1 if s > 0 else 0)


def _stride(n):
    for s in range(3, n + 1):
        if n % s == 0:
            return s
    raise ValueError("the neighbour-block colouring needs at least three elements per axis")


def jacobian_blocks(L, dq, r0=None):
    """J[k][0] = dR_k/dq_k and J[k][1 + slot(a, s)] = dR_k/dq_m, m the face
    neighbour (a, s) of k: [Ne][1 + 2 dim][nb][nb], rows and columns in the
    local order v*Np + i.  One-sided differences with the EJ step; elements
    perturbed together are at least three apart along some axis, so their
    residual stencils (the element, its face and edge neighbours) do not
    overlap."""
    dq = np.ascontiguousarray(dq, dtype=np.float64).reshape(L.shape)
    r0 = L.residual(dq) if r0 is None else r0
    dim, Ne, nb, Np = L.dim, L.Ne, L.nb, L.Np
    strides = [_stride(L.n[a]) for a in range(dim)]
    J = np.zeros((Ne, 1 + 2 * dim, nb, nb))
    colour = np.zeros(Ne, dtype=int)
    for k in range(Ne):
        c = _coords(L, k)
        col, mul = 0, 1
        for a in range(dim):
            col += (c[a] % strides[a]) * mul
            mul *= strides[a]
        colour[k] = col
    ncol = int(np.prod(strides))
    for col in range(ncol):
        members = np.nonzero(colour == col)[0]
        for j in range(nb):
            v, i = divmod(j, Np)
            qp = dq.copy()
            h = np.zeros(Ne)
            for m in members:
                hj = 1e-7 * max(1.0, abs(L.qinf[v] + dq[v, i, m]))
                qp[v, i, m] = dq[v, i, m] + hj
                h[m] = qp[v, i, m] - dq[v, i, m]
            d = (L.residual(qp) - r0).reshape(nb, Ne)
            for m in members:
                J[m, 0, :, j] = d[:, m] / h[m]
                for a in range(dim):
                    for s in (-1, 1):
                        k = face_neighbour(L, m, a, s)
                        # m is k's neighbour on the opposite side
                        J[k, 1 + slot(a, -s), :, j] = d[:, k] / h[m]
    return J


@dataclass
class Assembled:
    """A~ = sigma I - J on the face-neighbour block pattern."""
    L: object
    D: np.ndarray   # [Ne][nb][nb] diagonal blocks
    O: np.ndarray   # [Ne][2 dim][nb][nb] off-diagonal blocks (slot order)


def assemble(L, dq, sigma, r0=None) -> Assembled:
    J = jacobian_blocks(L, dq, r0)
    D = sigma * np.eye(L.nb)[None, :, :] - J[:, 0]
    return Assembled(L=L, D=D, O=-J[:, 1:])


def matvec(A: Assembled, x):
    L = A.L
    X = np.asarray(x).reshape(L.nb, L.Ne)
    Y = np.einsum("kij,jk->ik", A.D, X)
    for a in range(L.dim):
        for s in (-1, 1):
            nbr = np.array([face_neighbour(L, k, a, s) for k in range(L.Ne)])
            Y += np.einsum("kij,jk->ik", A.O[:, slot(a, s)], X[:, nbr])
    return Y.reshape(L.shape)


def red(L, k):
    return sum(_coords(L, k)[:L.dim]) % 2 == 0


@dataclass
class ILU0:
    A: Assembled
    Dinv: np.ndarray  # red: A_rr^{-1}; black: U_bb^{-1}
    is_red: np.ndarray


def ilu0(A: Assembled) -> ILU0:
    """Block ILU0 in red-black ordering (see the module docstring)."""
    L = A.L
    for a in range(L.dim):
        if L.n[a] % 2:
            raise ValueError("red-black ILU0 needs an even element count per axis")
    is_red = np.array([red(L, k) for k in range(L.Ne)])
    Dinv = np.zeros_like(A.D)
    for k in np.nonzero(is_red)[0]:
        Dinv[k] = np.linalg.inv(A.D[k])
    for b in np.nonzero(~is_red)[0]:
        U = A.D[b].copy()
        for a in range(L.dim):
            for s in (-1, 1):
                r = face_neighbour(L, b, a, s)
                U -= A.O[b, slot(a, s)] @ Dinv[r] @ A.O[r, slot(a, -s)]
        Dinv[b] = np.linalg.inv(U)
    return ILU0(A=A, Dinv=Dinv, is_red=is_red)


def ilu0_solve(f: ILU0, rhs):
    """z = (L U)^{-1} rhs: w_r = A_rr^{-1} r_r; x_b = U_bb^{-1} (r_b - sum A_br w_r);
    x_r = A_rr^{-1} (r_r - sum A_rb x_b)."""
    L, A = f.A.L, f.A
    R = np.asarray(rhs).reshape(L.nb, L.Ne)
    X = np.zeros_like(R)
    W = np.zeros_like(R)
    for k in np.nonzero(f.is_red)[0]:
        W[:, k] = f.Dinv[k] @ R[:, k]
    for b in np.nonzero(~f.is_red)[0]:
        y = R[:, b].copy()
        for a in range(L.dim):
            for s in (-1, 1):
                y -= A.O[b, slot(a, s)] @ W[:, face_neighbour(L, b, a, s)]
        X[:, b] = f.Dinv[b] @ y
    for r in np.nonzero(f.is_red)[0]:
        y = R[:, r].copy()
        for a in range(L.dim):
            for s in (-1, 1):
                y -= A.O[r, slot(a, s)] @ X[:, face_neighbour(L, r, a, s)]
        X[:, r] = f.Dinv[r] @ y
    return X.reshape(L.shape)


def mbnk_sweep(f: ILU0, G, tol=0.1, maxit=5):
    """delta ~ A~^{-1} G by GMRES (right-preconditioned by ILU0, at most maxit
    iterations, relative tolerance tol); the sweep is Y <- Y - delta."""
    delta, _ = fgmres(lambda v: matvec(f.A, v), lambda v: ilu0_solve(f, v), G, m=maxit, tol=tol, max_restarts=0)
    return delta
