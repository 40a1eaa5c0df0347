"""p-adaptation (Sec. 3.3): the spectral-decay smoothness indicator and the
degree update rule, nested per-element p-hierarchies, the FR operator on a
mesh of mixed polynomial degrees and the per-element transfers between the
levels of such a hierarchy.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle`` (see its header).  The
mixed-degree residual and EJ blocks are ``or_residual_pa`` /
``or_ej_blocks_pa`` in ``fr_oracle.c`` (the face-coupling reading is stated
there); everything here is numpy.

Padded state layout: [nvar][P_max^dim][nelem]; element k of degree deg[k]
uses its first (deg[k] + 1)^dim points, numbered i0 + P_k (i1 + P_k i2); the
remaining entries are zero.
"""
from __future__ import annotations

import ctypes

import numpy as np
from numpy.polynomial import legendre as npleg

from . import Level, _dp, lib, transfer1d

NU_MAX, NU_MIN = 0.2, 0.001   # Sec. 3.3: raise above nu_max eta_max, lower below nu_min eta_max


def _lib():
    L = lib()
    if not hasattr(L, "_pa_ready"):
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.or_residual_pa.argtypes = [ctypes.c_void_p, ip, dp, dp]
        L.or_residual_pa.restype = ctypes.c_int
        L.or_ej_blocks_pa.argtypes = [ctypes.c_void_p, ip, dp, dp, ctypes.c_double, dp]
        L.or_ej_blocks_pa.restype = ctypes.c_int
        L._pa_ready = True
    return L


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ---------------------------------------------------------------------------
# Spectral-decay indicator and degree update (Sec. 3.3)
# ---------------------------------------------------------------------------

def element_indicator(dim: int, P: int, s: np.ndarray) -> float:
    """eta = ||s_p - s_{p-1}|| / ||s_p|| (L2 over the element) for one element of
    P = p + 1 Gauss-Legendre points per direction; s holds the nodal values,
    point index i0 + P (i1 + P i2).  s_p is the element's polynomial in the
    tensor Legendre basis; s_{p-1} keeps the modes of degree <= p - 1 in every
    direction (the tensor space one degree lower), so s_p - s_{p-1} holds the
    modes whose largest index is p.  Reading of the tensor-product case: the
    indicator is defined per element without fixing the truncated space.
    The element's Jacobian is constant and cancels in the ratio."""
    if P < 2:
        raise ValueError("the indicator needs p >= 1")
    xi, _ = npleg.leggauss(P)
    V = npleg.legvander(xi, P - 1)            # V[i, n] = L_n(xi_i)
    Vi = np.linalg.inv(V)
    c = np.asarray(s, dtype=np.float64).reshape((P,) * dim)   # axes (i_{dim-1}, ..., i0)
    for ax in range(dim):
        c = np.moveaxis(np.tensordot(Vi, c, axes=([1], [ax])), 0, ax)
    nrm = 2.0 / (2.0 * np.arange(P) + 1.0)    # ||L_n||^2 on [-1, 1]
    w = nrm
    for _ in range(dim - 1):
        w = np.multiply.outer(nrm, w)
    idx = np.indices((P,) * dim)
    top = idx.max(axis=0) == P - 1
    e_all = float(np.sum(w * c * c))
    e_top = float(np.sum((w * c * c)[top]))
    return float(np.sqrt(e_top / e_all)) if e_all > 0 else 0.0


def indicators(dim: int, deg: np.ndarray, dq: np.ndarray, qinf, var: int = 1) -> np.ndarray:
    """eta_k of every element for the conservative variable var (default the
    x-momentum rho u, Sec. 3.3), from the absolute value q_inf + dq."""
    deg = np.asarray(deg)
    out = np.zeros(deg.shape[0])
    for k in range(deg.shape[0]):
        P = int(deg[k]) + 1
        out[k] = element_indicator(dim, P, qinf[var] + dq[var, :P ** dim, k])
    return out


def adapt_degrees(eta: np.ndarray, deg: np.ndarray, p_max: int, p_min: int = 1,
                  nu_max: float = NU_MAX, nu_min: float = NU_MIN) -> np.ndarray:
    """Sec. 3.3: p + 1 where eta_k > nu_max eta_max, p - 1 where
    eta_k < nu_min eta_max, kept within [p_min, p_max]."""
    emax = float(np.max(eta))
    new = np.asarray(deg, dtype=np.int32).copy()
    new[eta > nu_max * emax] += 1
    new[eta < nu_min * emax] -= 1
    return np.clip(new, p_min, p_max).astype(np.int32)


def nested_degrees(deg: np.ndarray, nlev: int, gap: int) -> list:
    """Per-element degrees on each of nlev p-sublevels for order gap 1 or 2
    (Sec. 3.3).  Reading that reproduces the paper's eight examples (p_max 4,
    3 sublevels): each sublevel lowers the degree by the gap, but keeps at
    least as many degrees as sublevels remain below it, never rises above
    one less than the sublevel above, and stops at 0:
        p_l = max(0, min(p_{l-1} - 1, max(p_0 - gap l, nlev - 1 - l))).
    Gap 2: P4, P3, P2, P1 -> p{4-2-0}, p{3-1-0}, p{2-1-0}, p{1-0-0};
    gap 1: p{4-3-2}, p{3-2-1}, p{2-1-0}, p{1-0-0}."""
    d0 = np.asarray(deg, dtype=np.int64)
    out = [d0.astype(np.int32)]
    for l in range(1, nlev):
        prev = out[-1].astype(np.int64)
        pl = np.minimum(prev - 1, np.maximum(d0 - gap * l, nlev - 1 - l))
        out.append(np.maximum(pl, 0).astype(np.int32))
    return out


# ---------------------------------------------------------------------------
# Mixed-degree level and per-element transfers
# ---------------------------------------------------------------------------

def transfer_pa(x: np.ndarray, dim: int, deg_from: np.ndarray, deg_to: np.ndarray, Pmax_to: int) -> np.ndarray:
    """Per-element L2 projection (Sec. 3.1 Eqs. (projection), (prolongation),
    element by element with each element's pair of degrees) of a padded state
    onto the padded layout of another degree map; equal degrees copy."""
    nv, _, Ne = x.shape
    out = np.zeros((nv, Pmax_to ** dim, Ne))
    for k in range(Ne):
        Pa, Pb = int(deg_from[k]) + 1, int(deg_to[k]) + 1
        xa = x[:, :Pa ** dim, k]
        if Pa == Pb:
            out[:, :Pb ** dim, k] = xa
            continue
        G, _ = transfer1d(Pa, Pb)     # Pb x Pa
        Gd = G
        for _ in range(dim - 1):
            Gd = np.kron(G, Gd)
        out[:, :Pb ** dim, k] = xa @ Gd.T
    return out


class PALevel(Level):
    """FR operator on a periodic mesh with per-element degree deg[k]
    (p-adaptive FR, Sec. 3.3).  P, Np and nb are those of the largest degree
    (the padded layout)."""

    def __init__(self, dim, n, h, deg, gamma, mu, Pr, tau, qinf):
        self.deg = np.ascontiguousarray(np.asarray(deg, dtype=np.int32))
        super().__init__(dim, n, h, int(self.deg.max()), gamma, mu, Pr, tau, qinf)
        if self.deg.shape[0] != self.Ne or self.deg.min() < 0:
            raise ValueError("one degree >= 0 per element")

    def mask(self) -> np.ndarray:
        """True on the entries element k uses, [nv][Np][Ne]."""
        npts = (self.deg.astype(np.int64) + 1) ** self.dim
        m = np.arange(self.Np)[:, None] < npts[None, :]
        return np.broadcast_to(m[None], self.shape).copy()

    def ndof(self) -> int:
        return int(self.nv * np.sum((self.deg.astype(np.int64) + 1) ** self.dim))

    def residual(self, dq: np.ndarray) -> np.ndarray:
        dq = np.ascontiguousarray(dq, dtype=np.float64).reshape(self.shape)
        r = np.empty(self.shape)
        rc = _lib().or_residual_pa(ctypes.byref(self._m), _ip(self.deg), _dp(dq), _dp(r))
        if rc:
            raise ValueError("or_residual_pa failed: %d" % rc)
        return r

    def ej_blocks(self, dq: np.ndarray, sigma: float, r0: np.ndarray | None = None) -> np.ndarray:
        dq = np.ascontiguousarray(dq, dtype=np.float64).reshape(self.shape)
        if r0 is None:
            r0 = self.residual(dq)
        B = np.empty((self.Ne, self.nb, self.nb))
        rc = _lib().or_ej_blocks_pa(ctypes.byref(self._m), _ip(self.deg), _dp(dq),
                                    _dp(np.ascontiguousarray(r0)), float(sigma), _dp(B))
        if rc == -1:
            raise ValueError("EJ colouring needs an even element count per axis")
        if rc:
            raise ValueError("or_ej_blocks_pa failed: %d" % rc)
        return B

    def restrict_to(self, coarse: "PALevel", x: np.ndarray) -> np.ndarray:
        return transfer_pa(x, self.dim, self.deg, coarse.deg, coarse.P)

    def prolong_from(self, coarse: "PALevel", x: np.ndarray) -> np.ndarray:
        return transfer_pa(x, self.dim, coarse.deg, self.deg, self.P)


def hierarchy(dim, n, h, deg, nlev, gap, gamma, mu, Pr, tau, qinf) -> list:
    """The nested p-sublevels of a mixed-degree mesh, finest first."""
    return [PALevel(dim, n, h, d, gamma, mu, Pr, tau, qinf) for d in nested_degrees(deg, nlev, gap)]
