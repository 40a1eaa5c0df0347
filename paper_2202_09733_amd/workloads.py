"""Seeded synthetic inputs for the stage-solve workloads.

This module only builds meshes, reference states, smooth initial fields and
stage parameters.  It holds none of the method's arithmetic (no residual, no
operator, no solver) and is the one module that both the GPU path's tests and
the CPU oracle's tests draw their inputs from.

States are returned as deviations dq = q - q_inf of the conservative variables
(rho, rho u, rho v, [rho w], E) from the reference state, laid out
[nvar][npts][nelem] with element index e = ix + nx (iy + ny iz) and local
point i = a + P (b + P c) (x fastest), at the Gauss-Legendre points of each
element (numpy's ``leggauss``).

Workload recipes (the paper's meshes and spin-up solutions are not available,
so these stand in for the stiffness of its cases: low Mach number and
high-aspect-ratio elements):

* ``bumps_8x8_p2``      periodic 8x8 on [0,1]^2, p{2-1}, Re 1000, Ma 0.1, freestream
  (1, 1, 0) plus four periodic Gaussian bumps (sigma 0.08, centres U[0,1)^2,
  amplitudes U(-1e-2, 1e-2) for rho, u, v independently), p = p_inf; one
  ESDIRK3 stage, dt = 10 dt_exp.
* ``vortical_64x64_p4`` 64x64, x uniform on [0,1], y geometric h_y,j = h_x 100^((j-63)/63)
  (aspect ratio 100 -> 1), p{4-2}, Ma 1e-3, Re 1000; u = 1 + u', v = v' from a
  random streamfunction with |kx|,|ky| <= 4, amplitudes N(0,1)/|k|^2, phases
  U[0, 2pi), scaled to max |u'| = 1e-3; rho = 1, p = p_inf; ESDIRK3 stage,
  dt = 1000 dt_exp.
* ``tgv_32cubed_p3``    periodic 32^3 on [0, 2pi)^3, p{3-2}, Re 1600, Ma 0.1,
  Taylor-Green vortex plus N(0,1) 1e-3 noise on u, v, w; first ROW stage
  (gamma 0.25), dt = 100 dt_exp.

dt_exp = h_min / ((|u|_max + c_inf)(2p + 1)) is a fixed reference convention
(the paper defines no CFL number, Sec. 2.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4
PRANDTL = 0.72
LDG_TAU = 0.1
# L-stable ESDIRK3 diagonal coefficient: root of 6 g^3 - 18 g^2 + 9 g - 1 = 0
ESDIRK3_GAMMA = 0.43586652150845899942
ROW_GAMMA = 0.25



@dataclass
class Workload:
    name: str
    dim: int
    n: tuple
    h: list                  # element widths per axis
    p0: int                  # fine degree
    p1: int                  # coarse degree
    gamma: float
    mu: float
    Pr: float
    tau: float
    qinf: np.ndarray         # conservative reference state
    dq: np.ndarray           # initial state deviation at the fine level
    dt: float
    a_ii: float
    scheme: str              # "esdirk" or "row"
    Ma: float
    Re: float
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def Ne(self):
        return int(np.prod(self.n))

    @property
    def nv(self):
        return self.dim + 2

    def level_kwargs(self, p):
        return dict(dim=self.dim, n=self.n, h=self.h, p=p, gamma=self.gamma, mu=self.mu,
                    Pr=self.Pr, tau=self.tau, qinf=self.qinf)

    def dof(self, p=None):
        p = self.p0 if p is None else p
        return self.nv * (p + 1) ** self.dim * self.Ne


def reference_state(dim: int, Ma: float, u_dir=(1.0, 0.0, 0.0), speed=1.0):
    """rho = 1, |u| = speed (components u_dir), p = 1/(gamma Ma^2)."""
    pinf = 1.0 / (GAMMA * Ma * Ma)
    u = np.array(u_dir[:dim], dtype=np.float64) * speed
    q = np.zeros(dim + 2)
    q[0] = 1.0
    q[1:1 + dim] = u
    q[dim + 1] = pinf / (GAMMA - 1.0) + 0.5 * float(u @ u)
    return q, pinf


def point_coords(n, h, p, dim):
    """Physical coordinates of the Gauss-Legendre points, each [Np][Ne]."""
    P = p + 1
    xi, _ = np.polynomial.legendre.leggauss(P)
    coords = []
    edges = [np.concatenate([[0.0], np.cumsum(h[a])]) for a in range(dim)]
    Ne = int(np.prod(n))
    Np = P ** dim
    e = np.arange(Ne)
    ec = [e % n[0], (e // n[0]) % n[1]] + ([e // (n[0] * n[1])] if dim == 3 else [])
    i = np.arange(Np)
    ic = [i % P, (i // P) % P] + ([i // (P * P)] if dim == 3 else [])
    for a in range(dim):
        left = edges[a][ec[a]]                  # [Ne]
        width = np.asarray(h[a])[ec[a]]         # [Ne]
        s = (xi[ic[a]] + 1.0) * 0.5             # [Np]
        coords.append(left[None, :] + s[:, None] * width[None, :])
    return coords


def deviation_from_primitives(qinf, pinf, rho, vel, p):
    """dq = q - q_inf for rho, velocity list and pressure arrays, written so
    that no p_inf-sized term is formed."""
    dim = len(vel)
    rinf = qinf[0]
    uinf = qinf[1:1 + dim] / rinf
    dq = np.zeros((dim + 2,) + rho.shape)
    dq[0] = rho - rinf
    kin = np.zeros_like(rho)
    kin_inf = 0.0
    for b in range(dim):
        dq[1 + b] = rho * vel[b] - rinf * uinf[b]
        kin += rho * vel[b] * vel[b]
        kin_inf += rinf * uinf[b] * uinf[b]
    dq[dim + 1] = (p - pinf) / (GAMMA - 1.0) + 0.5 * (kin - kin_inf)
    return np.ascontiguousarray(dq)


def _gaussian_bumps(rng, X, Y, n_bumps=4, sigma=0.08, amp=1e-2):
    """Sum of periodic (minimum-image) Gaussians on the unit square, one set
    of amplitudes per field rho, u, v."""
    centres = rng.uniform(0.0, 1.0, size=(n_bumps, 2))
    amps = rng.uniform(-amp, amp, size=(3, n_bumps))
    fields = [np.zeros_like(X) for _ in range(3)]
    for b in range(n_bumps):
        dx = X - centres[b, 0]
        dy = Y - centres[b, 1]
        dx -= np.round(dx)
        dy -= np.round(dy)
        g = np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))
        for f in range(3):
            fields[f] += amps[f, b] * g
    return fields


def make_bump_workload(n=(8, 8), p0=2, p1=1, Ma=0.1, Re=1000.0, seed=1, dt_factor=10.0,
                       scheme="esdirk", name="bumps", amp=1e-2):
    """2D periodic unit square, uniform elements, Gaussian bumps (the recipe of ``bumps_8x8_p2``)."""
    dim = 2
    h = [np.full(n[0], 1.0 / n[0]), np.full(n[1], 1.0 / n[1])]
    rng = np.random.default_rng(seed)
    qinf, pinf = reference_state(dim, Ma)
    X, Y = point_coords(n, h, p0, dim)
    br, bu, bv = _gaussian_bumps(rng, X, Y, amp=amp)
    rho = 1.0 + br
    u = 1.0 + bu
    v = bv
    p = np.full_like(X, pinf)
    dq = deviation_from_primitives(qinf, pinf, rho, [u, v], p)
    c = math.sqrt(GAMMA * pinf)
    hmin = min(float(np.min(h[0])), float(np.min(h[1])))
    dt_exp = hmin / ((1.0 + c) * (2 * p0 + 1))
    a_ii = ESDIRK3_GAMMA if scheme == "esdirk" else ROW_GAMMA
    return Workload(name=name, dim=dim, n=tuple(n), h=h, p0=p0, p1=p1, gamma=GAMMA, mu=1.0 / Re,
                    Pr=PRANDTL, tau=LDG_TAU, qinf=qinf, dq=dq, dt=dt_factor * dt_exp, a_ii=a_ii,
                    scheme=scheme, Ma=Ma, Re=Re, seed=seed, extra=dict(dt_exp=dt_exp))


def stretched_widths(nx, ny, ratio=100.0):
    """h_x uniform 1/nx; h_y,j = h_x ratio^((j - (ny-1))/(ny-1))."""
    hx = np.full(nx, 1.0 / nx)
    j = np.arange(ny)
    hy = (1.0 / nx) * ratio ** ((j - (ny - 1)) / (ny - 1))
    return [hx, hy]


def make_vortical_workload(n=(64, 64), p0=4, p1=2, Ma=1e-3, Re=1000.0, seed=2, dt_factor=1000.0,
                           amp=1e-3, kmax=4, ratio=100.0, scheme="esdirk", name="vortical"):
    """2D y-stretched periodic mesh with a smooth random vortical perturbation
    (the recipe of ``vortical_64x64_p4``)."""
    dim = 2
    h = stretched_widths(n[0], n[1], ratio)
    Lx = float(np.sum(h[0]))
    Ly = float(np.sum(h[1]))
    rng = np.random.default_rng(seed)
    qinf, pinf = reference_state(dim, Ma)
    X, Y = point_coords(n, h, p0, dim)
    up = np.zeros_like(X)
    vp = np.zeros_like(X)
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if kx == 0 and ky == 0:
                continue
            A = rng.normal() / (kx * kx + ky * ky)
            phi = rng.uniform(0.0, 2.0 * math.pi)
            arg = 2.0 * math.pi * (kx * X / Lx + ky * Y / Ly) + phi
            s = -A * np.sin(arg)
            up += s * (2.0 * math.pi * ky / Ly)      # d psi / dy
            vp -= s * (2.0 * math.pi * kx / Lx)      # -d psi / dx
    scale = amp / float(np.max(np.sqrt(up * up + vp * vp)))
    up *= scale
    vp *= scale
    rho = np.ones_like(X)
    p = np.full_like(X, pinf)
    dq = deviation_from_primitives(qinf, pinf, rho, [1.0 + up, vp], p)
    c = math.sqrt(GAMMA * pinf)
    hmin = min(float(np.min(h[0])), float(np.min(h[1])))
    dt_exp = hmin / ((1.0 + c) * (2 * p0 + 1))
    a_ii = ESDIRK3_GAMMA if scheme == "esdirk" else ROW_GAMMA
    return Workload(name=name, dim=dim, n=tuple(n), h=h, p0=p0, p1=p1, gamma=GAMMA, mu=1.0 / Re,
                    Pr=PRANDTL, tau=LDG_TAU, qinf=qinf, dq=dq, dt=dt_factor * dt_exp, a_ii=a_ii,
                    scheme=scheme, Ma=Ma, Re=Re, seed=seed, extra=dict(dt_exp=dt_exp))


def make_tgv_workload(n=(32, 32, 32), p0=3, p1=2, Ma=0.1, Re=1600.0, seed=4, dt_factor=100.0,
                      noise=1e-3, scheme="row", name="tgv"):
    """3D periodic [0, 2pi)^3 Taylor-Green vortex plus seeded velocity noise
    (the recipe of ``tgv_32cubed_p3``)."""
    dim = 3
    L = 2.0 * math.pi
    h = [np.full(n[a], L / n[a]) for a in range(3)]
    rng = np.random.default_rng(seed)
    qinf, pinf = reference_state(dim, Ma, u_dir=(0.0, 0.0, 0.0))
    X, Y, Z = point_coords(n, h, p0, dim)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(X)
    nz = rng.standard_normal((3,) + X.shape) * noise
    u = u + nz[0]
    v = v + nz[1]
    w = w + nz[2]
    rho = np.ones_like(X)
    p = pinf + (1.0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    dq = deviation_from_primitives(qinf, pinf, rho, [u, v, w], p)
    c = math.sqrt(GAMMA * pinf)
    hmin = float(np.min(h[0]))
    dt_exp = hmin / ((1.0 + c) * (2 * p0 + 1))
    a_ii = ROW_GAMMA if scheme == "row" else ESDIRK3_GAMMA
    return Workload(name=name, dim=dim, n=tuple(n), h=h, p0=p0, p1=p1, gamma=GAMMA, mu=1.0 / Re,
                    Pr=PRANDTL, tau=LDG_TAU, qinf=qinf, dq=dq, dt=dt_factor * dt_exp, a_ii=a_ii,
                    scheme=scheme, Ma=Ma, Re=Re, seed=seed, extra=dict(dt_exp=dt_exp))


def bumps_8x8_p2():
    return make_bump_workload(name="2D NS FR periodic 8x8 p=2, Ma 0.1, ESDIRK3 stage")


def vortical_64x64_p4():
    return make_vortical_workload(
        name="2D NS FR 64x64 y-stretched (AR 1-100) p=4, Ma 1e-3, ESDIRK3 stage, CFL~1000")


def tgv_32cubed_p3():
    return make_tgv_workload(name="3D NS FR periodic 32^3 p=3 TGV, Ma 0.1, ROW stage")


def random_state(level_shape, rng, qinf, amp=1e-2):
    """A rough random state (i.i.d. perturbations of rho, velocity and
    pressure) for operator-level tests."""
    nv, Np, Ne = level_shape
    dim = nv - 2
    pinf = (GAMMA - 1.0) * (qinf[dim + 1] - 0.5 * float(qinf[1:1 + dim] @ qinf[1:1 + dim]) / qinf[0])
    rho = 1.0 + amp * rng.uniform(-1, 1, (Np, Ne))
    uinf = qinf[1:1 + dim] / qinf[0]
    vel = [uinf[b] + amp * rng.uniform(-1, 1, (Np, Ne)) for b in range(dim)]
    p = pinf * (1.0 + amp * rng.uniform(-1, 1, (Np, Ne)))
    return deviation_from_primitives(qinf, pinf, rho, vel, p)


# ---------------------------------------------------------------------------
# mixed polynomial degrees (p-adaptive meshes)
# ---------------------------------------------------------------------------

def degree_rings(n, p_max, p_min=1, centre=(0.5, 0.5, 0.5), ring=0.125):
    """A synthetic p-adaptive degree map on the unit box: p_max on elements
    whose centre lies within `ring` of `centre` (periodic distance), one degree
    less per further `ring` of distance, down to p_min -- the high degrees
    sit on a localised feature, as the smoothness indicator puts them."""
    dim = len(n)
    Ne = int(np.prod(n))
    e = np.arange(Ne)
    ec = [e % n[0], (e // n[0]) % n[1]] + ([e // (n[0] * n[1])] if dim == 3 else [])
    d2 = np.zeros(Ne)
    for a in range(dim):
        x = (ec[a] + 0.5) / n[a]
        dx = np.abs(x - centre[a])
        dx = np.minimum(dx, 1.0 - dx)
        d2 += dx * dx
    deg = p_max - np.floor(np.sqrt(d2) / ring).astype(np.int64)
    return np.clip(deg, p_min, p_max).astype(np.int32)


def random_state_pa(deg, dim, rng, qinf, amp=1e-2):
    """random_state on a mixed-degree mesh, padded [nvar][P_max^dim][nelem]:
    element k's first (deg[k] + 1)^dim points hold values, the rest zero."""
    deg = np.asarray(deg)
    Pm = int(deg.max()) + 1
    full = random_state((dim + 2, Pm ** dim, deg.shape[0]), rng, qinf, amp)
    npts = (deg.astype(np.int64) + 1) ** dim
    mask = np.arange(Pm ** dim)[:, None] < npts[None, :]
    return np.ascontiguousarray(full * mask[None])


def sample_pa(deg, n, h, dim, fn):
    """Evaluate fn(coords) -> [nvar][npts] arrays at every element's own
    Gauss-Legendre points, padded to the largest degree."""
    deg = np.asarray(deg)
    Pm = int(deg.max()) + 1
    out = None
    for p in np.unique(deg):
        X = point_coords(n, h, int(p), dim)
        vals = fn(X)
        if out is None:
            out = np.zeros((vals.shape[0], Pm ** dim, deg.shape[0]))
        sel = deg == p
        out[:, :(int(p) + 1) ** dim, sel] = vals[:, :, sel]
    return np.ascontiguousarray(out)


def make_padapt_workload(n=(32, 32), p_max=4, Ma=0.1, Re=1000.0, seed=6, dt_factor=100.0, amp=5e-2,
                         kmax=4, ring=0.125, uniform=False, name="p-adaptive vortical"):
    """2D periodic unit square with the vortical perturbation of
    ``make_vortical_workload`` (uniform elements, |u'| <= amp) and the
    degree map ``degree_rings`` (p_max at the centre down to 1); each element
    holds the field at its own points.  First ROW stage.  uniform=True: the
    same mesh, field and step with p_max on every element."""
    dim = 2
    h = [np.full(n[a], 1.0 / n[a]) for a in range(dim)]
    rng = np.random.default_rng(seed)
    qinf, pinf = reference_state(dim, Ma)
    modes = []
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if kx == 0 and ky == 0:
                continue
            modes.append((kx, ky, rng.normal() / (kx * kx + ky * ky), rng.uniform(0.0, 2.0 * math.pi)))

    def vel(X, Y):
        up = np.zeros_like(X)
        vp = np.zeros_like(X)
        for kx, ky, A, phi in modes:
            s = -A * np.sin(2.0 * math.pi * (kx * X + ky * Y) + phi)
            up += s * (2.0 * math.pi * ky)
            vp -= s * (2.0 * math.pi * kx)
        return up, vp

    Xf, Yf = point_coords(n, h, p_max, dim)
    u0, v0 = vel(Xf, Yf)
    scale = amp / float(np.max(np.sqrt(u0 * u0 + v0 * v0)))
    deg = degree_rings(n, p_max, ring=ring)
    if uniform:
        deg = np.full_like(deg, p_max)

    def field(X):
        up, vp = vel(X[0], X[1])
        rho = np.ones_like(X[0])
        return deviation_from_primitives(qinf, pinf, rho, [1.0 + scale * up, scale * vp], np.full_like(X[0], pinf))

    dq = sample_pa(deg, n, h, dim, field)
    c = math.sqrt(GAMMA * pinf)
    dt_exp = float(h[0][0]) / ((1.0 + amp + c) * (2 * p_max + 1))
    return Workload(name=name, dim=dim, n=tuple(n), h=h, p0=p_max, p1=max(p_max - 2, 0), gamma=GAMMA,
                    mu=1.0 / Re, Pr=PRANDTL, tau=LDG_TAU, qinf=qinf, dq=dq, dt=dt_factor * dt_exp,
                    a_ii=ROW_GAMMA, scheme="row", Ma=Ma, Re=Re, seed=seed, extra=dict(dt_exp=dt_exp, deg=deg))
