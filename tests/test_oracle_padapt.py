"""Pins of the oracle's p-adaptation (Sec. 3.3): the spectral-decay
indicator against closed forms and an independent projection route, the
degree update rule, the nested p-hierarchies against the paper's listed
examples, the per-element transfers, and the mixed-degree FR operator
against the uniform one (bitwise on a uniform degree map), free-stream and
conservation, the uniform p_max operator on elements whose lower-degree
neighbours hold polynomials of their own degree, and axis symmetry."""
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from paper_2202_09733_amd import workloads as W

GAM = 1.4
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pa(orc):
    import oracle.padapt as pa
    return pa


def _levels(orc, pa, dim, n, deg, h=None, Ma=0.2, mu=1e-2, tau=0.1, u_dir=(0.8, 0.6, 0.0)):
    qinf, _ = W.reference_state(dim, Ma, u_dir=u_dir)
    if h is None:
        h = [np.full(n[a], 1.0 / n[a]) for a in range(dim)]
    kw = dict(dim=dim, n=n, h=h, gamma=GAM, mu=mu, Pr=0.72, tau=tau, qinf=qinf)
    return pa.PALevel(deg=deg, **kw), kw


def _mixed_deg(dim, n, p_max, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(1, p_max + 1, int(np.prod(n))).astype(np.int32)


# ---------------------------------------------------------------------------
# indicator, update rule, hierarchies
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,p", [(2, 1), (2, 4), (3, 2), (3, 3)])
def test_indicator_vanishes_on_lower_degree_polynomials(pa, dim, p):
    """s in the tensor space of degree p - 1: no energy in the top modes."""
    P = p + 1
    xi, _ = npleg.leggauss(P)
    rng = np.random.default_rng(p)
    c = rng.standard_normal((p,) * dim)               # coefficients of degree <= p - 1
    grids = np.meshgrid(*([xi] * dim), indexing="ij")  # axis a -> coordinate x_a
    s = np.zeros_like(grids[0])
    for idx in np.ndindex(*c.shape):
        term = c[idx]
        for a in range(dim):
            term = term * npleg.legval(grids[a], np.eye(p)[idx[a]])
        s = s + term
    # point index i0 + P (i1 + P i2): x_0 fastest
    s = np.transpose(s, tuple(range(dim))[::-1]).reshape(-1)
    assert pa.element_indicator(dim, P, s) < 1e-13


@pytest.mark.parametrize("dim,p,a", [(2, 2, 0.3), (2, 4, -2.0), (3, 3, 0.05)])
def test_indicator_closed_form(pa, dim, p, a):
    """s = 1 + a L_p(x): eta = |a| ||L_p|| / sqrt(||1||^2 + a^2 ||L_p||^2),
    ||L_n||^2 = 2 / (2n + 1) (the other directions cancel)."""
    P = p + 1
    xi, _ = npleg.leggauss(P)
    i = np.arange(P ** dim)
    x0 = xi[i % P]
    s = 1.0 + a * npleg.legval(x0, np.eye(P)[p])
    nLp = 2.0 / (2 * p + 1)
    want = abs(a) * np.sqrt(nLp) / np.sqrt(2.0 + a * a * nLp)
    assert abs(pa.element_indicator(dim, P, s) - want) < 1e-13
    # a pure top mode carries all the energy
    assert abs(pa.element_indicator(dim, P, npleg.legval(x0, np.eye(P)[p])) - 1.0) < 1e-13


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2)])
def test_indicator_equals_projection_route(orc, pa, dim, p):
    """s_{p-1} is also the L2 projection onto the P - 1 point space and back
    (the pMG transfers), with the norm by the element's Gauss rule."""
    P = p + 1
    rng = np.random.default_rng(11)
    s = rng.standard_normal(P ** dim)
    G, Pi = orc.transfer1d(P, P - 1)
    Gd, Pd = G, Pi
    for _ in range(dim - 1):
        Gd, Pd = np.kron(G, Gd), np.kron(Pi, Pd)
    low = Pd @ (Gd @ s)
    _, w = npleg.leggauss(P)
    wd = w
    for _ in range(dim - 1):
        wd = np.kron(w, wd)
    want = np.sqrt(np.sum(wd * (s - low) ** 2) / np.sum(wd * s * s))
    assert abs(pa.element_indicator(dim, P, s) - want) < 1e-12


def test_adapt_rule(pa):
    eta = np.array([1.0, 0.25, 0.2, 0.1, 0.002, 0.0009, 0.0, 0.5])
    deg = np.array([4, 2, 2, 3, 1, 2, 1, 4], dtype=np.int32)
    new = pa.adapt_degrees(eta, deg, p_max=4)
    # > 0.2 eta_max: +1 (capped at 4); < 0.001 eta_max: -1 (floored at 1)
    assert new.tolist() == [4, 3, 2, 3, 1, 1, 1, 4]


def test_nested_hierarchies_match_the_papers_examples(pa):
    rows = np.loadtxt(os.path.join(HERE, "golden", "nested_hierarchies.txt"), dtype=int)
    for gap in (1, 2):
        sel = rows[rows[:, 0] == gap]
        levels = pa.nested_degrees(sel[:, 1], 3, gap)
        got = np.stack(levels, axis=1)
        assert got.tolist() == sel[:, 2:].tolist(), gap


def test_transfers(orc, pa):
    rng = np.random.default_rng(3)
    dim, n = 2, (4, 4)
    deg = _mixed_deg(dim, n, 4, 1)
    qinf, _ = W.reference_state(dim, 0.2)
    x = W.random_state_pa(deg, dim, rng, qinf)
    up = np.minimum(deg + 1, 5).astype(np.int32)
    y = pa.transfer_pa(x, dim, deg, up, 6)
    # raising is exact, lowering back recovers the state
    back = pa.transfer_pa(y, dim, up, deg, 5)
    assert np.abs(back - x).max() < 1e-13 * np.abs(x).max()
    # lowering keeps each element's mean (constants are in every space)
    dn = np.maximum(deg - 1, 0).astype(np.int32)
    z = pa.transfer_pa(x, dim, deg, dn, 4)
    for k in range(deg.shape[0]):
        for src, d in ((x, deg[k]), (z, dn[k])):
            P = int(d) + 1
            _, w = npleg.leggauss(P)
            wd = np.kron(w, w)
            m = src[:, :P * P, k] @ wd
            if src is x:
                m0 = m
        assert np.allclose(m, m0, rtol=0, atol=1e-13 * np.abs(m0).max())
    # equal degrees copy bit for bit
    assert np.array_equal(pa.transfer_pa(x, dim, deg, deg, 5), x)


# ---------------------------------------------------------------------------
# mixed-degree operator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,p", [(2, (4, 6), 3), (3, (2, 2, 4), 2)])
def test_uniform_degree_map_is_bitwise_uniform(orc, pa, dim, n, p):
    deg = np.full(int(np.prod(n)), p, dtype=np.int32)
    L, kw = _levels(orc, pa, dim, n, deg)
    U = orc.Level(p=p, **kw)
    rng = np.random.default_rng(5)
    dq = W.random_state(U.shape, rng, U.qinf, amp=0.05)
    assert np.array_equal(L.residual(dq), U.residual(dq))
    assert np.array_equal(L.ej_blocks(dq, 7.0), U.ej_blocks(dq, 7.0))


@pytest.mark.parametrize("dim,n,pm", [(2, (4, 4), 4), (3, (2, 2, 2), 3)])
def test_mixed_other_uniform_state_is_steady(orc, pa, dim, n, pm):
    deg = _mixed_deg(dim, n, pm, 2)
    L, _ = _levels(orc, pa, dim, n, deg)
    dq = np.zeros(L.shape)
    dq[0], dq[1], dq[dim + 1] = 0.05, -0.1, 3.0
    dq *= L.mask()
    r = L.residual(dq)
    assert np.abs(r).max() < 1e-10
    assert np.all(r[~L.mask()] == 0.0)


@pytest.mark.parametrize("dim,n,pm,seed", [(2, (6, 4), 4, 0), (2, (4, 4), 3, 1), (3, (2, 4, 2), 3, 2)])
def test_mixed_discrete_conservation(orc, pa, dim, n, pm, seed):
    """sum_e sum_i w_i |J_e| R = 0 per variable: the mortar returns the
    common flux to both sides by L2 projection, which keeps its face
    integral."""
    rng = np.random.default_rng(seed)
    h = [rng.uniform(0.05, 0.2, n[a]) for a in range(dim)]
    deg = _mixed_deg(dim, n, pm, seed + 10)
    L, _ = _levels(orc, pa, dim, n, deg, h=h)
    dq = W.random_state_pa(deg, dim, rng, L.qinf, amp=0.05)
    r = L.residual(dq)
    e = np.arange(L.Ne)
    ec = [e % n[0], (e // n[0]) % n[1]] + ([e // (n[0] * n[1])] if dim == 3 else [])
    tot = np.zeros(L.nv)
    for k in range(L.Ne):
        P = int(deg[k]) + 1
        _, w = npleg.leggauss(P)
        wd = w
        for _ in range(dim - 1):
            wd = np.kron(w, wd)
        jac = np.prod([h[a][ec[a][k]] / 2 for a in range(dim)])
        tot += jac * (r[:, :P ** dim, k] @ wd)
    scale = np.abs(r).max() * float(np.prod([np.sum(h[a]) for a in range(dim)])) * 4
    assert np.all(np.abs(tot) < 1e-14 * scale), tot / scale


def _embed_low_as_polynomials(orc, pa, dim, deg, dq_pa, Pm):
    """The same state on the uniform p_max mesh: each element's polynomial
    interpolated to the p_max points (exact)."""
    full = np.maximum(deg, deg.max()).astype(np.int32)
    return pa.transfer_pa(dq_pa, dim, deg, full, Pm)


@pytest.mark.parametrize("dim,n,viscous", [(2, (6, 6), True), (2, (6, 6), False), (3, (4, 4, 4), True)])
def test_high_elements_see_the_uniform_operator(orc, pa, dim, n, viscous):
    """Where every lower-degree element holds a polynomial of its own degree,
    the mixed operator on a p_max element equals the uniform p_max operator
    applied to the same polynomials -- whenever the element's -axis
    neighbours are p_max too (their gradient traces are then the same);
    without viscosity on every p_max element.  This fixes the mortar at the
    larger degree and the interpolation of the lower side's traces."""
    pm = 3
    rng = np.random.default_rng(21 + dim)
    deg = np.random.default_rng(30 + dim).choice([1, 2, pm], size=int(np.prod(n)), p=[0.15, 0.15, 0.7])
    deg = deg.astype(np.int32)
    mu, tau = (1e-2, 0.1) if viscous else (0.0, 0.0)
    L, kw = _levels(orc, pa, dim, n, deg, mu=mu, tau=tau)
    U = orc.Level(p=pm, **kw)
    dq = W.random_state_pa(deg, dim, rng, L.qinf, amp=0.05)
    r = L.residual(dq)
    ru = U.residual(_embed_low_as_polynomials(orc, pa, dim, deg, dq, pm + 1))
    e = np.arange(L.Ne)
    ec = [e % n[0], (e // n[0]) % n[1]] + ([e // (n[0] * n[1])] if dim == 3 else [])
    checked = 0
    for k in range(L.Ne):
        if deg[k] != pm:
            continue
        if viscous:
            ok = True
            for a in range(dim):
                c = [ec[b][k] for b in range(dim)]
                c[a] = (c[a] - 1) % n[a]
                km = c[0] + n[0] * (c[1] + (n[1] * c[2] if dim == 3 else 0))
                ok &= deg[km] == pm
            if not ok:
                continue
        checked += 1
        assert np.allclose(r[:, :, k], ru[:, :, k], rtol=0, atol=1e-11 * np.abs(ru).max()), k
    assert checked >= 2
    # and the lower-degree elements do differ (the check is not vacuous)
    low = deg < pm
    assert np.abs(r[:, :, low] - pa.transfer_pa(ru, dim, np.full_like(deg, pm), deg, pm + 1)[:, :, low]).max() > 1e-6


def _swap_xy_pa(dq, deg, n):
    """Transpose a padded 2D state: (x, y) -> (y, x), rho u <-> rho v, and the
    element's own points i0 + P i1 -> i1 + P i0."""
    nv, Npm, Ne = dq.shape
    out = np.zeros_like(dq)
    for k in range(Ne):
        ix, iy = k % n, k // n
        k2 = iy + n * ix
        P = int(deg[k]) + 1
        a = dq[:, :P * P, k].reshape(nv, P, P).transpose(0, 2, 1)[[0, 2, 1, 3]]
        out[:, :P * P, k2] = a.reshape(nv, P * P)
    return out


def test_mixed_axis_swap_symmetry(orc, pa):
    nn = 6
    deg = _mixed_deg(2, (nn, nn), 4, 7)
    deg2 = deg.reshape(nn, nn).T.reshape(-1).copy()
    Lx, _ = _levels(orc, pa, 2, (nn, nn), deg, u_dir=(0.6, 0.8, 0.0))
    Ly, _ = _levels(orc, pa, 2, (nn, nn), deg2, u_dir=(0.8, 0.6, 0.0))
    rng = np.random.default_rng(9)
    dq = W.random_state_pa(deg, 2, rng, Lx.qinf, amp=0.05)
    r = Lx.residual(dq)
    r2 = Ly.residual(_swap_xy_pa(dq, deg, nn))
    assert np.allclose(r2, _swap_xy_pa(r, deg, nn), rtol=0, atol=1e-12 * np.abs(r).max())


def _cycle_xyz_pa(dq, deg, n):
    """(x, y, z) -> (y, z, x) on an n^3 mesh (new x = old y, ...)."""
    nv, Npm, Ne = dq.shape
    out = np.zeros_like(dq)
    for k in range(Ne):
        ix, iy, iz = k % n, (k // n) % n, k // (n * n)
        k2 = iy + n * (iz + n * ix)
        P = int(deg[k]) + 1
        a = dq[:, :P ** 3, k].reshape(nv, P, P, P)          # [v][i2][i1][i0]
        a = a.transpose(0, 3, 1, 2)[[0, 2, 3, 1, 4]]         # new [i2'=i0][i1'=i2][i0'=i1]
        out[:, :P ** 3, k2] = a.reshape(nv, P ** 3)
    return out


def test_mixed_axis_cycle_symmetry_3d(orc, pa):
    nn = 2
    deg = _mixed_deg(3, (nn, nn, nn), 3, 8)
    deg2 = np.zeros_like(deg)
    for k in range(deg.shape[0]):
        ix, iy, iz = k % nn, (k // nn) % nn, k // (nn * nn)
        deg2[iy + nn * (iz + nn * ix)] = deg[k]
    La, _ = _levels(orc, pa, 3, (nn, nn, nn), deg, u_dir=(0.48, 0.6, 0.64))
    Lb, _ = _levels(orc, pa, 3, (nn, nn, nn), deg2, u_dir=(0.6, 0.64, 0.48))
    rng = np.random.default_rng(10)
    dq = W.random_state_pa(deg, 3, rng, La.qinf, amp=0.05)
    r = La.residual(dq)
    r2 = Lb.residual(_cycle_xyz_pa(dq, deg, nn))
    assert np.allclose(r2, _cycle_xyz_pa(r, deg, nn), rtol=0, atol=1e-12 * np.abs(r).max())


def test_mixed_ej_blocks_brute_force(orc, pa):
    """Columns of B_k against perturbing element k alone in the full
    mixed-degree residual; padded rows and columns are the identity."""
    dim, n = 2, (4, 4)
    deg = _mixed_deg(dim, n, 3, 4)
    L, _ = _levels(orc, pa, dim, n, deg)
    rng = np.random.default_rng(6)
    dq = W.random_state_pa(deg, dim, rng, L.qinf, amp=0.05)
    sig = 5.0
    B = L.ej_blocks(dq, sig)
    r0 = L.residual(dq)
    Np = L.Np
    for k in (0, 5, 10):
        Npk = (int(deg[k]) + 1) ** dim
        for j in (0, Npk - 1, Np + 1, 3 * Np + Npk - 1):
            v, i = divmod(j, Np)
            qp = dq.copy()
            hj = 1e-7 * max(1.0, abs(L.qinf[v] + dq[v, i, k]))
            qp[v, i, k] = dq[v, i, k] + hj
            hact = qp[v, i, k] - dq[v, i, k]
            col = -(L.residual(qp)[:, :, k] - r0[:, :, k]).reshape(-1) / hact
            col[j] += sig
            valid = (np.arange(L.nb) % Np) < Npk
            assert np.array_equal(B[k][valid, j], col[valid])
        pad = np.where((np.arange(L.nb) % Np) >= Npk)[0]
        if pad.size:
            sub = B[k][np.ix_(pad, np.arange(L.nb))]
            assert np.array_equal(sub, np.eye(L.nb)[pad])
            assert np.all(B[k][np.ix_(np.setdiff1d(np.arange(L.nb), pad), pad)] == 0.0)


def test_mixed_row_stage_converges(orc, pa):
    """The oracle's ROW stage on a mixed-degree mesh with the EJ and the
    nested two-level pMG preconditioners reaches 1e-8 in the recomputed
    residual."""
    wl = W.make_padapt_workload(n=(8, 8), p_max=4, dt_factor=100.0, ring=0.2)
    deg = wl.extra["deg"]
    assert len(np.unique(deg)) >= 3
    kw = dict(dim=2, n=wl.n, h=wl.h, gamma=wl.gamma, mu=wl.mu, Pr=wl.Pr, tau=wl.tau, qinf=wl.qinf)
    levels = pa.hierarchy(kw["dim"], kw["n"], kw["h"], deg, 2, 2, kw["gamma"], kw["mu"], kw["Pr"], kw["tau"],
                          kw["qinf"])
    its = {}
    for prec in ("ej", "pmg"):
        Y, st = orc.row_stage(levels[0], levels[1], wl.dq, wl.dt, wl.a_ii, precond=prec, tol=1e-8)
        assert st.converged and st.rel_res <= 1e-8, (prec, st.rel_res)
        assert np.all(Y[~levels[0].mask()] == 0.0)
        its[prec] = st.gmres_iters
    assert its["pmg"] < its["ej"], its
