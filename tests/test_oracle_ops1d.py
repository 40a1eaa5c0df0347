"""Pins of the oracle's 1D operators and transfer operators against
library routines and closed forms (no call back into the oracle's formulas)."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6])
def test_gauss_legendre_matches_numpy(orc, P):
    o = orc.ops1d(P)
    x, w = npleg.leggauss(P)
    assert np.allclose(o["xi"], x, atol=1e-15, rtol=0)
    assert np.allclose(o["w"], w, atol=1e-15, rtol=0)


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_derivative_and_end_interpolation_exact_on_polynomials(orc, P):
    o = orc.ops1d(P)
    xi = o["xi"]
    for k in range(P):          # all monomials of degree <= p
        f = xi ** k
        df = k * xi ** (k - 1) if k > 0 else np.zeros(P)
        assert np.allclose(o["D"] @ f, df, atol=1e-13)
        assert abs(o["bm"] @ f - (-1.0) ** k) < 1e-13
        assert abs(o["bp"] @ f - 1.0) < 1e-13


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_correction_derivatives_are_dg_liftings(orc, P):
    """Huynh's DG-recovering corrections satisfy, for every phi of degree <= p,
    int g_L' phi = -phi(-1) and int g_R' phi = phi(+1): the FR correction then
    equals the DG lifting of the interface jump (FR = nodal DG on affine
    elements).  Checked with numpy's Legendre basis as test functions."""
    o = orc.ops1d(P)
    xi, w = o["xi"], o["w"]
    for m in range(P):
        c = np.zeros(m + 1)
        c[m] = 1.0
        phi = npleg.legval(xi, c)
        assert abs(np.sum(w * o["gLd"] * phi) + npleg.legval(-1.0, c)) < 1e-13
        assert abs(np.sum(w * o["gRd"] * phi) - npleg.legval(1.0, c)) < 1e-13


def _lagrange_matrix(nodes, x):
    """L[i, j] = l_j(x_i) via numpy polynomial fitting of unit vectors."""
    P = len(nodes)
    V = np.vander(nodes, P)
    out = np.zeros((len(x), P))
    for j in range(P):
        e = np.zeros(P)
        e[j] = 1.0
        coef = np.linalg.solve(V, e)
        out[:, j] = np.polyval(coef, x)
    return out


@pytest.mark.parametrize("P0,P1", [(3, 2), (5, 3), (4, 3), (4, 2), (5, 2), (2, 1), (4, 1), (3, 1)])
def test_transfer_closed_forms(orc, P0, P1):
    G, Pi = orc.transfer1d(P0, P1)
    x0, _ = npleg.leggauss(P0)
    x1, _ = npleg.leggauss(P1)
    # prolongation of a nested space is interpolation
    assert np.allclose(Pi, _lagrange_matrix(x1, x0), atol=1e-14)
    # Gamma Pi = I, Pi Gamma idempotent
    assert np.allclose(G @ Pi, np.eye(P1), atol=1e-14)
    PG = Pi @ G
    assert np.allclose(PG @ PG, PG, atol=1e-14)
    # restriction is Legendre-modal truncation: V1 [I 0] V0^{-1}
    V0 = npleg.legvander(x0, P0 - 1)
    V1 = npleg.legvander(x1, P1 - 1)
    T = np.zeros((P1, P0))
    T[:, :P1] = np.eye(P1)
    assert np.allclose(G, V1 @ T @ np.linalg.inv(V0), atol=1e-13)
    # constants survive restriction
    assert np.allclose(G @ np.ones(P0), np.ones(P1), atol=1e-14)


def test_transfer_tensor_product_reproduces_polynomials(orc):
    """Gamma in 2D/3D reproduces polynomials of degree <= p1 exactly."""
    for dim, P0, P1 in [(2, 5, 3), (3, 4, 3)]:
        x0, _ = npleg.leggauss(P0)
        x1, _ = npleg.leggauss(P1)
        grids0 = np.meshgrid(*([x0] * dim), indexing="ij")
        grids1 = np.meshgrid(*([x1] * dim), indexing="ij")
        # local index x fastest -> reverse the axes when flattening
        f0 = (1 + grids0[0] ** (P1 - 1) * grids0[-1] - 0.3 * grids0[1]).transpose().reshape(-1)
        f1 = (1 + grids1[0] ** (P1 - 1) * grids1[-1] - 0.3 * grids1[1]).transpose().reshape(-1)
        x = np.tile(f0[None, :, None], (dim + 2, 1, 3))
        y = orc.restrict(x, dim, P0, P1)
        assert np.allclose(y[1, :, 2], f1, atol=1e-13)
        back = orc.prolong(y, dim, P0, P1)
        assert np.allclose(back, x, atol=1e-13)
