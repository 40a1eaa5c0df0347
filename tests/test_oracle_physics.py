"""Pins of the oracle's pointwise physics against textbook forms written in
absolute (not deviation) variables, at moderate Mach numbers where the
absolute forms lose no digits."""
import ctypes

import numpy as np
import pytest

GAM = 1.4


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def textbook_flux(q, a, dim):
    """Euler flux of absolute conservative q along axis a."""
    rho = q[0]
    u = q[1:1 + dim] / rho
    E = q[dim + 1]
    p = (GAM - 1) * (E - 0.5 * rho * u @ u)
    f = np.zeros(dim + 2)
    f[0] = rho * u[a]
    f[1:1 + dim] = rho * u[a] * u
    f[1 + a] += p
    f[dim + 1] = u[a] * (E + p)
    return f


def prim_to_cons(rho, u, p):
    dim = len(u)
    q = np.zeros(dim + 2)
    q[0] = rho
    q[1:1 + dim] = rho * np.asarray(u)
    q[dim + 1] = p / (GAM - 1) + 0.5 * rho * np.dot(u, u)
    return q


def _inv(orc, dim, a, qinf, dq):
    F = np.zeros(dim + 2)
    orc.lib().or_inviscid_dflux(dim, a, GAM, _dp(qinf), _dp(np.ascontiguousarray(dq)), _dp(F))
    return F


def _roe(orc, dim, a, qinf, dqL, dqR):
    F = np.zeros(dim + 2)
    orc.lib().or_roe_dflux(dim, a, GAM, _dp(qinf), _dp(np.ascontiguousarray(dqL)),
                           _dp(np.ascontiguousarray(dqR)), _dp(F))
    return F


def _states(dim, rng, mach_ref=0.5):
    pinf = 1.0 / (GAM * mach_ref ** 2)
    qinf = prim_to_cons(1.0, [0.7, -0.2, 0.1][:dim], pinf)
    qs = []
    for _ in range(2):
        qs.append(prim_to_cons(1.0 + 0.3 * rng.uniform(-1, 1),
                               list(0.5 * rng.uniform(-1, 1, dim)),
                               pinf * (1 + 0.4 * rng.uniform(-1, 1))))
    return qinf, qs


@pytest.mark.parametrize("dim", [2, 3])
def test_inviscid_deviation_flux_equals_textbook_difference(orc, dim):
    rng = np.random.default_rng(11)
    for _ in range(20):
        qinf, (q, _) = _states(dim, rng)
        for a in range(dim):
            ref = textbook_flux(q, a, dim) - textbook_flux(qinf, a, dim)
            got = _inv(orc, dim, a, qinf, q - qinf)
            assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(textbook_flux(q, a, dim)).max())


def _flux_jacobian(q, a, dim, h=1e-6):
    n = dim + 2
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h * max(1.0, abs(q[j]))
        A[:, j] = (textbook_flux(q + e, a, dim) - textbook_flux(q - e, a, dim)) / (2 * e[j])
    return A


@pytest.mark.parametrize("dim", [2, 3])
def test_roe_dissipation_is_abs_jacobian_at_roe_average(orc, dim):
    """F = (f_L + f_R)/2 - |A(q~)| (q_R - q_L)/2 with A the Euler flux
    Jacobian at the Roe-averaged state, |A| = V |Lambda| V^{-1} from numpy's
    eigen-decomposition."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        qinf, (qL, qR) = _states(dim, rng)
        for a in range(dim):
            sL, sR = np.sqrt(qL[0]), np.sqrt(qR[0])
            uL, uR = qL[1:1 + dim] / qL[0], qR[1:1 + dim] / qR[0]
            pL = (GAM - 1) * (qL[-1] - 0.5 * qL[0] * uL @ uL)
            pR = (GAM - 1) * (qR[-1] - 0.5 * qR[0] * uR @ uR)
            HL, HR = (qL[-1] + pL) / qL[0], (qR[-1] + pR) / qR[0]
            ut = (sL * uL + sR * uR) / (sL + sR)
            Ht = (sL * HL + sR * HR) / (sL + sR)
            rt = sL * sR
            pt = (GAM - 1) / GAM * rt * (Ht - 0.5 * ut @ ut)
            qt = prim_to_cons(rt, list(ut), pt)
            A = _flux_jacobian(qt, a, dim)
            lam, V = np.linalg.eig(A)
            absA = (V @ np.diag(np.abs(lam)) @ np.linalg.inv(V)).real
            ref = 0.5 * (textbook_flux(qL, a, dim) + textbook_flux(qR, a, dim)) \
                - 0.5 * absA @ (qR - qL) - textbook_flux(qinf, a, dim)
            got = _roe(orc, dim, a, qinf, qL - qinf, qR - qinf)
            scale = np.abs(textbook_flux(qL, a, dim)).max()
            assert np.allclose(got, ref, rtol=0, atol=1e-7 * scale)


@pytest.mark.parametrize("dim", [2, 3])
def test_roe_consistency_and_supersonic_upwinding(orc, dim):
    rng = np.random.default_rng(7)
    qinf, (q, q2) = _states(dim, rng)
    for a in range(dim):
        # Roe(q, q) = f(q)
        assert np.allclose(_roe(orc, dim, a, qinf, q - qinf, q - qinf),
                           _inv(orc, dim, a, qinf, q - qinf), rtol=1e-13, atol=1e-12)
        # supersonic along +a: the Roe flux is the left flux exactly (Roe property)
        uL = np.zeros(dim); uL[a] = 4.0
        uR = np.zeros(dim); uR[a] = 4.3
        uR[(a + 1) % dim] = 0.2
        qL = prim_to_cons(1.1, list(uL), 1.0)
        qR = prim_to_cons(0.9, list(uR), 1.2)
        assert np.allclose(_roe(orc, dim, a, qinf, qL - qinf, qR - qinf),
                           textbook_flux(qL, a, dim) - textbook_flux(qinf, a, dim), rtol=1e-12, atol=1e-10)
        # supersonic along -a: the right flux
        qL = prim_to_cons(1.1, list(-uL), 1.0)
        qR = prim_to_cons(0.9, list(-uR), 1.2)
        assert np.allclose(_roe(orc, dim, a, qinf, qL - qinf, qR - qinf),
                           textbook_flux(qR, a, dim) - textbook_flux(qinf, a, dim), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("dim", [2, 3])
def test_viscous_flux_against_primitive_gradients(orc, dim):
    """Viscous flux from conservative gradients equals the textbook form from
    primitive gradients (Newtonian stress, Stokes hypothesis, Fourier heat
    flux with conductivity mu cp / Pr)."""
    mu, Pr = 0.013, 0.72
    rng = np.random.default_rng(3)
    rho = 1.2
    u = rng.uniform(-1, 1, dim)
    p = 3.0
    q = prim_to_cons(rho, list(u), p)
    grho = rng.uniform(-1, 1, dim)
    gu = rng.uniform(-1, 1, (dim, dim))    # gu[b, c] = d u_b / d x_c
    gp = rng.uniform(-1, 1, dim)
    # conservative gradients by the chain rule
    grad = np.zeros((dim, dim + 2))
    for c in range(dim):
        grad[c, 0] = grho[c]
        for b in range(dim):
            grad[c, 1 + b] = grho[c] * u[b] + rho * gu[b, c]
        grad[c, dim + 1] = gp[c] / (GAM - 1) + 0.5 * grho[c] * u @ u + rho * u @ gu[:, c]
    T = p / rho                           # temperature up to the gas constant R
    gT = (gp - T * grho) / rho
    cp = GAM / (GAM - 1)
    qinf = prim_to_cons(1.0, [0.0] * dim, 2.0)
    for a in range(dim):
        div = np.trace(gu)
        tau = np.array([mu * (gu[a, b] + gu[b, a]) - (2 / 3 * mu * div if a == b else 0.0)
                        for b in range(dim)])
        ref = np.concatenate([[0.0], tau, [u @ tau + mu * cp / Pr * gT[a]]])
        F = np.zeros(dim + 2)
        orc.lib().or_viscous_flux(dim, a, GAM, mu, Pr, _dp(qinf), _dp(q - qinf),
                                  _dp(np.ascontiguousarray(grad.reshape(-1))), _dp(F))
        assert np.allclose(F, ref, rtol=1e-12, atol=1e-13)
