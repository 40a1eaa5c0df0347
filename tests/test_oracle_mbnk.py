"""Pins of the oracle's MBNK smoother (assembled coarse Jacobian, red-black
block ILU0, GMRES sweep) against brute force and textbook definitions."""
import numpy as np
import pytest

from oracle import mbnk as MB
from oracle import multilevel as ML
from paper_2202_09733_amd import workloads as W
from test_oracle_solver import _dense_newton_stage, _tiny, dense_jacobian


def _dense(A, pattern=False):
    """The assembled operator as a dense matrix in the state layout
    (v*Np + i)*Ne + k; with pattern=True, its block sparsity pattern."""
    L = A.L
    N, nb, Ne = L.N, L.nb, L.Ne
    M = np.zeros((N, N))
    idx = lambda k: np.arange(nb) * Ne + k
    for k in range(Ne):
        M[np.ix_(idx(k), idx(k))] += 1.0 if pattern else A.D[k]
        for a in range(L.dim):
            for s in (-1, 1):
                m = MB.face_neighbour(L, k, a, s)
                M[np.ix_(idx(k), idx(m))] += 1.0 if pattern else A.O[k, MB.slot(a, s)]
    return M != 0.0 if pattern else M


@pytest.fixture(scope="module")
def tiny(orc):
    L, dq, rng = _tiny(orc, n=(6, 4), p=1, seed=31)
    return L, dq, rng, dense_jacobian(L, dq)


def test_jacobian_blocks_are_dense_jacobian_blocks(orc, tiny):
    L, dq, _, J = tiny
    Jb = MB.jacobian_blocks(L, dq)
    idx = lambda k: np.arange(L.nb) * L.Ne + k
    scale = np.abs(J).max()
    for k in range(L.Ne):
        assert np.abs(Jb[k, 0] - J[np.ix_(idx(k), idx(k))]).max() <= 1e-5 * scale
        for a in range(L.dim):
            for s in (-1, 1):
                m = MB.face_neighbour(L, k, a, s)
                assert np.abs(Jb[k, 1 + MB.slot(a, s)] - J[np.ix_(idx(k), idx(m))]).max() <= 1e-5 * scale
    # the diagonal blocks are bitwise the EJ blocks (same single-element perturbations)
    assert np.array_equal(-Jb[:, 0], L.ej_blocks(dq, 0.0) + 0.0)


def test_assembled_matvec_is_dense_product(orc, tiny):
    L, dq, rng, _ = tiny
    A = MB.assemble(L, dq, 25.0)
    x = rng.standard_normal(L.shape)
    assert np.allclose(MB.matvec(A, x).reshape(-1), _dense(A) @ x.reshape(-1), rtol=0, atol=1e-12 * np.abs(x).max()
                       * np.abs(_dense(A)).sum(axis=1).max())


def test_redblack_ilu0_is_textbook_ilu0(orc, tiny):
    """Pointwise ILU(0) (IKJ form, Saad Alg. 10.4) of the dense operator in
    red-black element order, on the block pattern (blocks dense), solved by
    dense triangular substitution, equals the block red-black ILU0 solve."""
    L, dq, rng, _ = tiny
    A = MB.assemble(L, dq, 25.0)
    f = MB.ilu0(A)
    M = _dense(A)
    red = [k for k in range(L.Ne) if MB.red(L, k)]
    black = [k for k in range(L.Ne) if not MB.red(L, k)]
    order = np.concatenate([np.arange(L.nb) * L.Ne + k for k in red + black])
    Mp = M[np.ix_(order, order)]
    pattern = _dense(A, pattern=True)[np.ix_(order, order)]
    n = Mp.shape[0]
    LU = Mp.copy()
    for i in range(1, n):
        for kk in range(i):
            if not pattern[i, kk]:
                continue
            LU[i, kk] /= LU[kk, kk]
            js = np.nonzero(pattern[i, kk + 1:])[0] + kk + 1
            LU[i, js] -= LU[i, kk] * LU[kk, js]
    Lo = np.tril(LU, -1) + np.eye(n)
    Up = np.triu(LU)
    r = rng.standard_normal(L.N)
    z_ref = np.zeros(n)
    z_ref[:] = np.linalg.solve(Up, np.linalg.solve(Lo, r[order]))
    z = MB.ilu0_solve(f, r.reshape(L.shape)).reshape(-1)[order]
    assert np.allclose(z, z_ref, rtol=0, atol=1e-10 * np.abs(z_ref).max())


def test_mbnk_sweep_converged_is_exact_solve(orc, tiny):
    L, dq, rng, _ = tiny
    A = MB.assemble(L, dq, 25.0)
    f = MB.ilu0(A)
    G = rng.standard_normal(L.shape)
    d = MB.mbnk_sweep(f, G, tol=1e-13, maxit=L.N)
    ref = np.linalg.solve(_dense(A), G.reshape(-1))
    assert np.allclose(d.reshape(-1), ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_ml_stage_with_ej_is_the_two_level_stage(orc):
    wl = W.make_bump_workload(n=(4, 4), p0=2, p1=1, Ma=0.2, dt_factor=10.0, seed=12, amp=5e-2)
    L0, L1 = orc.Level(**wl.level_kwargs(2)), orc.Level(**wl.level_kwargs(1))
    q2, s2 = orc.esdirk_stage(L0, L1, wl.dq, wl.dt, wl.a_ii, tol=1e-10)
    qm, sm = ML.esdirk_stage_ml([L0, L1], wl.dq, wl.dt, wl.a_ii, tol=1e-10)
    assert np.array_equal(q2, qm) and s2.gmres_iters == sm.gmres_iters


@pytest.mark.parametrize("ps", [(2, 1), (3, 2, 1)])
def test_stage_with_mbnk_coarse_reaches_newton_root(orc, ps):
    wl = W.make_bump_workload(n=(6, 4), p0=ps[0], p1=ps[1], Ma=0.2, dt_factor=10.0, seed=15, amp=5e-2)
    levels = [orc.Level(**wl.level_kwargs(p)) for p in ps]
    q, st = ML.esdirk_stage_ml(levels, wl.dq, wl.dt, wl.a_ii, coarse="mbnk", tol=1e-11)
    qe, se = ML.esdirk_stage_ml(levels, wl.dq, wl.dt, wl.a_ii, coarse="ej", tol=1e-11)
    assert st.converged and se.converged
    L0 = levels[0]
    qref = _dense_newton_stage(L0, wl.dq, wl.dt, wl.a_ii, lambda x: dense_jacobian(L0, x))
    assert np.linalg.norm(q - qref) <= 1e-8 * np.linalg.norm(qref - wl.dq)
    print("FGMRES with MBNK coarse smoothing %d, with EJ %d" % (st.gmres_iters, se.gmres_iters))
