"""Pins of the FP64 oracle of the learned coarse correction: gradients against
central differences, exact positive homogeneity and oddness, the feature
layout against per-element constant fields, bf16 rounding against torch, the
mirrored evaluation's geometry entries and the learned coarse step against
closed forms of hand-built networks, Adam against torch.optim.Adam and its
constant-gradient closed form, and the learned V-cycle against the pinned
plain V-cycle."""
import numpy as np
import pytest
import torch

from oracle import mlp


def _net(rng, nin=12, nh=16, nout_pad=8):
    return [rng.standard_normal((nh, nin)) / 3, rng.standard_normal((nh, nh)) / 4,
            rng.standard_normal((nout_pad, nh)) / 4]


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    Ws = _net(rng)
    X = rng.standard_normal((10, 12))
    T = rng.standard_normal((10, 8))
    nout = 5
    _, g = mlp.loss_grad(Ws, X, T, nout)
    h = 1e-6
    for l in range(3):
        for _ in range(25):
            i = rng.integers(Ws[l].shape[0])
            j = rng.integers(Ws[l].shape[1])
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (mlp.loss_grad(Wp, X, T, nout)[0] - mlp.loss_grad(Wm, X, T, nout)[0]) / (2 * h)
            assert abs(fd - g[l][i, j]) <= 1e-7 * max(1.0, abs(fd))


def test_padded_outputs_carry_no_gradient():
    rng = np.random.default_rng(1)
    Ws = _net(rng)
    X = rng.standard_normal((6, 12))
    T = rng.standard_normal((6, 8))
    _, g = mlp.loss_grad(Ws, X, T, 5)
    assert np.all(g[2][5:] == 0.0)


def test_homogeneity_and_oddness():
    rng = np.random.default_rng(2)
    Ws = _net(rng)
    X = rng.standard_normal((7, 12))
    Y, _ = mlp.forward(Ws, X)
    for c in (0.5, 3.7):
        Yc, _ = mlp.forward(Ws, c * X)
        assert np.allclose(Yc, c * Y, rtol=1e-14, atol=0)
    s = np.abs(rng.standard_normal(7)) + 0.1
    out_scale = np.array([2.0, 0.5, 1.5, 3.0])
    C = mlp.correction(Ws, X, s, out_scale, nv=4, Np=2, ndef=12)
    Cm = mlp.correction(Ws, -X, s, out_scale, nv=4, Np=2, ndef=12)
    assert np.array_equal(Cm, -C)


@pytest.mark.parametrize("dim,n,P1", [(2, (4, 6), 3), (3, (2, 4, 2), 3)])
def test_features_of_elementwise_constant_field(dim, n, P1):
    """A field constant inside each element: own part = the constant, every
    neighbour part = that neighbour's constant, so the layout and the
    neighbour on each side are pinned."""
    nv = dim + 2
    Np = P1 ** dim
    NF = P1 ** (dim - 1)
    Ne = int(np.prod(n))
    rng = np.random.default_rng(3)
    const = rng.uniform(1, 2, (nv, Ne))
    d1 = np.repeat(const[:, None, :], Np, axis=1)
    in_scale = np.array([1.0, 2.0, 4.0, 8.0, 16.0])
    nin = nv * Np * (1 + 2 * dim)
    h = [np.linspace(1.0, 2.0, n[a]) for a in range(dim)]
    rows, s = mlp.features(d1, dim, n, P1, in_scale, nin + dim + 3, h)
    nn = list(n) + [1] * (3 - len(n))
    for k in [0, 5, Ne - 1]:
        raw = rows[k] * s[k]
        assert np.allclose(raw[:nv * Np], np.repeat(const[:, k] / in_scale[:nv], Np))
        kc = [k % nn[0], (k // nn[0]) % nn[1], k // (nn[0] * nn[1])]
        off = nv * Np
        for a in range(dim):
            for side in (-1, 1):
                c = list(kc)
                c[a] = (c[a] + side) % nn[a]
                kn = c[0] + nn[0] * (c[1] + nn[1] * c[2])
                assert np.allclose(raw[off:off + nv * Np], np.repeat(const[:, kn] / in_scale[:nv], Np))
                off += nv * Np
        for a in range(dim):
            assert abs(rows[k, nin + a] - np.log(h[a][kc[a]] / 2.0)) < 1e-14
        assert np.all(rows[k, nin + dim:] == 0.0)
        assert abs(np.linalg.norm(rows[k, :nin]) - 1.0) < 1e-14


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-5, 5, 1000),
                        [1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, -1.5, 0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def _odd_select_net(ndef, ngeo, nin_pad, sel, alpha, nh=None):
    """Bias-free ReLU network with N(x, g) = x[sel] + alpha (sum g) 1:
    hidden units relu(x_j), relu(-x_j) for the selected entries and
    relu(g_a), relu(-g_a); relu(t) - relu(-t) = t rebuilds them exactly."""
    nout = len(sel)
    nh = nh or 2 * nout + 2 * ngeo
    W1 = np.zeros((nh, nin_pad))
    for o, j in enumerate(sel):
        W1[2 * o, j] = 1.0
        W1[2 * o + 1, j] = -1.0
    for a in range(ngeo):
        W1[2 * nout + 2 * a, ndef + a] = 1.0
        W1[2 * nout + 2 * a + 1, ndef + a] = -1.0
    W2 = np.eye(nh)
    W3 = np.zeros((nout, nh))
    for o in range(nout):
        W3[o, 2 * o] = 1.0
        W3[o, 2 * o + 1] = -1.0
        for a in range(ngeo):
            W3[o, 2 * nout + 2 * a] = alpha
            W3[o, 2 * nout + 2 * a + 1] = -alpha
    return [W1, W2, W3]


@pytest.mark.parametrize("uniform", [True, False])
def test_mirrored_evaluation_keeps_geometry(uniform):
    """(N(x, g) - N(-x, g))/2 with N(x, g) = x + alpha (sum g) 1 is x
    exactly: the geometry entries cancel only if the mirrored row keeps
    them.  On a uniform mesh every g is 0 (ln 1), so a rule that located
    the geometry columns from the non-zero entries would mirror the wrong
    ones; on a stretched mesh negating g would add 2 alpha sum g."""
    rng = np.random.default_rng(5)
    nv, Np, dim = 4, 3, 2
    ndef = nv * Np
    nin_pad = ndef + dim + 4
    rows = np.zeros((9, nin_pad))
    rows[:, :ndef] = rng.standard_normal((9, ndef))
    rows[:, ndef:ndef + dim] = 0.0 if uniform else np.log(rng.uniform(0.1, 1.0, (9, dim)))
    s = rng.uniform(0.5, 2.0, 9)
    tau = np.array([1.0, 2.0, 0.5, 4.0])
    Ws = _odd_select_net(ndef, dim, nin_pad, list(range(ndef)), alpha=0.7)
    C = mlp.correction(Ws, rows, s, tau, nv, Np, ndef, ngeo=dim)
    expect = rows[:, :ndef].reshape(9, nv, Np).transpose(1, 2, 0) * s[None, None, :] * tau[:, None, None]
    assert np.allclose(C, expect, rtol=1e-14, atol=1e-15)
    # the network itself does see the geometry (the pin is not vacuous)
    if not uniform:
        Yp, _ = mlp.forward(Ws, rows)
        assert np.abs(Yp - rows[:, :ndef]).max() > 1e-3


@pytest.mark.parametrize("dim,n,P1,part", [(2, (4, 6), 3, 0), (2, (4, 6), 3, 2), (2, (4, 6), 3, 3),
                                           (3, (2, 4, 2), 2, 5), (3, (2, 4, 2), 2, 6)])
def test_learned_coarse_step_closed_form(dim, n, P1, part):
    """A network that returns one part of the feature row (part 0 = the
    element itself, part 1 + 2a + side = its -a / +a face neighbour) gives
    C = C1 + (tau / in_scale) C1(that element), per variable: the feature
    layout, the neighbour orientation, the scales, the row norm and the
    output layout all enter this closed form."""
    rng = np.random.default_rng(6)
    nv = dim + 2
    Np = P1 ** dim
    Ne = int(np.prod(n))
    nb = nv * Np
    ndef = nb * (1 + 2 * dim)
    nin_pad = ndef + dim + 5
    h = [rng.uniform(0.5, 1.5, n[a]) for a in range(dim)]
    C1 = rng.standard_normal((nv, Np, Ne))
    in_scale = rng.uniform(0.5, 2.0, nv)
    out_scale = rng.uniform(0.5, 2.0, nv)
    Ws = _odd_select_net(ndef, dim, nin_pad, list(range(part * nb, (part + 1) * nb)), alpha=0.3)
    lc = mlp.LearnedCoarse(Ws, in_scale, out_scale, dim, n, h, P1, nin_pad)
    C = lc.correct(C1)
    nn = list(n) + [1] * (3 - len(n))
    for k in range(Ne):
        kc = [k % nn[0], (k // nn[0]) % nn[1], k // (nn[0] * nn[1])]
        if part > 0:
            a, side = (part - 1) // 2, (-1, 1)[(part - 1) % 2]
            kc[a] = (kc[a] + side) % nn[a]
        kn = kc[0] + nn[0] * (kc[1] + nn[1] * kc[2])
        expect = C1[:, :, k] + (out_scale / in_scale)[:, None] * C1[:, :, kn]
        assert np.allclose(C[:, :, k], expect, rtol=1e-13, atol=1e-14)


def test_bf16_products_exact_on_representable_values():
    """With inputs, weights, targets and every intermediate exactly
    representable in bfloat16 (small integers over a power-of-two batch),
    the BF16-rounded forward pass and gradient equal the FP64 ones: the
    rounding points drop or reorder no term."""
    rng = np.random.default_rng(7)
    Ws = [rng.integers(-1, 2, (8, 6)).astype(float), rng.integers(-1, 2, (8, 8)).astype(float),
          rng.integers(-1, 2, (8, 8)).astype(float)]
    X = rng.integers(-1, 2, (4, 6)).astype(float)
    T = rng.integers(-3, 4, (4, 8)).astype(float)
    Y, (H1, H2) = mlp.forward(Ws, X)
    # every intermediate is a multiple of 1/4 below 64 in magnitude (8 significant bits)
    E = Y - T
    for v in (Y, H1, H2, E / 4, (E / 4) @ Ws[2], ((E / 4) @ Ws[2]) @ Ws[1]):
        assert np.abs(v).max() < 64
    assert np.abs(H2).max() > 0
    Yb, _ = mlp.forward(Ws, X, bf16=True)
    assert np.array_equal(Y, Yb)
    l, g = mlp.loss_grad(Ws, X, T, 6)
    lb, gb = mlp.loss_grad(Ws, X, T, 6, bf16=True)
    assert l == lb
    for a, b in zip(g, gb):
        assert np.array_equal(a, b)
    # and they differ once the operands are not representable
    Xr = rng.standard_normal((4, 6))
    assert not np.array_equal(mlp.forward(Ws, Xr)[0], mlp.forward(Ws, Xr, bf16=True)[0])


def test_adam_matches_torch():
    """Several Adam steps with changing gradients equal torch.optim.Adam
    (FP64 tensors, same hyper-parameters)."""
    rng = np.random.default_rng(8)
    W0 = rng.standard_normal((5, 7))
    grads = [rng.standard_normal((5, 7)) * 10.0 ** rng.integers(-3, 2) for _ in range(6)]
    w = torch.tensor(W0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    W, M, V = W0.copy(), np.zeros_like(W0), np.zeros_like(W0)
    for t, G in enumerate(grads, start=1):
        opt.zero_grad()
        w.grad = torch.tensor(G, dtype=torch.float64)
        opt.step()
        W, M, V = mlp.adam_step(W, G, M, V, t, 3e-3)
    assert np.allclose(W, w.detach().numpy(), rtol=1e-14, atol=1e-16)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2, so every step moves each weight by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(9)
    W0 = rng.standard_normal(11)
    G = rng.standard_normal(11) * np.logspace(-6, 2, 11)
    W, M, V = W0.copy(), np.zeros(11), np.zeros(11)
    for t in range(1, 8):
        W, M, V = mlp.adam_step(W, G, M, V, t, 1e-2)
        expect = W0 - t * 1e-2 * G / (np.abs(G) + 1e-8)
        assert np.allclose(W, expect, rtol=1e-12, atol=1e-15)


def _tiny_pmg(orc, learned=None, n1=2):
    from paper_2202_09733_amd import workloads as Wk
    wl = Wk.make_vortical_workload(n=(4, 4), p0=2, p1=1, dt_factor=100.0, seed=3)
    L0 = orc.Level(**wl.level_kwargs(wl.p0))
    L1 = orc.Level(**wl.level_kwargs(wl.p1))
    sigA = 1.0 / wl.dt + 1.0 / (wl.a_ii * wl.dt)
    sigS = 1.0 / wl.dt + sigA
    fac0 = orc.lu_factor(L0.ej_blocks(wl.dq, sigS))
    q1 = orc.restrict(wl.dq, 2, wl.p0 + 1, wl.p1 + 1)
    fac1 = orc.lu_factor(L1.ej_blocks(q1, sigS))
    pm = orc.PMG(L0, L1, fac0, fac1, orc.PMGParams(sigma_D=sigA, n1=n1, learned=learned))
    pm.set_point(wl.dq, L0.residual(wl.dq))
    return wl, L0, L1, fac1, pm


def test_learned_vcycle_with_zero_network_is_one_coarse_sweep(orc):
    """With W3 = 0 the learned correction is C1 = B1^{-1} Gamma d, which is
    what the first coarse EJ sweep of the plain V-cycle adds to Z0: the
    learned V-cycle equals the pinned plain V-cycle with n1 = 1."""
    wl, L0, L1, fac1, pm_plain = _tiny_pmg(orc, n1=1)
    nv, Np1 = L1.nv, L1.Np
    nin_pad = nv * Np1 * 5 + 2 + 6
    rng = np.random.default_rng(10)
    Ws = [rng.standard_normal((32, nin_pad)), rng.standard_normal((32, 32)), np.zeros((16, 32))]
    lc = mlp.LearnedCoarse(Ws, np.ones(nv), np.ones(nv), 2, wl.n, wl.h, wl.p1 + 1, nin_pad)
    _, _, _, _, pm_l = _tiny_pmg(orc, learned=lc)
    X = rng.standard_normal(L0.shape)
    Yp = pm_plain.apply(X)
    Yl = pm_l.apply(X)
    assert np.linalg.norm(Yl - Yp) <= 1e-13 * np.linalg.norm(Yp)
    # a non-zero network changes the cycle
    Ws[2] = rng.standard_normal((16, 32))
    assert np.linalg.norm(pm_l.apply(X) - Yp) > 1e-3 * np.linalg.norm(Yp)
