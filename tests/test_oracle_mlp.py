"""Pins of the FP64 oracle of the learned coarse correction: gradients against
central differences, exact positive homogeneity and oddness, the feature
layout against per-element constant fields, and bf16 rounding against torch."""
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
    C = mlp.correction(Ws, X, s, out_scale, nv=4, Np=2)
    Cm = mlp.correction(Ws, -X, s, out_scale, nv=4, Np=2)
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
