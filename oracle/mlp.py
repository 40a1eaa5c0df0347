"""FP64 oracle of the learned coarse correction (test infrastructure only).

Not in the paper: a bias-free ReLU network N(x) = W3 relu(W2 relu(W1 x))
applied per element to a feature row built from the element-local coarse
step on the element and on its face neighbours, replacing the
coarse smoothing sweeps of the p-multigrid V-cycle (Sec. 3.1's coarse
correction C).  Everything here is the plain definition in FP64.

``bf16=True`` rounds the operands of every product to bfloat16 where the GPU
stores them in that format (inputs, weights, hidden activations, output
gradients), and keeps FP64 everywhere else, so that a comparison with the
GPU's BF16-input, FP32-accumulate products measures only accumulation order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def relu(x):
    return np.maximum(x, 0.0)


def bf16_round(x):
    """Round float values to bfloat16 (round to nearest, ties to even) and
    back, as the GPU products see their operands."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (a >> 16) & 1
    a = (a + 0x7FFF + lsb) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def _maybe_bf(x, bf16):
    return bf16_round(x) if bf16 else x


def forward(Ws, X, bf16=False):
    """Rows of X (each a normalised feature row) -> rows of N(x)."""
    W1, W2, W3 = [_maybe_bf(w, bf16) for w in Ws]
    H1 = _maybe_bf(relu(_maybe_bf(X, bf16) @ W1.T), bf16)
    H2 = _maybe_bf(relu(H1 @ W2.T), bf16)
    return H2 @ W3.T, (H1, H2)


def loss_grad(Ws, X, T, nout, bf16=False):
    """Batch loss 0.5 sum_j<nout (N(x) - t)^2 / B and its gradient with
    respect to W1, W2, W3 by the chain rule."""
    W1, W2, W3 = [_maybe_bf(w, bf16) for w in Ws]
    Xb = _maybe_bf(X, bf16)
    B = X.shape[0]
    Y, (H1, H2) = forward(Ws, Xb, bf16)
    E = Y - T
    E[:, nout:] = 0.0
    loss = 0.5 * float(np.sum(E * E)) / B
    dY = _maybe_bf(E / B, bf16)
    dW3 = dY.T @ H2
    dH2 = _maybe_bf((dY @ W3) * (H2 > 0), bf16)
    dW2 = dH2.T @ H1
    dH1 = _maybe_bf((dH2 @ W2) * (H1 > 0), bf16)
    dW1 = dH1.T @ Xb
    return loss, [dW1, dW2, dW3]


def adam_step(W, G, M, V, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of the weights W with gradient
    G, first and second moments M, V and step number t >= 1:
    M <- b1 M + (1 - b1) G, V <- b2 V + (1 - b2) G^2,
    W <- W - lr (M / (1 - b1^t)) / (sqrt(V / (1 - b2^t)) + eps).
    Returns the new (W, M, V)."""
    M = b1 * M + (1.0 - b1) * G
    V = b2 * V + (1.0 - b2) * G * G
    mhat = M / (1.0 - b1 ** t)
    vhat = V / (1.0 - b2 ** t)
    return W - lr * mhat / (np.sqrt(vhat) + eps), M, V


def features(d1, dim, n, P1, in_scale, nin_pad, h):
    """Feature rows of a level-1 field d1 [nv][Np1][Ne]: the element's own
    values, then per axis the values of the -axis neighbour and of the +axis
    neighbour, each divided by the variable's scale; this defect part divided
    by its 2-norm s; then, per axis, ln(h_a / max h_a) of the element (h:
    element widths per axis).  Returns (rows, s)."""
    nv, Np, Ne = d1.shape
    nn = list(n) + [1] * (3 - len(n))
    rows = np.zeros((Ne, nin_pad))
    s = np.zeros(Ne)
    scale = np.repeat(np.asarray(in_scale, dtype=np.float64)[:nv], Np)
    for k in range(Ne):
        kc = [k % nn[0], (k // nn[0]) % nn[1], k // (nn[0] * nn[1])]
        parts = [d1[:, :, k].reshape(-1) / scale]
        for a in range(dim):
            for side in (-1, 1):
                c = list(kc)
                c[a] = (c[a] + side) % nn[a]
                kn = c[0] + nn[0] * (c[1] + nn[1] * c[2])
                parts.append(d1[:, :, kn].reshape(-1) / scale)
        row = np.concatenate(parts)
        nr = float(np.linalg.norm(row))
        s[k] = nr
        rows[k, :row.size] = row / nr if nr > 0 else 0.0
        for a in range(dim):
            ha = np.asarray(h[a], dtype=np.float64)
            rows[k, row.size + a] = np.log(ha[kc[a]] / ha.max())
    return rows, s


def correction(Ws, rows, s, out_scale, nv, Np, ndef, ngeo=0, bf16=False):
    """C[v][i][k] = tau_v s_k (N(x_k, g_k) - N(-x_k, g_k)) / 2, where x_k are
    the first ndef entries of row k (the normalised defect part) and g_k the
    next ngeo entries (geometry), which the mirrored evaluation keeps."""
    Yp, _ = forward(Ws, rows, bf16)
    neg = rows.copy()
    neg[:, :ndef] = -rows[:, :ndef]
    Ym, _ = forward(Ws, neg, bf16)
    Y = 0.5 * (Yp - Ym)[:, :nv * Np]
    tau = np.asarray(out_scale, dtype=np.float64)[:nv]
    C = Y.reshape(-1, nv, Np).transpose(1, 2, 0) * s[None, None, :] * tau[:, None, None]
    return np.ascontiguousarray(C)


@dataclass
class LearnedCoarse:
    """The learned coarse step of the V-cycle: given the element-local coarse
    EJ step C1 = B1^{-1} Gamma d on the coarse level (layout [nv][Np1][Ne]),
    the coarse correction is C = C1 + tau s (N(x, g) - N(-x, g)) / 2 with the
    feature rows x of C1 (own element and its 2 dim face neighbours, scaled
    per variable by in_scale and by the row norm s) and the geometry entries
    g = ln(h_a / max h_a).  Ws = (W1 [nh x nin_pad], W2, W3 [nout_pad x nh])."""
    Ws: list
    in_scale: np.ndarray
    out_scale: np.ndarray
    dim: int
    n: tuple
    h: list
    P1: int
    nin_pad: int
    bf16: bool = False

    def correct(self, C1: np.ndarray) -> np.ndarray:
        nv, Np, _ = C1.shape
        rows, s = features(C1, self.dim, self.n, self.P1, self.in_scale, self.nin_pad, self.h)
        ndef = nv * Np * (1 + 2 * self.dim)
        return C1 + correction(self.Ws, rows, s, self.out_scale, nv, Np, ndef, self.dim, self.bf16)
