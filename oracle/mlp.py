"""FP64 oracle of the learned coarse correction (test infrastructure only).

Not in the paper: a bias-free ReLU network N(x) = W3 relu(W2 relu(W1 x))
applied per element to a feature row built from the element-local coarse
step on the element and on its face neighbours, replacing the
coarse smoothing sweeps of the p-multigrid V-cycle (Sec. 3.1's coarse
correction C).  Everything here is the plain definition in FP64.
"""
from __future__ import annotations

import numpy as np



def relu(x):
    return np.maximum(x, 0.0)


def forward(Ws, X):
    """Rows of X (each a normalised feature row) -> rows of N(x)."""
    W1, W2, W3 = Ws
    H1 = relu(X @ W1.T)
    H2 = relu(H1 @ W2.T)
    return H2 @ W3.T, (H1, H2)


def loss_grad(Ws, X, T, nout):
    """Batch loss 0.5 sum_j<nout (N(x) - t)^2 / B and its gradient with
    respect to W1, W2, W3 by the chain rule."""
    W1, W2, W3 = Ws
    B = X.shape[0]
    Y, (H1, H2) = forward(Ws, X)
    E = Y - T
    E[:, nout:] = 0.0
    loss = 0.5 * float(np.sum(E * E)) / B
    dY = E / B
    dW3 = dY.T @ H2
    dH2 = (dY @ W3) * (H2 > 0)
    dW2 = dH2.T @ H1
    dH1 = (dH2 @ W2) * (H1 > 0)
    dW1 = dH1.T @ X
    return loss, [dW1, dW2, dW3]


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
    scale = np.repeat(in_scale[:nv], Np)
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


def correction(Ws, rows, s, out_scale, nv, Np, ngeo=0):
    """C[v][i][k] = tau_v s_k (N(x_k, g_k) - N(-x_k, g_k)) / 2, g the last
    ngeo (geometry) entries of the used part of a row."""
    Yp, _ = forward(Ws, rows)
    neg = -rows
    if ngeo:
        used = np.max(np.nonzero(np.any(rows != 0, axis=0))[0]) + 1
        neg[:, used - ngeo:used] = rows[:, used - ngeo:used]
    Ym, _ = forward(Ws, neg)
    Y = 0.5 * (Yp - Ym)[:, :nv * Np]
    C = Y.reshape(-1, nv, Np).transpose(1, 2, 0) * s[None, None, :] * out_scale[:nv, None, None]
    return np.ascontiguousarray(C)


def bf16_round(x):
    """Round float values to bfloat16 (round to nearest, ties to even) and
    back, as the GPU products see their operands."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (a >> 16) & 1
    a = (a + 0x7FFF + lsb) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)
