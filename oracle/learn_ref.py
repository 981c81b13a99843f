"""Float64 CPU reference of the learned symbol-grouping model.

TEST INFRASTRUCTURE ONLY (like the rest of this package): it is the plain
definition the GPU training kernels are checked against, written with numpy
matrix products as its only library steps.

Model (per symbol c, a row of X):
    pre = X W1 + b1,  h = relu(pre),  z = h W2 + b2,  P = softmax(z)
over B fields and one "no field" column; L = log(1 - P[:, :B]).
A string with symbol set S leaves field j clear with probability
Z_S,j = exp(sum_{c in S} L_cj) when every symbol picks its field
independently from P_c; a pair (A, B) then has expected fingerprint distance
    E = sum_j Z_A,j + Z_B,j - 2 Z_{A u B},j
(a field differs iff exactly one side sets it).  For one-hot P, E is the
occurrence F_D of Section 3.3 under the map c -> argmax P_c (a grouping of
symbols into fields, which keeps Theorem 1 and Eq. 1).  Loss per non-matching
pair: softplus(beta (t - E)) / beta, t = 2k + 1 + margin; plus
entropy_weight * mean_c H(P_c).
"""
from __future__ import annotations

import numpy as np

CLAMP = 1e-7  # 1 - P is clamped below at this value, as in the GPU kernels


def unpack(params, d_in, hidden, bits):
    p = np.asarray(params, dtype=np.float64)
    n1 = d_in * hidden
    n2 = hidden * (bits + 1)
    W1 = p[:n1].reshape(d_in, hidden)
    b1 = p[n1:n1 + hidden]
    W2 = p[n1 + hidden:n1 + hidden + n2].reshape(hidden, bits + 1)
    b2 = p[n1 + hidden + n2:n1 + hidden + n2 + bits + 1]
    return W1, b1, W2, b2


def n_params(d_in, hidden, bits):
    return d_in * hidden + hidden + hidden * (bits + 1) + bits + 1


def masks_to_dense(masks, sigma):
    """(n, 2) uint64 masks -> (n, sigma) float64 membership matrix."""
    m = np.asarray(masks, dtype=np.uint64).reshape(-1, 2)
    out = np.zeros((m.shape[0], sigma))
    for c in range(sigma):
        word, bit = divmod(c, 64)
        out[:, c] = (m[:, word] >> np.uint64(bit)) & np.uint64(1)
    return out


def forward(X, params, hidden, bits):
    X = np.asarray(X, dtype=np.float64)
    W1, b1, W2, b2 = unpack(params, X.shape[1], hidden, bits)
    pre = X @ W1 + b1
    h = np.maximum(pre, 0.0)
    z = h @ W2 + b2
    z = z - z.max(axis=1, keepdims=True)
    P = np.exp(z)
    P /= P.sum(axis=1, keepdims=True)
    L = np.log(np.maximum(1.0 - P[:, :bits], CLAMP))
    return pre, h, P, L


def expected_fd(L, A, B):
    """E per pair from membership matrices A, B (n x sigma)."""
    U = np.maximum(A, B)
    ZA, ZB, ZU = np.exp(A @ L), np.exp(B @ L), np.exp(U @ L)
    return (ZA + ZB - 2.0 * ZU).sum(axis=1), (ZA, ZB, ZU, U)


def loss(X, params, hidden, bits, A, B, k, margin, beta, entropy_weight):
    """(mean pair loss, mean symbol entropy, mean E, total loss)."""
    _, _, P, L = forward(X, params, hidden, bits)
    E, _ = expected_fd(L, A, B)
    t = 2 * k + 1 + margin
    x = beta * (t - E)
    pair = np.logaddexp(0.0, x) / beta
    ent = -(P * np.log(np.maximum(P, 1e-300))).sum(axis=1)
    pl = pair.mean() if pair.size else 0.0
    return pl, ent.mean(), (E.mean() if E.size else 0.0), pl + entropy_weight * ent.mean()


def grads(X, params, hidden, bits, A, B, k, margin, beta, entropy_weight):
    """Analytic gradient of the total loss, packed like params."""
    X = np.asarray(X, dtype=np.float64)
    sigma, d_in = X.shape
    W1, b1, W2, b2 = unpack(params, d_in, hidden, bits)
    pre, h, P, L = forward(X, params, hidden, bits)
    n = A.shape[0]
    E, (ZA, ZB, ZU, U) = expected_fd(L, A, B)
    t = 2 * k + 1 + margin
    s = -1.0 / (1.0 + np.exp(-beta * (t - E)))  # d pair loss / d E
    s = s / max(n, 1)
    G = A.T @ (s[:, None] * ZA) + B.T @ (s[:, None] * ZB) + U.T @ (-2.0 * s[:, None] * ZU)
    dP = np.zeros_like(P)
    dP[:, :bits] = G * (-1.0 / np.maximum(1.0 - P[:, :bits], CLAMP))
    dP += (entropy_weight / sigma) * (-(np.log(np.maximum(P, 1e-300)) + 1.0))
    dz = P * (dP - (P * dP).sum(axis=1, keepdims=True))
    dW2 = h.T @ dz
    db2 = dz.sum(axis=0)
    dh = (dz @ W2.T) * (pre > 0)
    dW1 = X.T @ dh
    db1 = dh.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2])
