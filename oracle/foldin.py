"""FP64 NumPy oracle of the learned fold-in (test infrastructure).

The fold-in answers a new user from the item factors M (frozen) and the
user's ratings, and is checked against the exact regression of eq. (U) /
eq. core_ui for that user (Section 2.1, Section 3).  The network:

    bag  b = (1/d) sum_k r_k m_{j_k}            (ratings-weighted mean of item factors)
    h1 = GELU(W1 b + c1),  h2 = GELU(W2 h1 + c2),  u_hat = W3 h2 + c3

with GELU(x) = x Phi(x) (exact, through erf).  Loss: mean squared error over
the batch and the n_f outputs against target factors produced by ALS.

Parameters are one flat vector in the order W1 [H x F], c1 [H], W2 [H x H],
c2 [H], W3 [F x H], c3 [F] (row-major), the layout the HIP library uses.
Only the tests, the smoke check and the benchmark's CPU leg import this.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def shapes(n_f: int, hidden: int):
    return [("W1", (hidden, n_f)), ("c1", (hidden,)), ("W2", (hidden, hidden)), ("c2", (hidden,)),
            ("W3", (n_f, hidden)), ("c3", (n_f,))]


def param_count(n_f: int, hidden: int) -> int:
    return sum(int(np.prod(s)) for _, s in shapes(n_f, hidden))


def unpack(theta: np.ndarray, n_f: int, hidden: int) -> dict:
    out, off = {}, 0
    for name, shp in shapes(n_f, hidden):
        size = int(np.prod(shp))
        out[name] = np.asarray(theta[off:off + size], np.float64).reshape(shp)
        off += size
    return out


def pack(p: dict, n_f: int, hidden: int) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in shapes(n_f, hidden)])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * phi


def bag(M, ptr, items, vals, rows):
    """b_i = (1/d_i) sum_k r_k M[j_k] for each listed row (zero for d_i = 0)."""
    M = np.asarray(M, np.float64)
    out = np.zeros((len(rows), M.shape[1]))
    for t, i in enumerate(rows):
        b, e = ptr[i], ptr[i + 1]
        if e > b:
            out[t] = (np.asarray(vals[b:e], np.float64)[:, None] * M[items[b:e]]).sum(0) / (e - b)
    return out


def forward(theta, x, n_f, hidden):
    p = unpack(theta, n_f, hidden)
    z1 = x @ p["W1"].T + p["c1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["c2"]
    h2 = gelu(z2)
    out = h2 @ p["W3"].T + p["c3"]
    return out, (x, z1, h1, z2, h2)


def loss_and_grad(theta, x, target, n_f, hidden):
    """L = mean((u_hat - target)^2) over batch and outputs; gradient in pack order."""
    p = unpack(theta, n_f, hidden)
    out, (x, z1, h1, z2, h2) = forward(theta, x, n_f, hidden)
    B = x.shape[0]
    diff = out - target
    L = float(np.mean(diff ** 2))
    d_out = 2.0 * diff / (B * n_f)
    g = {"W3": d_out.T @ h2, "c3": d_out.sum(0)}
    d_h2 = d_out @ p["W3"]
    d_z2 = d_h2 * gelu_grad(z2)
    g["W2"] = d_z2.T @ h1
    g["c2"] = d_z2.sum(0)
    d_h1 = d_z2 @ p["W2"]
    d_z1 = d_h1 * gelu_grad(z1)
    g["W1"] = d_z1.T @ x
    g["c1"] = d_z1.sum(0)
    return L, pack(g, n_f, hidden)


def adamw(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One AdamW step (decoupled weight decay); returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


def core_system(X, y, lam, s):
    """A = X*^T X + lam n E and b = X*^T y of one row (eq. core_ui; eq. (U) when
    s = n), with X* the CES sketch of Algorithm 1 (the C oracle's selection)."""
    from . import select
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    n, nf = X.shape
    W = np.zeros_like(X)
    if s >= n:
        W[:] = X
    elif s > 0:
        pos = select(X, s)
        for a in range(nf):
            W[pos[a], a] = X[pos[a], a]
    return W.T @ X + lam * n * np.eye(nf), W.T @ y


def relative_residual(X, y, lam, s, u):
    """|b - A u| / |b| of the row's system; inf when b = 0 (Section 3 estimator)."""
    A, b = core_system(X, y, lam, s)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return math.inf
    return float(np.linalg.norm(b - A @ np.asarray(u, np.float64)) / nb)
