"""Pins of the fold-in oracle: finite differences, GELU closed forms, a hand
worked embedding bag and the AdamW update."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import foldin
from paper_2509_18024_amd import synth


def test_gelu_closed_forms():
    assert foldin.gelu(np.array(0.0)) == 0.0
    x = np.array([-3.0, -1.0, 0.5, 2.0])
    np.testing.assert_allclose(foldin.gelu(x), x * norm.cdf(x), rtol=1e-14)
    h = 1e-6
    np.testing.assert_allclose(foldin.gelu_grad(x), (foldin.gelu(x + h) - foldin.gelu(x - h)) / (2 * h),
                               rtol=1e-7)


def test_bag_hand_example():
    M = np.array([[1.0, 2.0], [3.0, -1.0], [0.0, 4.0]])
    ptr = np.array([0, 2, 2, 3])
    items = np.array([0, 2, 1])
    vals = np.array([2.0, 1.0, 5.0])
    b = foldin.bag(M, ptr, items, vals, [0, 1, 2])
    np.testing.assert_allclose(b[0], [(2 * 1 + 1 * 0) / 2, (2 * 2 + 1 * 4) / 2])
    assert np.all(b[1] == 0)
    np.testing.assert_allclose(b[2], [15.0, -5.0])


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    n_f, H, B = 5, 7, 4
    rng = np.random.default_rng(seed)
    theta = synth.foldin_init_params(seed, n_f, H).astype(np.float64) + 0.1 * rng.standard_normal(
        foldin.param_count(n_f, H))
    x = rng.standard_normal((B, n_f))
    tgt = rng.standard_normal((B, n_f))
    L, g = foldin.loss_and_grad(theta, x, tgt, n_f, H)
    eps = 1e-6
    for k in rng.choice(len(theta), size=40, replace=False):
        e = np.zeros_like(theta)
        e[k] = eps
        lp, _ = foldin.loss_and_grad(theta + e, x, tgt, n_f, H)
        lm, _ = foldin.loss_and_grad(theta - e, x, tgt, n_f, H)
        assert abs((lp - lm) / (2 * eps) - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_adamw_first_step_is_signed_lr():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = foldin.adamw(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01, wd=0.0)
    # bias-corrected first step: m_hat / sqrt(v_hat) = sign(g) (up to eps)
    np.testing.assert_allclose(t1, theta - 0.01 * np.sign(g), rtol=1e-5)
    t2, _, _ = foldin.adamw(theta, np.zeros(3), np.zeros(3), np.zeros(3), 1, lr=0.01, wd=0.1)
    np.testing.assert_allclose(t2, theta * (1 - 0.001))


def test_param_count_matches_layer_sizes():
    assert foldin.param_count(64, 256) == 64 * 256 + 256 + 256 * 256 + 256 + 256 * 64 + 64 == 98880


def test_relative_residual_pins():
    import oracle
    rng = np.random.default_rng(5)
    n, nf, lam = 40, 6, 0.05
    X = rng.standard_normal((n, nf))
    y = rng.standard_normal(n)
    # full data: the system is the ridge normal equation, solved independently by lstsq
    Xa = np.vstack([X, math.sqrt(lam * n) * np.eye(nf)])
    ya = np.concatenate([y, np.zeros(nf)])
    u_ridge = np.linalg.lstsq(Xa, ya, rcond=None)[0]
    assert foldin.relative_residual(X, y, lam, n, u_ridge) < 1e-12
    assert foldin.relative_residual(X, y, lam, n, np.zeros(nf)) == 1.0
    # core system: the oracle's own core solve satisfies it; a perturbed answer does not
    s = 4
    u, st = oracle.core_row(X, y, lam, s)
    assert st == 0
    assert foldin.relative_residual(X, y, lam, s, u) < 1e-12
    assert foldin.relative_residual(X, y, lam, s, u * 1.01) > 1e-3
    # a sketch that keeps one entry per column: A has the hand-computable form
    A, b = foldin.core_system(X, y, lam, 1)
    k = np.argmax(np.abs(X), axis=0)
    for a in range(nf):
        np.testing.assert_allclose(A[a], X[k[a], a] * X[k[a]] + lam * n * np.eye(nf)[a], rtol=1e-14)
        assert abs(b[a] - X[k[a], a] * y[k[a]]) < 1e-14
    assert foldin.relative_residual(np.zeros((0, nf)), np.zeros(0), lam, 0, np.ones(nf)) == math.inf


def test_forward_hand_worked_network():
    """A 2 -> 2 -> 2 -> 2 network whose pre-activations are 0 or +-10, where
    GELU is 0, 10 and about -7.6e-23: the output follows by hand.  A dropped
    bias or a transposed weight matrix changes it.  Second network: the only
    activation is GELU(1) = Phi(1), so out = 2 Phi(1) - 1 = P(|Z| < 1), the
    tabulated 0.682689492137086."""
    W1 = np.array([[3.0, 1.0], [-2.0, -4.0]])
    c1 = np.array([5.0, 0.0])
    W2 = np.array([[0.1, 5.0], [0.2, 0.0]])
    c2 = np.array([-1.0, 8.0])
    W3 = np.array([[1.0, 0.5], [2.0, -0.25]])
    c3 = np.array([0.5, 1.0])
    theta = foldin.pack({"W1": W1, "c1": c1, "W2": W2, "c2": c2, "W3": W3, "c3": c3}, 2, 2)
    out, _ = foldin.forward(theta, np.array([[1.0, 2.0]]), 2, 2)
    # z1 = [10, -10] -> h1 = [10, ~0]; z2 = [~0, 10] -> h2 = [~0, 10]; out = W3 h2 + c3
    np.testing.assert_allclose(out[0], [5.5, -1.5], rtol=0, atol=1e-12)
    theta1 = foldin.pack({"W1": [[1.0]], "c1": [0.0], "W2": [[0.0]], "c2": [1.0], "W3": [[2.0]], "c3": [-1.0]},
                         1, 1)
    out1, _ = foldin.forward(theta1, np.array([[0.3]]), 1, 1)
    assert abs(out1[0, 0] - 0.682689492137086) <= 1e-15
