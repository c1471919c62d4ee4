"""Pins for the oracle's MLP, Adam and POD (the learned extrapolator that
sits beside the DMD extrapolation of Sec. 6)."""

import numpy as np
import pytest

from oracle import mlp, pod


def test_bf16_rounding_known_values():
    one = 1.0
    ulp = 2.0 ** -7                       # bfloat16 spacing at 1
    assert mlp.bf16_round(one) == one
    assert mlp.bf16_round(one + ulp / 2) == one               # tie -> even mantissa (0)
    assert mlp.bf16_round(one + 1.5 * ulp) == one + 2 * ulp   # tie -> even mantissa (2)
    assert mlp.bf16_round(one + 0.6 * ulp) == one + ulp
    assert mlp.bf16_round(-3.0) == -3.0
    assert mlp.bf16_round(0.0) == 0.0
    assert np.isinf(mlp.bf16_round(3.4e38))                   # beyond the largest bfloat16
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 10000)
    r = mlp.bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-7))
    assert np.all(mlp.bf16_round(r) == r)                     # idempotent
    bits = (r.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    assert np.all(mlp.bf16_bits_to_float(bits) == r)


def _net(seed, dims, B):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.param_count(dims)) * 0.5
    X = rng.standard_normal((B, dims[0]))
    T = rng.standard_normal((B, dims[-1]))
    return p, X, T


def test_gradient_matches_central_differences():
    dims = [6, 5, 4, 3]
    p, X, T = _net(3, dims, 4)
    loss, g = mlp.loss_and_grad(dims, p, X, T, quantize=False)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(dims, p + e, X, T, False)[0] - mlp.loss_and_grad(dims, p - e, X, T, False)[0]) / (2 * h)
    assert np.abs(g - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())
    assert loss == pytest.approx(np.mean((mlp.forward(dims, p, X, False)[0] - T) ** 2))


def test_quantisation_is_exact_on_representable_values():
    """Small integers are exact in bfloat16 and their products and sums stay
    exact, so the quantised and the plain network agree exactly."""
    dims = [4, 3, 2]
    rng = np.random.default_rng(5)
    p = rng.integers(-3, 4, mlp.param_count(dims)).astype(float)
    X = rng.integers(-3, 4, (5, 4)).astype(float)
    T = rng.integers(-3, 4, (5, 2)).astype(float)
    assert np.array_equal(mlp.forward(dims, p, X, True)[0], mlp.forward(dims, p, X, False)[0])
    # the loss gradient 2 (y - t) / (B n) is a dyadic fraction here (B n = 10 is not): compare with tolerance
    g1 = mlp.loss_and_grad(dims, p, X, T, True)[1]
    g0 = mlp.loss_and_grad(dims, p, X, T, False)[1]
    assert np.abs(g1 - g0).max() <= 2.0 ** -8 * np.abs(g0).max()


def test_adam_first_step_moves_by_lr_times_sign():
    """With m = v = 0, the bias-corrected first Adam step is lr g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    p1, m, v = mlp.adam(p, g, np.zeros(100), np.zeros(100), 1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_moves_by_lr_times_sign_every_step():
    """With a constant gradient g the moments are m_t = (1 - beta1^t) g and
    v_t = (1 - beta2^t) g^2, so the bias-corrected ratio is g / |g| at every
    step t: each step moves by lr g / (|g| + eps).  A bias correction with the
    wrong power (beta t instead of beta^t, or t - 1) fails from t = 2 on."""
    rng = np.random.default_rng(17)
    p0 = rng.standard_normal(64)
    g = rng.standard_normal(64)
    p, m, v = p0.copy(), np.zeros(64), np.zeros(64)
    lr, b1, b2 = 0.003, 0.9, 0.999
    for t in range(1, 6):
        p, m, v = mlp.adam(p, g, m, v, t, lr=lr, beta1=b1, beta2=b2)
        np.testing.assert_allclose(m, (1 - b1 ** t) * g, rtol=1e-14)
        np.testing.assert_allclose(v, (1 - b2 ** t) * g * g, rtol=1e-13)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)


def test_pod_recovers_planted_modes():
    """Snapshots mean + sum_i a_si s_i v_i with orthonormal v_i and
    orthonormal zero-mean amplitude columns a_i: the POD returns s_i and +-v_i."""
    rng = np.random.default_rng(11)
    S, n, k = 30, 400, 5
    V, _ = np.linalg.qr(rng.standard_normal((n, k)))
    A = rng.standard_normal((S, k))
    A -= A.mean(axis=0)
    A, _ = np.linalg.qr(A)
    s = np.array([10.0, 5.0, 2.0, 1.0, 0.5])
    mu = rng.standard_normal(n)
    X = mu + (A * s) @ V.T
    mean, basis, sigma = pod.pod(X, k)
    np.testing.assert_allclose(mean, mu, atol=1e-12)
    np.testing.assert_allclose(sigma, s, rtol=1e-12)
    for i in range(k):
        assert abs(abs(basis[i] @ V[:, i]) - 1) < 1e-12
    c = pod.project(X, mean, basis)
    np.testing.assert_allclose(pod.reconstruct(c, mean, basis), X, atol=1e-12)
