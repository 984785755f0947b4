"""Pins of the FP64 network oracle (no GPU): gradients against central finite differences,
Adam against its closed-form first step, BF16 rounding against exact bit patterns."""
import numpy as np
import pytest

from oracle import mlp


def _small_params(rng, hidden):
    shp = mlp.param_shapes(hidden)
    return {k: rng.standard_normal(v) * (0.3 if k != "c" else 0.5) for k, v in shp.items()}


def _data(rng, M):
    hist = rng.standard_normal((5, M)) + 1j * rng.standard_normal((5, M))
    fh, fm = rng.standard_normal(M) * 0.2, rng.standard_normal(M) * 0.2
    s = (rng.random(M) < 0.5).astype(float)
    x, u, rho = mlp.features(hist[:4], fh, fm, s, 1e-3)
    return x, u, rho, s, hist[4] / rho


def _loss(p, x, u, s, t):
    out, _ = mlp.forward(p, x, u, s)
    return float(np.mean(np.abs(out - t) ** 2))


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    hidden = 12
    p = _small_params(rng, hidden)
    x, u, rho, s, t = _data(rng, 40)
    out, cache = mlp.forward(p, x, u, s)
    L, g = mlp.loss_and_grads(p, out, t, cache)
    assert abs(L - _loss(p, x, u, s, t)) < 1e-14
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = _loss(p, x, u, s, t)
            flat[i] = old - h
            lm = _loss(p, x, u, s, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].ravel()[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, an)


def test_planted_wrong_activation_derivative_is_caught():
    """Planted mistake: silu' replaced by sigmoid; the finite-difference pin must fail."""
    rng = np.random.default_rng(1)
    p = _small_params(rng, 8)
    x, u, rho, s, t = _data(rng, 30)
    orig = mlp.dsilu
    mlp.dsilu = lambda z: 1.0 / (1.0 + np.exp(-z))
    try:
        out, cache = mlp.forward(p, x, u, s)
        _, g = mlp.loss_and_grads(p, out, t, cache)
    finally:
        mlp.dsilu = orig
    flat = p["W1"].ravel()
    h = 1e-6
    worst = 0.0
    for i in range(flat.size):
        old = flat[i]
        flat[i] = old + h
        lp = _loss(p, x, u, s, t)
        flat[i] = old - h
        lm = _loss(p, x, u, s, t)
        flat[i] = old
        worst = max(worst, abs((lp - lm) / (2 * h) - g["W1"].ravel()[i]))
    assert worst > 1e-4


def test_skip_path_alone_is_exact_linear_predictor():
    """With the MLP output zeroed, out = sum_k c[s][k] u_k exactly (rotation z on both components)."""
    rng = np.random.default_rng(2)
    p = _small_params(rng, 8)
    for k in ("W3", "b3"):
        p[k] = np.zeros_like(p[k])
    z = np.exp(-1j * 0.7)
    p["c"][:] = 0.0
    p["c"][:, 0, 0], p["c"][:, 0, 1] = z.real, z.imag
    x, u, rho, s, t = _data(rng, 10)
    out, _ = mlp.forward(p, x, u, s)
    assert np.allclose(out, z * u[0], atol=1e-15)


def test_adam_first_step_closed_form():
    """First bias-corrected Adam step moves each parameter by lr * sign(g) (|g| >> eps)."""
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    mlp.adam_update(p, g, m, v, 1, 0.01)
    assert np.allclose(p["a"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], atol=1e-7)


def test_bf16_rounding_bit_patterns():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.140625, 65504.0])
    r = mlp.bf16_round(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even (1.0); 1 + 3*2^-9 rounds up
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert r[3] == -3.140625 and r[4] == 65536.0
