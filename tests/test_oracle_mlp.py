"""Pins of the warm-start oracle (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 (Random123 distribution)."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = mlp.philox4x32_10(*[np.array([c]) for c in ctr], key[0], key[1])
        assert tuple(int(g[0]) for g in got) == want


def test_uniforms_and_normals():
    assert mlp.u01(0)[()] == 0.5 / 2**24 if np.ndim(mlp.u01(0)) else mlp.u01(0) == 0.5 / 2**24
    assert float(mlp.u01(np.uint32(0xFFFFFFFF))) == (2**24 - 0.5) / 2**24
    n = mlp.training_noise(123, 0, 50000, 8)
    assert abs(n.mean()) < 5 / math.sqrt(n.size)
    assert abs(n.var() - 1) < 5 * math.sqrt(2 / n.size)
    # independent columns
    c = np.corrcoef(n.T)
    assert np.abs(c - np.eye(8)).max() < 0.03


def test_training_state_distribution():
    x0 = np.array([0.01, 1000.0, 150.0, 0.2, 0.0])
    x = mlp.draw_training_states(7, 0, 200000, x0)
    lf = np.log(x[:, 0])
    # log-uniform f: uniform log f on [ln 1e-4, ln 0.3]
    a, b = math.log(1e-4), math.log(0.3)
    assert abs(lf.mean() - (a + b) / 2) < 0.02 and abs(lf.var() - (b - a) ** 2 / 12) < 0.03
    assert x[:, 1].min() >= 600 and x[:, 1].max() <= 1400 and abs(x[:, 1].mean() - 1000) < 3
    assert abs(x[:, 2].mean() - 175) < 1 and abs(x[:, 4].mean()) < 1e-6
    # offsets index the same stream
    np.testing.assert_array_equal(mlp.draw_training_states(7, 100, 50, x0), x[100:150])
    xb = mlp.draw_training_states(7, 0, 20000, x0, bg_fraction=0.25)
    assert abs((xb[:, 0] == 0).mean() - 0.25) < 0.015


def test_gelu_identities():
    x = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-15)   # odd part is x/2 * 2
    assert mlp.gelu(0.0) == 0.0 and mlp.gelu_grad(0.0) == 0.5
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-8)
    # the tanh form stays within 2e-3 of the exact x Phi(x)
    from scipy.special import erf
    np.testing.assert_allclose(mlp.gelu(x), 0.5 * x * (1 + erf(x / math.sqrt(2))), atol=2e-3)


def test_backprop_matches_finite_differences():
    sizes = (6, 8, 7, 5, 3)
    p = mlp.init_params(sizes, 3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(9, 6))
    t = np.tanh(rng.normal(size=(9, 3)))
    loss, g = mlp.loss_and_grads(p, sizes, X, t)
    assert g.shape == p.shape == (mlp.n_params(sizes),)
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd[i] = (mlp.loss_and_grads(p + e, sizes, X, t)[0] - mlp.loss_and_grads(p - e, sizes, X, t)[0]) / 2e-6
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-10)


def test_adam_first_step_closed_form():
    """After one step from zero moments the bias-corrected update is
    lr * g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=100)
    g = rng.normal(size=100)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(100), np.zeros(100), 1, lr=0.01)
    np.testing.assert_allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_round_bf16():
    """bfloat16 keeps the top 16 bits of a float32, rounding to nearest even."""
    assert mlp.round_bf16(np.float32(1.0)) == 1.0
    assert mlp.round_bf16(1.0 + 2.0**-8) == 1.0                       # tie -> even (1.0)
    assert mlp.round_bf16(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6         # tie -> even (up)
    assert mlp.round_bf16(1.0 + 2.0**-8 + 2.0**-20) == 1.0 + 2.0**-7  # above the tie
    assert mlp.round_bf16(-3.0) == -3.0
    x = np.random.default_rng(0).normal(size=10000)
    r = mlp.round_bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0**-8)
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
