"""FP64 oracle of the learned warm start (test infrastructure only).

  * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): 10 rounds of
    (hi, lo) = M * c on counters (c0, c2) with M0 = 0xD2511F53,
    M1 = 0xCD9E8D57, new state (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0), key
    bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.
  * uniforms u = (x >> 8 + 1/2) / 2^24 and Box-Muller normals.
  * the training-data draw: one-component states f ~ logU[1e-4, 0.3],
    m ~ U[600, 1400] K, s ~ U[50, 300] K, rho0 ~ U[0.05, 0.4],
    rho1 ~ U[-1e-4, 1e-4] /nm; sample g uses Philox blocks (g, 0), (g, 1) for
    the state and (g, 2 + b/4) for the noise of bands 4(b/4) .. +3.
  * a multilayer perceptron n_in -> h1 -> h2 -> h3 -> n_out with GELU in
    its tanh form (Hendrycks & Gimpel 2016) on hidden layers and tanh on
    the output; mean-squared-error loss and its gradient by reverse-mode
    differentiation written out layer by layer; Adam (Kingma & Ba 2015 --
    the update of the paper's Sec. 2.5).
Parameter layout: W1 [h1][n_in], b1, W2 [h2][h1], b2, W3 [h3][h2], b3,
W4 [n_out][h3], b4, flattened row-major.
"""
from __future__ import annotations

import math

import numpy as np

from . import forward as _forward

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 arrays (broadcast)."""
    c0, c1, c2, c3 = (np.asarray(x, np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    for r in range(10):
        if r > 0:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return [x.astype(np.uint32) for x in (c0, c1, c2, c3)]


def u01(x):
    return ((np.asarray(x, np.uint32) >> np.uint32(8)).astype(np.float64) + 0.5) / 16777216.0


def draw_training_states(seed, offset, P, x0, bg_fraction=0.0):
    g = np.uint64(offset) + np.arange(P, dtype=np.uint64)
    glo = g & np.uint64(MASK)
    ghi = g >> np.uint64(32)
    k0, k1 = seed & MASK, (seed >> 32) & MASK
    r0 = philox4x32_10(glo, ghi, 0, 0, k0, k1)
    r1 = philox4x32_10(glo, ghi, 1, 0, k0, k1)
    lf0, lf1 = math.log(1e-4), math.log(0.3)
    x = np.empty((P, 5))
    x[:, 0] = np.exp(lf0 + (lf1 - lf0) * u01(r0[0]))
    x[:, 1] = 600.0 + 800.0 * u01(r0[1])
    x[:, 2] = 50.0 + 250.0 * u01(r0[2])
    x[:, 3] = 0.05 + 0.35 * u01(r0[3])
    x[:, 4] = -1e-4 + 2e-4 * u01(r1[0])
    bg = u01(r1[1]) < bg_fraction
    x[bg, 0] = 0.0
    x[bg, 1] = x0[1]
    x[bg, 2] = x0[2]
    return x


def training_noise(seed, offset, P, B):
    """Standard normals [P, B]: Box-Muller on Philox blocks (g, 2 + b/4)."""
    g = np.uint64(offset) + np.arange(P, dtype=np.uint64)
    glo = g & np.uint64(MASK)
    ghi = g >> np.uint64(32)
    k0, k1 = seed & MASK, (seed >> 32) & MASK
    out = np.empty((P, ((B + 3) // 4) * 4))
    for j in range((B + 3) // 4):
        r = philox4x32_10(glo, ghi, 2 + j, 0, k0, k1)
        for h in range(2):
            ua, ub = u01(r[2 * h]), u01(r[2 * h + 1])
            rr = np.sqrt(-2.0 * np.log(ua))
            out[:, 4 * j + 2 * h] = rr * np.cos(2 * np.pi * ub)
            out[:, 4 * j + 2 * h + 1] = rr * np.sin(2 * np.pi * ub)
    return out[:, :B]


def generate(tab, lo, hi, x0, seed, offset, P, snr=300.0, bg_fraction=0.0):
    """(radiance float32 [P, B], target z [P, 5], states [P, 5]) of the
    training-data draw, with the oracle's FP64 forward model."""
    x = draw_training_states(seed, offset, P, x0, bg_fraction)
    L = _forward(tab, x, 1)
    if snr and snr > 0:
        L = L * (1.0 + training_noise(seed, offset, P, tab.B) / snr)
    z = np.clip(2.0 * (x - lo) / (hi - lo) - 1.0, -1.0, 1.0)
    return L.astype(np.float32), z, x


# ----------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------
def layer_shapes(n_in, h1, h2, h3, n_out):
    ins = [n_in, h1, h2, h3]
    outs = [h1, h2, h3, n_out]
    return list(zip(outs, ins))


def n_params(sizes):
    return sum(o * i + o for o, i in layer_shapes(*sizes))


def unflatten(p, sizes):
    layers, off = [], 0
    for o, i in layer_shapes(*sizes):
        W = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        layers.append((W, b))
    return layers


def init_params(sizes, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for l, (o, i) in enumerate(layer_shapes(*sizes)):
        sd = math.sqrt(2.0 / i) * (0.1 if l == 3 else 1.0)
        parts.append(rng.normal(0.0, sd, o * i))
        parts.append(rng.normal(0.0, 0.05, o))
    return np.concatenate(parts)


_C = math.sqrt(2.0 / math.pi)
_A = 0.044715


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_C * (x + _A * x ** 3)))


def gelu_grad(x):
    t = np.tanh(_C * (x + _A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _C * (1.0 + 3.0 * _A * x * x)


def features(L, mean, inv_std, floor):
    return (np.log(np.maximum(np.asarray(L, np.float64), floor)) - mean) * inv_std


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, sizes, X, bf16_storage=False):
    """z = tanh(network(X)); returns z and the per-layer cache.

    bf16_storage rounds every layer input and weight matrix to bfloat16
    (biases and sums stay exact), the storage format of a matrix-core
    implementation, so that a comparison with one isolates summation order.
    """
    layers = unflatten(p, sizes)
    q = round_bf16 if bf16_storage else (lambda v: v)
    a = X
    cache = []
    for l, (W, b) in enumerate(layers):
        h = q(a) @ q(W).T + b
        cache.append((a, h))
        a = gelu(h) if l < 3 else h
    return np.tanh(a), cache


def loss_and_grads(p, sizes, X, target):
    """loss = mean((z - t)^2) and its gradient (flat, parameter layout)."""
    z, cache = forward(p, sizes, X)
    n = z.size
    loss = float(np.mean((z - target) ** 2))
    d = 2.0 * (z - target) / n * (1.0 - z * z)   # d loss / d pre-tanh output
    layers = unflatten(p, sizes)
    grads = [None] * 4
    for l in range(3, -1, -1):
        a_in, h = cache[l]
        if l < 3:
            d = d * gelu_grad(h)
        W, _ = layers[l]
        grads[l] = (d.T @ a_in, d.sum(axis=0))
        d = d @ W
    return loss, np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
