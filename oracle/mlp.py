"""FP64 reference ("oracle") for the learned surrogate of the smooth distance.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg import this module.  It shares no code with the
HIP library and never calls it: plain numpy in FP64.

The paper has no surrogate; the network below is the fixed architecture the
library trains (its only readings are listed with each function):

  gamma(x) = [sin(2 pi B x), cos(2 pi B x)]     B: 64 x 3 frequencies, 128 features
  z_l = W_l a_{l-1} + b_l,  a_l = silu(z_l)     l = 1..4, width 256, a_0 = gamma(x)
  y = w5 . a_4 + b5                             the surrogate of the smooth distance

silu(z) = z / (1 + exp(-z)).  Training minimises the mean squared error against
labels produced by the exact method (Eq. 3) with Adam (bias-corrected moments).

Parameters are one flat vector, in this order (row-major matrices, W_l is
out x in): W1 (256x128), b1, W2 (256x256), b2, W3, b3, W4, b4, w5 (256), b5.

The library computes with BF16 weights; tests pass those weights here promoted
to FP64 (``bf16_round`` gives the round-to-nearest-even BF16 value of FP32
masters).  Activations stay FP64 here.
"""
from __future__ import annotations

import numpy as np

N_FREQ = 64
WIDTH = 256
DEPTH = 4
N_IN = 2 * N_FREQ


def layout():
    """[(name, shape, offset)] of the flat parameter vector."""
    shapes = [("W1", (WIDTH, N_IN)), ("b1", (WIDTH,))]
    for l in range(2, DEPTH + 1):
        shapes += [(f"W{l}", (WIDTH, WIDTH)), (f"b{l}", (WIDTH,))]
    shapes += [("w5", (WIDTH,)), ("b5", (1,))]
    out, off = [], 0
    for name, shp in shapes:
        out.append((name, shp, off))
        off += int(np.prod(shp))
    return out


N_PARAMS = sum(int(np.prod(s)) for _, s, _ in layout())


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    assert theta.shape == (N_PARAMS,)
    return {name: theta[off:off + int(np.prod(shp))].reshape(shp) for name, shp, off in layout()}


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _, _ in layout()])


def bf16_round(a):
    """Round FP32 values to the nearest BF16 value (ties to even), returned as
    FP32.  Written from the definition: keep the upper 16 bits of the FP32
    encoding after adding half a BF16 unit in the last place, plus one when
    the kept part is odd and the dropped part is exactly half.  NaN stays NaN."""
    a = np.ascontiguousarray(np.asarray(a, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    keep_odd = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + keep_odd) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), np.float32(np.nan), out).astype(np.float32)


def fourier(X, B):
    """gamma(x): sines of 2 pi B x followed by cosines of the same arguments."""
    th = 2.0 * np.pi * (np.asarray(X, np.float64) @ np.asarray(B, np.float64).T)
    return np.concatenate([np.sin(th), np.cos(th)], axis=1), th


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    """d silu / dz = s (1 + z (1 - s)) with s the logistic function."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, B, X):
    """Surrogate value for every row of X (n x 3).  Returns (y, cache)."""
    p = unpack(theta)
    g, th = fourier(X, B)
    a = [g]
    z = []
    for l in range(1, DEPTH + 1):
        zl = a[-1] @ p[f"W{l}"].T + p[f"b{l}"]
        z.append(zl)
        a.append(silu(zl))
    y = a[-1] @ p["w5"] + p["b5"][0]
    return y, {"p": p, "a": a, "z": z, "theta": th, "B": np.asarray(B, np.float64)}


def _backward_to_gamma(cache, dy):
    """dL/d gamma for upstream dL/dy = dy (n), plus dL/dz_l for every layer."""
    p, a, z = cache["p"], cache["a"], cache["z"]
    u = dy[:, None] * p["w5"][None, :] * silu_grad(z[-1])      # dL/dz_4
    dz = [None] * DEPTH
    dz[DEPTH - 1] = u
    for l in range(DEPTH, 1, -1):
        u = (u @ p[f"W{l}"]) * silu_grad(z[l - 2])
        dz[l - 2] = u
    return dz[0] @ p["W1"], dz


def input_grad(theta, B, X):
    """(y, dy/dx) for every row of X: chain rule through the layers and the
    Fourier features, d sin(2 pi b.x)/dx = 2 pi b cos(2 pi b.x), d cos/dx =
    -2 pi b sin."""
    y, c = forward(theta, B, X)
    gg, _ = _backward_to_gamma(c, np.ones_like(y))
    th, Bm = c["theta"], c["B"]
    gs, gc = gg[:, :N_FREQ], gg[:, N_FREQ:]
    coef = 2.0 * np.pi * (gs * np.cos(th) - gc * np.sin(th))     # n x 64
    return y, coef @ Bm


def loss_grad(theta, B, X, t):
    """Mean squared error L = mean((y - t)^2) and dL/dtheta (flat, FP64)."""
    y, c = forward(theta, B, X)
    n = len(y)
    r = y - np.asarray(t, np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    _, dz = _backward_to_gamma(c, dy)
    a = c["a"]
    g = {"w5": a[-1].T @ dy, "b5": np.array([dy.sum()])}
    for l in range(1, DEPTH + 1):
        g[f"W{l}"] = dz[l - 1].T @ a[l - 1]
        g[f"b{l}"] = dz[l - 1].sum(0)
    return loss, pack(g)


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1): moments m <- b1 m + (1-b1) g,
    v <- b2 v + (1-b2) g^2, bias corrections 1 - b^step, then
    theta <- theta - lr m_hat / (sqrt(v_hat) + eps)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
