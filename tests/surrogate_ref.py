"""Tolerances of the surrogate parity tests, derived from where the library
rounds.

The library multiplies BF16 operands and accumulates in FP32; the oracle
(oracle/mlp.py) is FP64 with the same BF16-rounded weights.  The difference is
dominated by the BF16 rounding of activations (and, backwards, of the products
fed to the next matrix product): each rounding is a relative error of at most
u = 2^-8.  ``envelope`` re-runs the FP64 computation with every such rounding
replaced by an independent random relative perturbation in [-u, u] and
returns, per output, the largest deviation over the samples; the tests accept
the library's result within K times that envelope plus an FP32-level floor.

Rounding points mirrored here (everything else is FP32 in the library):
  inference  gamma; a_1..a_3 and silu'(z_1..z_3) (kept for the backward sweep);
             u_4 = w5 silu'(z_4); u_l = (W_{l+1}^T u_{l+1}) silu'(z_l), l = 1..3
  training   gamma; a_1..a_4; G_4 = dy w5 silu'(z_4); G_l = (G_{l+1} W_{l+1}) silu'(z_l)

With no perturbation the functions below reproduce the oracle exactly (a CPU
test checks that), so they cannot drift from it.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp as M

U_BF16 = 2.0 ** -8


def effective_theta(theta32):
    """The network the library evaluates: BF16 W1..W4 and w5, FP32 biases."""
    th = np.asarray(theta32, np.float32).copy()
    for name, shp, off in M.layout():
        if name.startswith("W") or name == "w5":
            n = int(np.prod(shp))
            th[off:off + n] = M.bf16_round(th[off:off + n])
    return th.astype(np.float64)


def _p(x, rng):
    if rng is None:
        return x
    return x * (1.0 + rng.uniform(-U_BF16, U_BF16, x.shape))


def infer(theta, B, X, rng=None):
    """(y, dy/dx) with perturbations at the inference rounding points."""
    p = M.unpack(theta)
    g, th = M.fourier(X, B)
    a = _p(g, rng)
    z, sp = [], []
    for l in range(1, M.DEPTH + 1):
        zl = a @ p[f"W{l}"].T + p[f"b{l}"]
        z.append(zl)
        al = M.silu(zl)
        s = M.silu_grad(zl)
        if l < M.DEPTH:
            al, s = _p(al, rng), _p(s, rng)
        sp.append(s)
        a = al
    y = a @ p["w5"] + p["b5"][0]
    u = _p(p["w5"][None, :] * sp[-1], rng)
    for l in range(M.DEPTH, 1, -1):
        u = _p((u @ p[f"W{l}"]) * sp[l - 2], rng)
    gg = u @ p["W1"]
    gs, gc = gg[:, :M.N_FREQ], gg[:, M.N_FREQ:]
    coef = 2.0 * np.pi * (gs * np.cos(th) - gc * np.sin(th))
    return y, coef @ np.asarray(B, np.float64)


def loss_grad(theta, B, X, t, rng=None):
    """(loss, flat gradient) with perturbations at the training rounding points."""
    p = M.unpack(theta)
    g, _ = M.fourier(X, B)
    a = [_p(g, rng)]
    z = []
    a4f = None
    for l in range(1, M.DEPTH + 1):
        zl = a[-1] @ p[f"W{l}"].T + p[f"b{l}"]
        z.append(zl)
        al = M.silu(zl)
        if l == M.DEPTH:
            a4f = al
        a.append(_p(al, rng))
    y = a4f @ p["w5"] + p["b5"][0]
    n = len(y)
    r = y - np.asarray(t, np.float64)
    dy = 2.0 * r / n
    G = [None] * M.DEPTH
    G[-1] = _p(dy[:, None] * p["w5"][None, :] * M.silu_grad(z[-1]), rng)
    for l in range(M.DEPTH, 1, -1):
        G[l - 2] = _p((G[l - 1] @ p[f"W{l}"]) * M.silu_grad(z[l - 2]), rng)
    out = {"w5": a4f.T @ dy, "b5": np.array([dy.sum()])}
    for l in range(1, M.DEPTH + 1):
        out[f"W{l}"] = G[l - 1].T @ a[l - 1]
        out[f"b{l}"] = G[l - 1].sum(0)
    return float(np.mean(r * r)), M.pack(out)


def envelope(fn, *args, samples=16, seed=0):
    """Exact result and, per output, the largest deviation over `samples`
    perturbed runs (outputs flattened and concatenated)."""
    flat = lambda res: np.concatenate([np.atleast_1d(np.asarray(x, np.float64)).ravel() for x in res])
    ref = flat(fn(*args, rng=None))
    rng = np.random.default_rng(seed)
    dev = np.zeros_like(ref)
    for _ in range(samples):
        dev = np.maximum(dev, np.abs(flat(fn(*args, rng=rng)) - ref))
    return ref, dev
