"""Python binding of the learned surrogate (sd_surrogate_* and sd_eval_surrogate
in include/sd.h) and the training driver.

Argument marshalling only: the network's forward and backward passes, the
loss, Adam, certification, routing and the exact fallback all run in the HIP
kernels behind the C ABI.  The driver below chooses batches (a seeded
shuffled order per epoch, passed to the library as an index array) and the
learning rate of each step (cosine schedule).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import api, scenes
from .api import _c_p, _check, _dptr, _i64, _stream, lib

N_PARAMS = 230657
N_FREQ = 64


class Surrogate:
    """Owns an sd_surrogate handle."""

    def __init__(self, B, theta, max_batch=65536):
        B = np.ascontiguousarray(B, np.float32)
        theta = np.ascontiguousarray(theta, np.float32)
        if B.shape != (N_FREQ, 3) or theta.shape != (N_PARAMS,):
            raise ValueError("B must be 64 x 3 and theta must hold 230657 parameters")
        h = _c_p()
        _check(lib().sd_surrogate_create(_c_p(B.ctypes.data), _c_p(theta.ctypes.data),
                                         _i64(max_batch), _stream(), ctypes.byref(h)))
        self._h = h
        self.max_batch = max_batch

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("surrogate already freed")
        return self._h

    def free(self):
        if self._h is not None and api._lib is not None:
            lib().sd_surrogate_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def forward(self, Q, grad=True):
        Qp, n = _dptr(Q, torch.float32, "Q", 3)
        d = torch.empty(n, dtype=torch.float32, device=Q.device)
        g = torch.empty((n, 3), dtype=torch.float32, device=Q.device) if grad else None
        _check(lib().sd_surrogate_forward(self.handle, Qp, _i64(n), _c_p(d.data_ptr()),
                                          _c_p(g.data_ptr() if g is not None else 0), _stream()))
        return (d, g) if grad else d

    def loss_grad(self, X, labels, idx=None, n=None):
        Xp, nx = _dptr(X, torch.float32, "X", 3)
        yp, ny = _dptr(labels, torch.float32, "labels")
        if ny != nx:
            raise ValueError("X and labels disagree on the number of rows")
        ip, ni = _dptr(idx, torch.int32, "idx")
        n = n if n is not None else (ni if idx is not None else nx)
        grad = torch.empty(N_PARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(lib().sd_surrogate_loss_grad(self.handle, Xp, yp, _i64(nx), ip, _i64(n), _c_p(grad.data_ptr()),
                                            _c_p(loss.data_ptr()), _stream()))
        return grad, loss

    def adam(self, lr, grad=None):
        gp = _c_p(0) if grad is None else _dptr(grad, torch.float32, "grad")[0]
        _check(lib().sd_surrogate_adam(self.handle, gp, ctypes.c_float(lr), _stream()))

    def train_step(self, X, labels, idx_ptr, n, lr, loss_ptr=0):
        """One step on the batch rows idx[0..n) (idx_ptr: device address of
        int32 indices into X / labels)."""
        if X.shape[0] != labels.shape[0]:
            raise ValueError("X and labels disagree on the number of rows")
        _check(lib().sd_surrogate_train_step(self.handle, _c_p(X.data_ptr()), _c_p(labels.data_ptr()),
                                             _i64(X.shape[0]), _c_p(idx_ptr), _i64(n), ctypes.c_float(lr),
                                             _c_p(loss_ptr), _stream()))

    def certify(self, X, labels, safety=1.5):
        Xp, n = _dptr(X, torch.float32, "X", 3)
        yp, _ = _dptr(labels, torch.float32, "labels")
        eps = ctypes.c_float()
        _check(lib().sd_surrogate_certify(self.handle, Xp, yp, _i64(n), ctypes.c_float(safety),
                                          _stream(), ctypes.byref(eps)))
        return eps.value

    def certify_cells(self, X, labels, lo, hi, grid=32, safety=1.5, max_margin=math.inf):
        """Global margin (returned) plus a grid of local margins over [lo, hi];
        cells whose margin exceeds max_margin route every query."""
        Xp, n = _dptr(X, torch.float32, "X", 3)
        yp, _ = _dptr(labels, torch.float32, "labels")
        lo = np.ascontiguousarray(lo, np.float32)
        hi = np.ascontiguousarray(hi, np.float32)
        eps = ctypes.c_float()
        _check(lib().sd_surrogate_certify_cells(self.handle, Xp, yp, _i64(n), ctypes.c_float(safety),
                                                ctypes.c_int(grid), _c_p(lo.ctypes.data), _c_p(hi.ctypes.data),
                                                ctypes.c_float(max_margin), _stream(), ctypes.byref(eps)))
        return eps.value

    def save(self):
        th, m, v = (np.empty(N_PARAMS, np.float32) for _ in range(3))
        B = np.empty((N_FREQ, 3), np.float32)
        step, eps = ctypes.c_int64(), ctypes.c_float()
        f = lambda a: _c_p(a.ctypes.data)
        _check(lib().sd_surrogate_save(self.handle, f(th), f(m), f(v), f(B), ctypes.byref(step),
                                       ctypes.byref(eps)))
        return dict(theta=th, m=m, v=v, B=B, step=step.value, eps_cert=eps.value)

    def load(self, theta, m=None, v=None, step=0, eps_cert=math.inf):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (theta, m, v)]
        f = lambda a: _c_p(0 if a is None else a.ctypes.data)
        _check(lib().sd_surrogate_load(self.handle, f(arrs[0]), f(arrs[1]), f(arrs[2]), _i64(step),
                                       ctypes.c_float(eps_cert), _stream()))


def sd_eval_surrogate(scene, sur, Q, alpha, beta=0.5, band=0.05, alpha_u=0.0, flags=0, out=None,
                      grad_out=None, routed=None):
    """(d, grad, routed flags, number of exactly evaluated queries as a
    one-element int32 tensor on the device: the call does not wait for the
    GPU; int() of it does)."""
    Qp, n = _dptr(Q, torch.float32, "Q", 3)
    d = out if out is not None else torch.empty(n, dtype=torch.float32, device=Q.device)
    g = grad_out if grad_out is not None else torch.empty((n, 3), dtype=torch.float32, device=Q.device)
    r = routed if routed is not None else torch.empty(n, dtype=torch.uint8, device=Q.device)
    p = api.params(alpha, beta, alpha_u, flags)
    nfb = torch.empty(1, dtype=torch.int32, device=Q.device)
    _check(lib().sd_eval_surrogate(scene.handle, sur.handle, Qp, _i64(n), ctypes.byref(p),
                                   ctypes.c_float(band), _c_p(d.data_ptr()), _c_p(g.data_ptr()),
                                   _c_p(r.data_ptr()), _c_p(nfb.data_ptr()), _stream()))
    return d, g, r, nfb


def cosine_lr(step, total, lr0, lr_min, warmup=0):
    """Linear warm-up over `warmup` steps, then cosine decay to lr_min."""
    if step < warmup:
        return lr0 * (step + 1) / warmup
    t = (step - warmup) / max(total - warmup, 1)
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * min(t, 1.0)))


def train(sur, X, labels, epochs, batch=65536, lr0=3e-3, lr_min=1e-5, seed=13, log_every=0, warmup=0,
          on_epoch=None):
    """Adam over `epochs` passes of (X, labels) (device tensors) in seeded
    shuffled order; returns the per-step losses (host array).  on_epoch(e, k),
    when given, runs after epoch e (1-based) with k steps done."""
    n = X.shape[0]
    steps_per_epoch = n // batch
    if steps_per_epoch == 0:
        raise ValueError("fewer samples than one batch")
    total = epochs * steps_per_epoch
    losses = torch.empty(total, dtype=torch.float32, device=X.device)
    k = 0
    for ep in range(epochs):
        order = torch.as_tensor(scenes.epoch_order(n, ep, seed), device=X.device)
        base = order.data_ptr()
        for b in range(steps_per_epoch):
            lr = cosine_lr(k, total, lr0, lr_min, warmup)
            sur.train_step(X, labels, base + 4 * b * batch, batch, lr, losses.data_ptr() + 4 * k)
            k += 1
        if log_every and (ep + 1) % log_every == 0:
            print(f"epoch {ep + 1}/{epochs} loss {float(losses[k - 1]):.3e}", flush=True)
        if on_epoch is not None:
            on_epoch(ep + 1, k)
    return losses.cpu().numpy()
