"""Pins of the FP64 surrogate oracle (CPU only).

The oracle's network is checked against things other than itself:
* torch.nn layers in float64 (a library forward of the same architecture);
* central finite differences of its own forward (input gradient, loss gradient);
* torch.autograd on the library forward;
* closed forms: silu and its derivative, the Fourier features at x = 0 and
  sin^2 + cos^2 = 1, Adam's first step lr * g / (|g| + eps);
* torch.optim.Adam over several steps;
* BF16 rounding against torch's float32 -> bfloat16 conversion and hand values.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_2108_10480_amd import scenes


def _params(seed=0, scale=1.0):
    th = scenes.surrogate_init(seed=seed).astype(np.float64) * scale
    B = scenes.fourier_matrix(seed=seed + 1).astype(np.float64)
    return th, B


def _torch_net(theta, B):
    p = M.unpack(theta)
    Bt = torch.tensor(B, dtype=torch.float64)
    layers = []
    ins = 2 * M.N_FREQ
    for l in range(1, M.DEPTH + 1):
        lin = torch.nn.Linear(ins, M.WIDTH, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.tensor(p[f"W{l}"]))
            lin.bias.copy_(torch.tensor(p[f"b{l}"]))
        layers += [lin, torch.nn.SiLU()]
        ins = M.WIDTH
    out = torch.nn.Linear(M.WIDTH, 1, dtype=torch.float64)
    with torch.no_grad():
        out.weight.copy_(torch.tensor(p["w5"][None, :]))
        out.bias.copy_(torch.tensor(p["b5"]))
    net = torch.nn.Sequential(*layers, out)

    def f(X):
        th = 2 * torch.pi * (X @ Bt.T)
        return net(torch.cat([torch.sin(th), torch.cos(th)], 1))[:, 0]
    return f, net


def test_parameter_count_and_layout():
    assert M.N_PARAMS == 128 * 256 + 256 + 3 * (256 * 256 + 256) + 256 + 1 == 230657
    assert sum(int(np.prod(s)) for s in scenes.surrogate_param_shapes()) == M.N_PARAMS
    th, _ = _params()
    assert np.array_equal(M.pack(M.unpack(th)), th)


def test_forward_matches_torch_layers():
    th, B = _params()
    X = np.random.default_rng(1).uniform(-1.5, 1.5, (300, 3))
    y, _ = M.forward(th, B, X)
    f, _ = _torch_net(th, B)
    yt = f(torch.tensor(X)).detach().numpy()
    np.testing.assert_allclose(y, yt, rtol=1e-12, atol=1e-13)


def test_input_gradient_finite_differences_and_autograd():
    th, B = _params(seed=3)
    X = np.random.default_rng(2).uniform(-1.5, 1.5, (40, 3))
    y, g = M.input_grad(th, B, X)
    h = 1e-6
    fd = np.zeros_like(X)
    for a in range(3):
        e = np.zeros(3); e[a] = h
        fd[:, a] = (M.forward(th, B, X + e)[0] - M.forward(th, B, X - e)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)
    f, _ = _torch_net(th, B)
    Xt = torch.tensor(X, requires_grad=True)
    f(Xt).sum().backward()
    np.testing.assert_allclose(g, Xt.grad.numpy(), rtol=1e-11, atol=1e-12)


def test_loss_gradient_finite_differences_and_autograd():
    th, B = _params(seed=5)
    rng = np.random.default_rng(4)
    X = rng.uniform(-1.5, 1.5, (64, 3))
    t = rng.normal(0, 0.5, 64)
    loss, g = M.loss_grad(th, B, X, t)
    # autograd of the library forward
    f, net = _torch_net(th, B)
    lt = ((f(torch.tensor(X)) - torch.tensor(t)) ** 2).mean()
    lt.backward()
    assert abs(loss - float(lt.detach())) < 1e-12 * max(1.0, loss)
    lin = [m for m in net if isinstance(m, torch.nn.Linear)]
    ref = {}
    for l in range(1, M.DEPTH + 1):
        ref[f"W{l}"] = lin[l - 1].weight.grad.numpy()
        ref[f"b{l}"] = lin[l - 1].bias.grad.numpy()
    ref["w5"] = lin[-1].weight.grad.numpy()[0]
    ref["b5"] = lin[-1].bias.grad.numpy()
    np.testing.assert_allclose(g, M.pack(ref), rtol=1e-10, atol=1e-13)
    # central differences on parameters from every block
    lay = M.layout()
    idx = []
    for name, shp, off in lay:
        n = int(np.prod(shp))
        idx += [off, off + n - 1, off + n // 2]
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th); e[i] = h
        fd = (M.loss_grad(th + e, B, X, t)[0] - M.loss_grad(th - e, B, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_silu_closed_forms():
    z = np.linspace(-30, 30, 1201)
    np.testing.assert_allclose(M.silu(z), z * (1 / (1 + np.exp(-z))), rtol=1e-15)
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert abs(M.silu(np.array([40.0]))[0] - 40.0) < 1e-12
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.silu_grad(z), fd, atol=1e-8)
    assert M.silu_grad(np.array([0.0]))[0] == 0.5
    # the maximum slope of silu (used in error propagation): 1.0998 near z = 2.3994
    zz = np.linspace(0, 5, 200001)
    assert abs(M.silu_grad(zz).max() - 1.0998) < 1e-4


def test_fourier_features_closed_forms():
    _, B = _params()
    g, _ = M.fourier(np.zeros((1, 3)), B)
    assert np.all(g[0, :64] == 0) and np.all(g[0, 64:] == 1)
    X = np.random.default_rng(5).uniform(-1.5, 1.5, (50, 3))
    g, th = M.fourier(X, B)
    np.testing.assert_allclose(g[:, :64] ** 2 + g[:, 64:] ** 2, 1.0, atol=1e-14)
    # one frequency along x: sin(2 pi k x)
    Bk = np.zeros((64, 3)); Bk[0, 0] = 3.0
    g, _ = M.fourier(X, Bk)
    np.testing.assert_allclose(g[:, 0], np.sin(6 * np.pi * X[:, 0]), atol=1e-14)


def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(6)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50); v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    t1, m1, v1 = M.adam_step(th, m, v, g, 1, lr, eps=eps)
    np.testing.assert_allclose(t1, th - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-16)
    # several steps against torch.optim.Adam (float64)
    p = torch.tensor(th, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=eps)
    cur, m, v = th.copy(), np.zeros(50), np.zeros(50)
    for k in range(1, 8):
        gk = rng.normal(size=50)
        opt.zero_grad()
        p.grad = torch.tensor(gk)
        opt.step()
        cur, m, v = M.adam_step(cur, m, v, gk, k, lr, eps=eps)
    np.testing.assert_allclose(cur, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_bf16_rounding():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -1 - 2 ** -8,
                     np.inf, -np.inf, 0.0, -0.0, 3.0e38, 1e-40], np.float32)
    r = M.bf16_round(vals)
    assert r[0] == one
    assert r[1] == one                       # tie goes to the even neighbour 1.0
    assert r[2] == one + 2 * ulp             # tie between 1+ulp (odd) and 1+2ulp (even)
    assert r[3] == one + ulp                 # just above the tie rounds up
    assert r[4] == -one
    assert r[5] == np.inf and r[6] == -np.inf and r[7] == 0 and np.signbit(r[8])
    assert np.isnan(M.bf16_round(np.array([np.nan], np.float32)))[0]
    x = np.random.default_rng(7).normal(0, 3, 100000).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_rounding_envelope_helper_reproduces_oracle():
    """The tolerance helper of the surrogate parity tests, unperturbed, is the
    oracle (so its rounding model cannot drift from the oracle's math)."""
    from tests import surrogate_ref as R
    th, B = _params(seed=8)
    X = np.random.default_rng(9).uniform(-1.5, 1.5, (64, 3))
    y, g = R.infer(th, B, X)
    y0, g0 = M.input_grad(th, B, X)
    np.testing.assert_allclose(y, y0, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(g, g0, rtol=1e-12, atol=1e-13)
    t = np.random.default_rng(10).normal(0, 0.3, 64)
    l, gr = R.loss_grad(th, B, X, t)
    l0, gr0 = M.loss_grad(th, B, X, t)
    assert abs(l - l0) < 1e-13
    np.testing.assert_allclose(gr, gr0, rtol=1e-12, atol=1e-15)
    # effective weights: BF16 matrices, FP32 biases
    te = R.effective_theta(th.astype(np.float32))
    p, q = M.unpack(te), M.unpack(th.astype(np.float32).astype(np.float64))
    assert np.array_equal(p["b2"], q["b2"]) and not np.array_equal(p["W2"], q["W2"])
    assert np.array_equal(p["W3"], M.bf16_round(q["W3"].astype(np.float32)).astype(np.float64))
