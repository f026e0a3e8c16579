"""GPU: the learned surrogate's kernels against the FP64 oracle (oracle/mlp.py).

* inference (value and input gradient) and the training loss gradient, with
  tolerances from the library's BF16 rounding points (tests/surrogate_ref.py);
* Adam against the oracle's update, train_step = loss_grad + adam bitwise;
* certification, save/load, routing to the exact evaluation.
"""
import numpy as np
import pytest

from oracle import mlp as M
from tests import surrogate_ref as R
from tests.gpu_common import api, cuda, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu

K_ENV = 4.0   # accept K_ENV times the largest deviation of 16 perturbed runs


def _surrogate(seed=0, scale=1.0, max_batch=256):
    from paper_2108_10480_amd import surrogate as S
    th = (scenes.surrogate_init(seed=seed) * np.float32(scale)).astype(np.float32)
    B = scenes.fourier_matrix(seed=seed + 1)
    return S.Surrogate(B, th, max_batch=max_batch), th, B


def _check_infer(sur, th, B, X, what):
    d, g = sur.forward(cuda(X))
    d, g = d.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    n = len(X)
    ref, dev = R.envelope(R.infer, R.effective_theta(th), B.astype(np.float64), X.astype(np.float64))
    yr, gr = ref[:n], ref[n:].reshape(n, 3)
    yd, gd = dev[:n], dev[n:].reshape(n, 3)
    # FP32 floor: accumulation and hardware exp2 / rcp / sin errors
    fy = 2.0 ** -16 * (np.abs(yr) + np.abs(yr).mean())
    fg = 2.0 ** -16 * (np.abs(gr) + np.abs(gr).mean())
    ey = np.abs(d - yr) / (K_ENV * yd + fy)
    eg = np.abs(g - gr) / (K_ENV * gd + fg)
    print(f"{what}: value err/tol max {ey.max():.3f}, grad err/tol max {eg.max():.3f}, "
          f"typical rel value err {np.median(np.abs(d - yr) / (np.abs(yr) + 1e-3)):.2e}")
    assert ey.max() <= 1.0, f"{what}: value"
    assert eg.max() <= 1.0, f"{what}: gradient"
    return d, g


@pytest.mark.parametrize("scale", [1.0, 3.0])
def test_forward_matches_oracle(scale):
    require_gpu()
    sur, th, B = _surrogate(seed=1, scale=scale)
    # several workgroups of 128 queries and a ragged tail
    X = np.random.default_rng(2).uniform(-1.5, 1.5, (1000 + 77, 3)).astype(np.float32)
    d, g = _check_infer(sur, th, B, X, f"scale {scale}")
    # the value-only kernel computes the same forward pass
    d2 = sur.forward(cuda(X), grad=False).cpu().numpy()
    assert np.array_equal(d2, d.astype(np.float32))
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(g))


def test_forward_edge_cases():
    require_gpu()
    sur, th, B = _surrogate(seed=3)
    d = sur.forward(cuda(np.zeros((0, 3), np.float32)), grad=False)
    assert d.numel() == 0
    X = np.array([[0, 0, 0], [np.nan, 0, 0], [1e3, -1e3, 5e2]], np.float32)
    d, g = sur.forward(cuda(X))
    d, g = d.cpu().numpy(), g.cpu().numpy()
    assert np.isnan(d[1]) and np.isfinite(d[0]) and np.isfinite(d[2])
    y0, g0 = M.input_grad(R.effective_theta(th), B.astype(np.float64), X[[0]].astype(np.float64))
    assert abs(d[0] - y0[0]) < 0.05 * (abs(y0[0]) + 0.01)
    # single query (one live lane in the workgroup)
    d1 = sur.forward(cuda(X[[0]]), grad=False).cpu().numpy()
    assert d1[0] == d[0]


def test_loss_gradient_matches_oracle():
    require_gpu()
    sur, th, B = _surrogate(seed=4, scale=2.0, max_batch=512)
    rng = np.random.default_rng(5)
    X = rng.uniform(-1.5, 1.5, (700, 3)).astype(np.float32)
    t = rng.normal(0.0, 0.4, 700).astype(np.float32)
    idx = rng.permutation(700)[:320].astype(np.int32)
    for use_idx in (False, True):
        n = 320
        rows = idx if use_idx else np.arange(n)
        gr, loss = sur.loss_grad(cuda(X), cuda(t), cuda(idx) if use_idx else None, n=n)
        gr, loss = gr.cpu().numpy().astype(np.float64), float(loss.cpu()[0])
        ref, dev = R.envelope(R.loss_grad, R.effective_theta(th), B.astype(np.float64),
                              X[rows].astype(np.float64), t[rows].astype(np.float64))
        lref, gref, gdev = ref[0], ref[1:], dev[1:]
        assert abs(loss - lref) <= K_ENV * dev[0] + 1e-6 * lref, (loss, lref)
        floor = 2.0 ** -14 * (np.abs(gref) + np.abs(gref).mean())
        e = np.abs(gr - gref) / (K_ENV * gdev + floor)
        worst = int(np.argmax(e))
        print(f"idx={use_idx}: grad err/tol max {e.max():.3f} at {worst} "
              f"({[nm for nm, s, o in M.layout() if o <= worst][-1]})")
        assert e.max() <= 1.0


def test_adam_matches_oracle_and_train_step():
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    sur, th, B = _surrogate(seed=6)
    rng = np.random.default_rng(7)
    th64, m, v = th.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    for step, lr in ((1, 1e-3), (2, 5e-4), (3, 2e-3)):
        g = (rng.normal(0, 1e-2, M.N_PARAMS) * rng.uniform(0, 3, M.N_PARAMS)).astype(np.float32)
        sur.adam(lr, grad=cuda(g))
        st = sur.save()
        g64 = g.astype(np.float64)
        # FP32 rounding of each moment update is relative to the magnitudes of
        # its two terms (they may cancel), of the parameter update to lr
        tol_m = 2.0 ** -21 * (0.9 * np.abs(m) + 0.1 * np.abs(g64))
        tol_v = 2.0 ** -21 * (0.999 * v + 0.001 * g64 * g64)
        th_prev = th64
        th64, m, v = M.adam_step(th64, m, v, g64, step, lr)
        assert st["step"] == step
        assert np.all(np.abs(st["m"] - m) <= tol_m)
        assert np.all(np.abs(st["v"] - v) <= tol_v)
        assert np.all(np.abs(st["theta"] - th64) <= 2.0 ** -23 * np.abs(th_prev) + 1e-5 * lr)
        th64, m, v = (st[k].astype(np.float64) for k in ("theta", "m", "v"))
    # the BF16 copies follow the update
    X = np.random.default_rng(8).uniform(-1.5, 1.5, (300, 3)).astype(np.float32)
    _check_infer(sur, st["theta"], B, X, "after adam")
    # train_step == loss_grad + adam, bitwise
    a, th0, _ = _surrogate(seed=9, max_batch=128)
    b = S.Surrogate(scenes.fourier_matrix(seed=10), th0, max_batch=128)
    Xd = cuda(X[:128])
    t = cuda(np.random.default_rng(11).normal(0, 0.3, 128).astype(np.float32))
    a.train_step(Xd, t, 0, 128, 1e-3)
    a.train_step(Xd, t, 0, 128, 1e-3)
    for _ in range(2):
        b.loss_grad(Xd, t)
        b.adam(1e-3)
    torch.cuda.synchronize()
    assert np.array_equal(a.save()["theta"], b.save()["theta"])


def test_certify_save_load():
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    sur, th, B = _surrogate(seed=12)
    X = np.random.default_rng(13).uniform(-1.5, 1.5, (5000, 3)).astype(np.float32)
    lab = np.random.default_rng(14).normal(0, 0.2, 5000).astype(np.float32)
    eps = sur.certify(cuda(X), cuda(lab), safety=1.5)
    y = sur.forward(cuda(X), grad=False).cpu().numpy()
    assert eps == np.float32(1.5) * np.abs(y - lab).max()
    st = sur.save()
    assert st["eps_cert"] == eps and np.array_equal(st["B"], B) and np.array_equal(st["theta"], th)
    th2 = scenes.surrogate_init(seed=15)
    sur.load(th2, step=7, eps_cert=0.25)
    st = sur.save()
    assert st["step"] == 7 and st["eps_cert"] == np.float32(0.25) and np.array_equal(st["theta"], th2)
    assert not st["m"].any() and not st["v"].any()
    fresh = S.Surrogate(B, th2, max_batch=0)
    assert torch.equal(sur.forward(cuda(X), grad=False), fresh.forward(cuda(X), grad=False))


def test_invalid_arguments():
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    th = scenes.surrogate_init(seed=0)
    B = scenes.fourier_matrix(seed=1)
    with pytest.raises(api.SdError):
        S.Surrogate(B, th, max_batch=100)
    sur = S.Surrogate(B, th, max_batch=128)
    X = cuda(np.zeros((200, 3), np.float32))
    t = cuda(np.zeros(200, np.float32))
    with pytest.raises(api.SdError):
        sur.loss_grad(X, t, n=100)           # not a multiple of 64
    with pytest.raises(api.SdError):
        sur.loss_grad(X, t, n=192)           # above max_batch
    with pytest.raises(api.SdError):
        sur.certify(X, t, safety=0.5)
    sc = scenes.bumpy_icosphere(level=2, seed=3)
    scene = api.upload_scene(sc)
    with pytest.raises(api.SdError):
        S.sd_eval_surrogate(scene, sur, X, 50.0, band=-1.0)
    empty = api.sd_build_bvh(cuda(np.zeros((4, 3), np.float32)))
    with pytest.raises(api.SdError):
        S.sd_eval_surrogate(empty, sur, X, 50.0)


@pytest.mark.parametrize("nq,flags", [(3000, 0), (20000, 0), (20000, api.SD_NO_QUERY_SORT)])
def test_routing_to_exact_evaluation(nq, flags):
    """Queries with |surrogate| < band + eps go to Barnes-Hut; the others keep
    the surrogate's value and gradient."""
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    sc = scenes.bumpy_icosphere(level=3, seed=16)
    scene = api.upload_scene(sc)
    sur, th, B = _surrogate(seed=17, scale=2.0)
    X = np.random.default_rng(18).uniform(-1.5, 1.5, (nq, 3)).astype(np.float32)
    Xd = cuda(X)
    y, gy = sur.forward(Xd)
    y, gy = y.cpu().numpy(), gy.cpu().numpy()
    band, eps = 0.08, 0.02
    sur.load(th, eps_cert=eps)
    d, g, routed, nfb = S.sd_eval_surrogate(scene, sur, Xd, 50.0, 0.5, band=band, flags=flags)
    nfb = int(nfb)
    d, g, routed = d.cpu().numpy(), g.cpu().numpy(), routed.cpu().numpy().astype(bool)
    want = np.abs(y) < np.float32(band) + np.float32(eps)
    assert np.array_equal(routed, want)
    assert nfb == int(want.sum()) and 0 < nfb < nq
    assert np.array_equal(d[~routed], y[~routed]) and np.array_equal(g[~routed], gy[~routed])
    de, ge = api.sd_eval_grad(scene, Xd, 50.0, 0.5, flags=flags)
    de, ge = de.cpu().numpy(), ge.cpu().numpy()
    floor = 1e-3 * float(np.linalg.norm(sc.V.max(0) - sc.V.min(0)))
    err = np.abs(d[routed] - de[routed]) / np.maximum(np.abs(de[routed]), floor)
    assert err.max() <= 2e-6, err.max()
    gerr = np.linalg.norm(g[routed] - ge[routed], axis=1) / np.maximum(np.linalg.norm(ge[routed], axis=1), 1e-2)
    assert gerr.max() <= 1e-4, gerr.max()
    # nothing routed / everything routed
    sur.load(th, eps_cert=0.0)
    d0, _, r0, n0 = S.sd_eval_surrogate(scene, sur, Xd, 50.0, 0.5, band=0.0)
    n0 = int(n0)
    assert n0 == 0 and not r0.any() and np.array_equal(d0.cpu().numpy(), y)
    sur.load(th, eps_cert=float("inf"))
    d1, _, r1, n1 = S.sd_eval_surrogate(scene, sur, Xd, 50.0, 0.5, band=0.05)
    n1 = int(n1)
    assert n1 == nq and bool(r1.all())


def _cells(X, lo, ginv, G):
    """Certificate cell of each point (same FP32 operations as the library), -1 outside."""
    t = (X.astype(np.float32) - lo.astype(np.float32)) * ginv
    inside = np.all((t >= 0) & (t <= np.float32(G)), axis=1)
    c = np.minimum(np.floor(np.where(inside[:, None], t, 0)).astype(np.int64), G - 1)
    return np.where(inside, (c[:, 0] * G + c[:, 1]) * G + c[:, 2], -1)


def test_local_certificate_and_routing():
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    sc = scenes.bumpy_icosphere(level=3, seed=16)
    scene = api.upload_scene(sc)
    sur, th, B = _surrogate(seed=19, scale=2.0)
    rng = np.random.default_rng(20)
    Xv = rng.uniform(-1.5, 1.5, (20000, 3)).astype(np.float32)
    # held-out labels that disagree with the network by a small amount for
    # x < 0 and a large one for x > 0, so that the local margins differ
    y0 = sur.forward(cuda(Xv), grad=False).cpu().numpy()
    amp = np.where(Xv[:, 0] < 0, 1e-3, 0.3).astype(np.float32)
    lab = (y0 + amp * rng.standard_normal(len(Xv)).astype(np.float32)).astype(np.float32)
    G, safety = 8, 1.5
    lo = np.full(3, -1.5, np.float32)
    hi = np.full(3, 1.5, np.float32)
    eps = sur.certify_cells(cuda(Xv), cuda(lab), lo, hi, grid=G, safety=safety)
    y = sur.forward(cuda(Xv), grad=False).cpu().numpy()
    err = np.abs(y - lab)
    assert eps == np.float32(safety) * err.max()
    ginv = (np.float32(G) / (hi - lo)).astype(np.float32)
    cell = _cells(Xv, lo, ginv, G)
    cmax = np.full(G ** 3, -1.0, np.float32)
    np.maximum.at(cmax, cell[cell >= 0], err[cell >= 0])
    cm = cmax.reshape(G, G, G)
    pad = np.pad(cm, 1, constant_values=-1.0)
    nb = np.max([pad[1 + a:1 + a + G, 1 + b:1 + b + G, 1 + c:1 + c + G]
                 for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], axis=0).reshape(-1)
    ceps = np.where(nb < 0, np.float32(eps), np.float32(safety) * nb).astype(np.float32)
    # routing with the local margins (queries partly outside the grid box)
    Xq = rng.uniform(-1.7, 1.7, (30000, 3)).astype(np.float32)
    yq = sur.forward(cuda(Xq), grad=False).cpu().numpy()
    band = np.float32(0.05)
    d, g, routed, nfb = S.sd_eval_surrogate(scene, sur, cuda(Xq), 50.0, 0.5, band=float(band))
    nfb = int(nfb)
    cq = _cells(Xq, lo, ginv, G)
    thr = np.where(cq >= 0, band + ceps[np.maximum(cq, 0)], band + np.float32(eps)).astype(np.float32)
    want = np.abs(yq) < thr
    assert np.array_equal(routed.cpu().numpy().astype(bool), want)
    assert nfb == int(want.sum()) and 0 < nfb < len(Xq)
    # a margin cap: cells above it route every query (the cap splits the
    # cells of the accurate half)
    cap = np.float32(np.median(ceps[ceps < 0.1]))
    sur.certify_cells(cuda(Xv), cuda(lab), lo, hi, grid=G, safety=safety, max_margin=float(cap))
    _, _, rc, nc = S.sd_eval_surrogate(scene, sur, cuda(Xq), 50.0, 0.5, band=float(band))
    nc = int(nc)
    ceps_c = np.where(ceps > cap, np.float32(np.inf), ceps)
    thr_c = np.where(cq >= 0, band + ceps_c[np.maximum(cq, 0)], band + np.float32(eps)).astype(np.float32)
    want_c = np.abs(yq) < thr_c
    assert np.array_equal(rc.cpu().numpy().astype(bool), want_c)
    assert nc == int(want_c.sum()) and nc > nfb
    # a global certificate drops the grid
    eps2 = sur.certify(cuda(Xv), cuda(lab), safety=safety)
    _, _, r2, n2 = S.sd_eval_surrogate(scene, sur, cuda(Xq), 50.0, 0.5, band=float(band))
    n2 = int(n2)
    assert np.array_equal(r2.cpu().numpy().astype(bool), np.abs(yq) < band + np.float32(eps2))
