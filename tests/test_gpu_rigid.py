"""GPU: rigidly moved queries and the hand-written adjoint in (R, t, X).

* sd_rigid_transform against the oracle's x' = R x + t;
* sd_rigid_adjoint against the oracle's reductions on the same (gbar, grad);
* sd_rigid_qmesh_adjoint (upstream w * Dbar formed on the GPU) against
  sd_rigid_adjoint on the same product;
* the autograd function (forward sd_eval_grad, backward sd_rigid_adjoint)
  against central finite differences of the FP64 oracle (h = 1e-4, beta = 0),
  and its X gradient against the oracle gradient pulled back through R.
"""
import numpy as np
import pytest

from tests.gpu_common import O, api, cuda, oracle_scene, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu


def _rotations(K, rng):
    q = rng.standard_normal((K, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                  2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                  2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1)
    return R.reshape(K, 3, 3).astype(np.float32)


def _body(m, rng):
    return (0.25 * rng.standard_normal((m, 3))).astype(np.float32)


def test_rigid_transform_matches_oracle():
    require_gpu()
    rng = np.random.default_rng(50)
    X, R = _body(3001, rng), _rotations(17, rng)
    t = rng.uniform(-1, 1, (17, 3)).astype(np.float32)
    Q = api.sd_rigid_transform(cuda(X), cuda(R), cuda(t)).cpu().numpy()
    ref = O.rigid_apply(X, R, t)
    # three FMAs on FP32 inputs: a few ulps of the magnitudes involved
    assert np.all(np.abs(Q - ref) <= 4e-7 * (1 + np.abs(ref)))


def test_rigid_adjoint_matches_oracle_reductions():
    require_gpu()
    rng = np.random.default_rng(51)
    K, m = 13, 2777
    X, R = _body(m, rng), _rotations(K, rng)
    gbar = rng.standard_normal(K * m).astype(np.float32)
    grad = rng.standard_normal((K * m, 3)).astype(np.float32)
    Rb, tb, Xb = api.sd_rigid_adjoint(cuda(X), cuda(R), cuda(gbar), cuda(grad))
    Rr, tr, Xr = O.rigid_adjoint(X, R, gbar, grad)
    scale_R = np.abs(gbar[:, None] * grad).reshape(K, m, 3).sum(1)   # |u| sums per transform
    np.testing.assert_allclose(tb.cpu().numpy(), tr, atol=1e-5 * scale_R.max())
    np.testing.assert_allclose(Rb.cpu().numpy(), Rr, atol=1e-5 * scale_R.max())
    np.testing.assert_allclose(Xb.cpu().numpy(), Xr, atol=1e-5 * np.abs(Xr).max() + 1e-6)
    # deterministic: the reductions use a fixed order
    Rb2, tb2, Xb2 = api.sd_rigid_adjoint(cuda(X), cuda(R), cuda(gbar), cuda(grad))
    assert torch.equal(Rb, Rb2) and torch.equal(tb, tb2) and torch.equal(Xb, Xb2)


def test_query_mesh_adjoint_forms_the_weighted_upstream_on_the_gpu():
    """sd_rigid_qmesh_adjoint (gbar_kj = w_kj Dbar_k formed in the kernels)
    equals sd_rigid_adjoint on the FP32 product w * Dbar bit for bit (the same
    product, then the same fixed-order reductions), and the oracle's
    reductions on that gbar."""
    require_gpu()
    rng = np.random.default_rng(52)
    K, m = 7, 3001
    X, R = _body(m, rng), _rotations(K, rng)
    w = rng.uniform(0.0, 2.0 / m, (K, m)).astype(np.float32)
    Dbar = rng.standard_normal(K).astype(np.float32)
    grad = rng.standard_normal((K * m, 3)).astype(np.float32)
    Rq, tq, Xq = api.sd_rigid_qmesh_adjoint(cuda(X), cuda(R), cuda(w), cuda(Dbar), cuda(grad))
    gbar = (w * Dbar[:, None]).astype(np.float32)
    Rb, tb, Xb = api.sd_rigid_adjoint(cuda(X), cuda(R), cuda(gbar.reshape(-1)), cuda(grad))
    assert torch.equal(Rq, Rb) and torch.equal(tq, tb) and torch.equal(Xq, Xb)
    Rr, tr, Xr = O.rigid_adjoint(X, R, gbar.reshape(-1), grad)
    scale = np.abs(gbar.reshape(-1)[:, None] * grad).reshape(K, m, 3).sum(1).max()
    np.testing.assert_allclose(tq.cpu().numpy(), tr, atol=1e-5 * scale)
    np.testing.assert_allclose(Rq.cpu().numpy(), Rr, atol=1e-5 * scale)
    np.testing.assert_allclose(Xq.cpu().numpy(), Xr, atol=1e-5 * np.abs(Xr).max() + 1e-9)
    with pytest.raises(ValueError):
        api.sd_rigid_qmesh_adjoint(cuda(X), cuda(R), cuda(w), cuda(Dbar[:-1]), cuda(grad))
    with pytest.raises(TypeError):
        api.sd_rigid_qmesh_adjoint(cuda(X), cuda(R), cuda(w), cuda(Dbar.astype(np.float64)), cuda(grad))


def test_rigid_adjoint_empty_and_invalid():
    require_gpu()
    X = cuda(np.zeros((0, 3), np.float32))
    R = cuda(np.eye(3, dtype=np.float32)[None])
    Rb, tb, Xb = api.sd_rigid_adjoint(X, R, cuda(np.zeros(0, np.float32)), cuda(np.zeros((0, 3), np.float32)))
    assert torch.all(Rb == 0) and torch.all(tb == 0)
    with pytest.raises(ValueError):
        api.sd_rigid_adjoint(cuda(np.zeros((4, 3), np.float32)), R, cuda(np.zeros(3, np.float32)),
                             cuda(np.zeros((4, 3), np.float32)))


def test_autograd_function_matches_oracle_finite_differences():
    require_gpu()
    rng = np.random.default_rng(52)
    sc = scenes.bumpy_icosphere(level=3, seed=8)
    scene = api.upload_scene(sc)
    osc = oracle_scene(sc)
    K, m = 3, 12
    X, R = _body(m, rng), _rotations(K, rng)
    t = rng.uniform(-0.4, 0.4, (K, 3)).astype(np.float32)
    t += (rng.standard_normal((K, 3)) * 0.6).astype(np.float32)
    gbar = rng.standard_normal((K, m))
    alpha = 20.0
    Xt = cuda(X).requires_grad_(True)
    Rt = cuda(R).requires_grad_(True)
    tt = cuda(t).requires_grad_(True)
    d = api.rigid_smooth_distance(Xt, Rt, tt, scene, alpha, beta=0.0)
    (d * cuda(gbar.astype(np.float32))).sum().backward()

    def loss(Xd, Rd, td):
        Q = (np.einsum("kab,jb->kja", Rd, Xd) + td[:, None, :]).reshape(-1, 3)
        dd, _, _ = O.brute(osc, Q, alpha)
        return float((gbar.reshape(-1) * dd).sum())

    Xd, Rd, td = X.astype(np.float64), R.astype(np.float64), t.astype(np.float64)
    h = 1e-4
    fd_t = np.zeros((K, 3)); fd_R = np.zeros((K, 3, 3)); fd_X = np.zeros((m, 3))
    for k in range(K):
        for a in range(3):
            e = np.zeros_like(td); e[k, a] = h
            fd_t[k, a] = (loss(Xd, Rd, td + e) - loss(Xd, Rd, td - e)) / (2 * h)
            for b in range(3):
                e = np.zeros_like(Rd); e[k, a, b] = h
                fd_R[k, a, b] = (loss(Xd, Rd + e, td) - loss(Xd, Rd - e, td)) / (2 * h)
    for j in range(m):
        for a in range(3):
            e = np.zeros_like(Xd); e[j, a] = h
            fd_X[j, a] = (loss(Xd + e, Rd, td) - loss(Xd - e, Rd, td)) / (2 * h)
    sc_t = max(1.0, np.abs(fd_t).max())
    np.testing.assert_allclose(tt.grad.cpu().numpy(), fd_t, atol=2e-4 * sc_t)
    np.testing.assert_allclose(Rt.grad.cpu().numpy(), fd_R, atol=2e-4 * max(1.0, np.abs(fd_R).max()))
    np.testing.assert_allclose(Xt.grad.cpu().numpy(), fd_X, atol=2e-4 * max(1.0, np.abs(fd_X).max()))


def test_street_scene_rigid_step_matches_oracle():
    """The mixed street workload at small scale (points, wire segments and the
    resting torus in one scene): rigidly moved body vertices evaluated with
    Barnes-Hut against the oracle on the exported hierarchies, and the adjoint
    against the oracle's reductions of the oracle gradient."""
    require_gpu()
    from tests.gpu_common import compare, floor_of, oracle_trees
    sc, body = scenes.street_scene(scale=0.004, seed=3)
    assert all(c > 0 for c in sc.counts())
    scene = api.upload_scene(sc)
    R, t = scenes.rigid_transforms(6, seed=5)
    Q = api.sd_rigid_transform(cuda(body), cuda(R), cuda(t))
    d, g = api.sd_eval_grad(scene, Q, 50.0, 0.5)
    Qn = Q.cpu().numpy().astype(np.float64)
    osc = oracle_scene(sc)
    dr, gr, st = O.barnes_hut(osc, oracle_trees(scene), Qn, 50.0, 0.5, cut_f32=True)
    compare(d.cpu().numpy(), g.cpu().numpy(), dr, gr, floor_of(sc), what="street")
    K, m = R.shape[0], body.shape[0]
    gbar = np.random.default_rng(4).normal(size=K * m).astype(np.float32)
    Rb, tb, Xb = api.sd_rigid_adjoint(cuda(body), cuda(R), cuda(gbar), g)
    Rr, tr, Xr = O.rigid_adjoint(body, R, gbar, gr.astype(np.float32))
    scale = np.abs(gbar[:, None] * gr).reshape(K, m, 3).sum(1).max()
    np.testing.assert_allclose(tb.cpu().numpy(), tr, atol=2e-4 * scale)
    np.testing.assert_allclose(Rb.cpu().numpy(), Rr, atol=2e-4 * scale)
