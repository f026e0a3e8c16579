"""GPU parity: the smooth distance to a query mesh (Sec. 3.6, Eq. 6-8) through
the C ABI against the FP64 oracle (oracle/qmesh.py) on the same inputs, and
the rigid-body composite D_k(R_k, t_k) with its hand-written adjoint against
central differences of the oracle composite."""
import numpy as np
import pytest

from oracle import qmesh as QM
from tests.gpu_common import O, api, cuda, oracle_scene, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu


def _mixed_prims(rng, nV, n):
    kinds = rng.integers(1, 4, n)
    prim = -np.ones((n, 3), np.int32)
    for j, c in enumerate(kinds):
        prim[j, :c] = rng.choice(nV, c, replace=False)
    return prim


def _check(D, w, vg, Dr, wr, vr, what):
    D = D.cpu().numpy().astype(np.float64)
    fin = np.isfinite(Dr)
    assert np.array_equal(np.isposinf(D), np.isposinf(Dr)), what
    assert np.array_equal(np.isnan(D), np.isnan(Dr)), what
    np.testing.assert_allclose(D[fin], Dr[fin], rtol=2e-7, atol=2e-7, err_msg=what)
    if w is not None:
        np.testing.assert_allclose(w.cpu().numpy()[fin], wr[fin], rtol=2e-5, atol=1e-9, err_msg=what)
    if vg is not None:
        scale = np.abs(vr[fin]).max() if fin.any() else 1.0
        np.testing.assert_allclose(vg.cpu().numpy()[fin], vr[fin], rtol=0, atol=2e-6 * max(scale, 1e-3),
                                   err_msg=what)


@pytest.mark.parametrize("alpha_q", [5.0, 200.0])
def test_point_query_mesh_matches_oracle(alpha_q):
    """Several instances, a ragged length spanning three 4096-wide chunks."""
    require_gpu()
    rng = np.random.default_rng(1)
    K, m = 5, 10001
    d = rng.uniform(-0.1, 2.0, (K, m)).astype(np.float32)
    g = rng.normal(size=(K, m, 3)).astype(np.float32)
    D, w, vg = api.sd_query_mesh_lse(cuda(d), cuda(g), alpha_q)
    torch.cuda.synchronize()
    Dr, wr, vr = QM.query_mesh_lse(d, g, alpha_q)
    _check(D, w, vg, Dr, wr, vr, f"points alpha_q={alpha_q}")


def test_mixed_query_mesh_matches_oracle():
    """Points, edges and triangles as query primitives: the split shares of
    Eq. 7 and the one-ring sums of Eq. 8."""
    require_gpu()
    rng = np.random.default_rng(2)
    K, m, nV = 3, 5000, 1800
    prim = _mixed_prims(rng, nV, m)
    d = rng.uniform(0.0, 1.0, (K, m)).astype(np.float32)
    g = rng.normal(size=(K, m, 3)).astype(np.float32)
    D, w, vg = api.sd_query_mesh_lse(cuda(d), cuda(g), 30.0, prim=cuda(prim), nV=nV)
    torch.cuda.synchronize()
    Dr, wr, vr = QM.query_mesh_lse(d, g, 30.0, prim.astype(np.int64), nV)
    _check(D, w, vg, Dr, wr, vr, "mixed")
    # outputs are optional
    D2, w2, vg2 = api.sd_query_mesh_lse(cuda(d), cuda(g), 30.0, prim=cuda(prim), nV=nV, want_w=False,
                                        want_vgrad=False)
    assert w2 is None and vg2 is None
    assert torch.equal(D2, D)


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_triangle_query_mesh_end_to_end(beta):
    """A triangle query mesh (a torus beside a bumpy sphere): the distances
    and gradients of its triangles from the query-primitive traversal
    (Sec. 3.4), combined by Eq. 6-8, against the oracle's query-primitive
    Barnes-Hut (FP32 opening decisions) combined by the oracle's Eq. 6-8.
    Tolerances follow from the per-primitive ones (the 1e-5 gate for value
    and gradient): D is a log-sum-exp of the d_j, so its relative error is at
    most theirs; w_j = softmin weights move by about alpha_q |delta d_j|; the
    vertex gradients mix the gradient errors (relative to the largest)."""
    require_gpu()
    from tests.gpu_common import oracle_trees
    data = scenes.bumpy_icosphere(level=3, seed=5)
    scene = api.upload_scene(data)
    tv, tf = scenes.torus_grid(24, 12, 0.5, 0.15)
    tv = (tv + np.array([2.3, 0.0, 0.2])).astype(np.float32)     # clear of the sphere (radius <= 1.4)
    G = tv[tf].astype(np.float32)
    alpha, alpha_q = 40.0, 30.0
    d, g = api.sd_eval_grad_prims(scene, cuda(G), alpha, beta, flags=api.SD_NO_CONSERVATIVE_ROUNDING)
    D, w, vg = api.sd_query_mesh_lse(d.reshape(1, -1), g.reshape(1, -1, 3), alpha_q,
                                     prim=cuda(tf.astype(np.int32)), nV=len(tv))
    torch.cuda.synchronize()
    osc, trees = oracle_scene(data), oracle_trees(scene)
    dr, gr, _ = O.barnes_hut_prims(osc, trees, G.astype(np.float64), alpha, beta, cut_f32=True)
    _, _, dm = O.brute_prims(osc, G.astype(np.float64), alpha)
    assert dm.min() > 0.1
    Dr, wr, vr = QM.query_mesh_lse(dr[None], gr[None], alpha_q, tf.astype(np.int64), len(tv))
    D, w, vg = D.cpu().numpy().astype(np.float64), w.cpu().numpy(), vg.cpu().numpy()
    ev, eg = abs(D[0] - Dr[0]) / abs(Dr[0]), np.abs(vg[0] - vr[0]).max() / np.abs(vr).max()
    print(f"query mesh beta={beta}: D relative error {ev:.2e}, vertex gradient error {eg:.2e} of the largest")
    assert ev <= 1e-5
    dd = np.abs(d.cpu().numpy() - dr).max()
    np.testing.assert_allclose(w[0], wr[0], rtol=0, atol=3 * alpha_q * dd * wr.max() + 1e-7)
    assert eg <= 1e-5


def test_edge_cases():
    require_gpu()
    g = np.zeros((4, 3, 3), np.float32)
    d = np.array([[0.5, 0.25, 1.0], [np.inf, np.inf, np.inf], [0.5, np.inf, 0.75], [0.5, np.nan, 0.1]],
                 np.float32)
    D, w, vg = api.sd_query_mesh_lse(cuda(d), cuda(g), 10.0)
    Dr, wr, vr = QM.query_mesh_lse(d, g, 10.0)
    _check(D, w, vg, Dr, wr, vr, "edge rows")
    assert np.all(w.cpu().numpy()[1] == 0)
    # no primitives: every instance is the empty sum
    D0, w0, vg0 = api.sd_query_mesh_lse(torch.empty((3, 0), device="cuda"), torch.empty((3, 0, 3), device="cuda"),
                                        10.0)
    assert torch.all(torch.isposinf(D0))
    # a single primitive is its own distance
    D1, w1, vg1 = api.sd_query_mesh_lse(cuda(np.array([[0.3]], np.float32)),
                                        cuda(np.array([[[1.0, 0.0, 0.0]]], np.float32)), 7.0)
    assert D1.item() == pytest.approx(0.3, abs=1e-7) and w1.item() == 1.0
    bad = [dict(alpha_q=0.0), dict(alpha_q=float("inf"))]
    for kw in bad:
        with pytest.raises(api.SdError):
            api.sd_query_mesh_lse(cuda(d), cuda(g), **kw)
    prim = np.array([[0, 1, -1], [2, -1, -1], [1, 5, -1]], np.int32)   # id 5 >= nV
    with pytest.raises(api.SdError):
        api.sd_query_mesh_lse(cuda(d), cuda(g), 10.0, prim=cuda(prim), nV=4)
    prim = np.array([[0, 1, -1], [-1, -1, -1], [1, 2, 3]], np.int32)  # an empty primitive
    with pytest.raises(api.SdError):
        api.sd_query_mesh_lse(cuda(d), cuda(g), 10.0, prim=cuda(prim), nV=4)


def test_rigid_query_mesh_distance_and_adjoint():
    """D_k for K rigid placements of a point body (exact evaluation, beta = 0)
    against the oracle composite, and dD/dt, dD/dR from the adjoint against
    central differences of the oracle composite."""
    require_gpu()
    sc = scenes.bumpy_icosphere(level=2, seed=3)
    scene = api.upload_scene(sc)
    osc = oracle_scene(sc)
    rng = np.random.default_rng(7)
    X = (rng.normal(size=(150, 3)) * 0.15).astype(np.float32)
    R, t = scenes.rigid_transforms(4, seed=8)
    t = (t * 0.0 + rng.uniform(-1.6, 1.6, t.shape)).astype(np.float32)
    alpha, alpha_q = 30.0, 12.0

    def oracle_D(Rh, th):
        Q = O.rigid_apply(X, Rh, th)
        d, g, _ = O.brute(osc, Q, alpha)
        return QM.query_mesh_lse(d.reshape(len(Rh), -1), g.reshape(len(Rh), -1, 3), alpha_q)[0]

    Xt, Rt, tt = cuda(X), cuda(R).requires_grad_(True), cuda(t).requires_grad_(True)
    D = api.rigid_query_mesh_distance(Xt, Rt, tt, scene, alpha, alpha_q, beta=0.0)
    D.sum().backward()
    Dr = oracle_D(R.astype(np.float64), t.astype(np.float64))
    np.testing.assert_allclose(D.detach().cpu().numpy(), Dr, rtol=1e-5, atol=1e-5)
    h = 1e-4
    fd_t = np.zeros(t.shape)
    for k in range(len(t)):
        for c in range(3):
            tp, tm = t.astype(np.float64).copy(), t.astype(np.float64).copy()
            tp[k, c] += h
            tm[k, c] -= h
            fd_t[k, c] = (oracle_D(R.astype(np.float64), tp)[k] - oracle_D(R.astype(np.float64), tm)[k]) / (2 * h)
    np.testing.assert_allclose(tt.grad.cpu().numpy(), fd_t, atol=2e-4 * max(1.0, np.abs(fd_t).max()))
    fd_R = np.zeros(R.shape)
    for k in range(len(R)):
        for a in range(3):
            for b in range(3):
                Rp, Rm = R.astype(np.float64).copy(), R.astype(np.float64).copy()
                Rp[k, a, b] += h
                Rm[k, a, b] -= h
                fd_R[k, a, b] = (oracle_D(Rp, t.astype(np.float64))[k] - oracle_D(Rm, t.astype(np.float64))[k]) / (2 * h)
    np.testing.assert_allclose(Rt.grad.cpu().numpy(), fd_R, atol=2e-4 * max(1.0, np.abs(fd_R).max()))
