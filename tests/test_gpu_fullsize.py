"""GPU parity at the full sizes of the benchmark workloads (icosphere, street
rigid step, terrain precision sweep, surrogate inference), each in the launch
the benchmark times.  Icosphere: the level-7 bumpy icosphere (327,680 triangles)
with 1,000,000 queries (half uniform in the box, half within 0.02 of the
surface), Morton ordering of the queries, then the ordered value + gradient
kernel over all of them.  Sampled outputs (the default, conservative ones)
are compared one by one with the FP64 oracle's Barnes-Hut (Alg. 1/Alg. 2,
App. D) on the exported hierarchy, with the opening decision taken in FP32 on
both sides; properties that hold at any size are checked on every output,
among them d <= d_min against the oracle's exact nearest distance."""
import numpy as np
import pytest

from tests.gpu_common import O, api, compare, cuda, floor_of, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu

_STATE = {}


def _workload():
    if not _STATE:
        sc = scenes.bumpy_icosphere(level=7, seed=2)
        Q = scenes.icosphere_queries(sc, 1_000_000, seed_box=3, seed_surf=4)
        scene = api.upload_scene(sc)
        tree = O.OracleTree(*api.sd_export_bvh(scene, 2))
        _STATE.update(sc=sc, Q=Q, scene=scene, osc=O.OracleScene(sc.V, T=sc.T), trees=[None, None, tree])
    return _STATE


@pytest.mark.parametrize("alpha", [50.0, 500.0])
def test_full_size_icosphere_in_benchmark_launch(alpha):
    require_gpu()
    w = _workload()
    sc, Q, scene = w["sc"], w["Q"], w["scene"]
    beta = 0.5
    Qd = cuda(Q)
    perm = api.sd_query_order(scene, Qd)
    dc, gc = api.sd_eval_grad_ordered(scene, Qd, perm, alpha, beta)
    dp, _ = api.sd_eval_grad_ordered(scene, Qd, perm, alpha, beta, flags=api.SD_NO_CONSERVATIVE_ROUNDING)
    torch.cuda.synchronize()
    # the permutation is one of 0..n-1
    p = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(p), np.arange(len(Q)))
    dp, gc, dc = dp.cpu().numpy(), gc.cpu().numpy(), dc.cpu().numpy()
    # every output: finite; the clamp only ever lowers the unclamped result
    assert np.all(np.isfinite(dp)) and np.all(np.isfinite(gc)) and np.all(np.isfinite(dc))
    assert np.all(dc <= dp)
    # every output at or below the exact minimum distance (App. A)
    dm_all = O.dmin_tree(w["osc"], w["trees"], Q.astype(np.float64))
    assert np.all(dc.astype(np.float64) <= dm_all)
    # 2,000 sampled outputs against the oracle
    idx = np.sort(np.random.default_rng(int(alpha)).choice(len(Q), 2000, replace=False))
    Qs = Q[idx].astype(np.float64)
    dr, gr, _ = O.barnes_hut(w["osc"], w["trees"], Qs, alpha, beta, cut_f32=True)
    compare(dc[idx], gc[idx], dr, gr, floor_of(sc), what=f"full size alpha={alpha:g}", dmin=dm_all[idx])


def test_full_size_hierarchy_is_tight():
    """The level-7 hierarchy (655,359 nodes over 1,280 workgroups of leaves):
    every internal box is exactly the union of its children's boxes and
    every leaf box exactly its triangle's box, so the bottom-up refit saw
    every child box it combined."""
    require_gpu()
    w = _workload()
    box, left, right, prim = api.sd_export_bvh(w["scene"], 2)
    internal = np.where(left >= 0)[0]
    l, r = left[internal], right[internal]
    assert np.array_equal(box[internal, :3], np.minimum(box[l, :3], box[r, :3]))
    assert np.array_equal(box[internal, 3:], np.maximum(box[l, 3:], box[r, 3:]))
    lv = np.where(left < 0)[0]
    tri = w["sc"].V[w["sc"].T[prim[lv]]]
    assert np.array_equal(box[lv, :3], tri.min(1)) and np.array_equal(box[lv, 3:], tri.max(1))


def test_full_size_street_rigid_step_in_benchmark_launch():
    """The rigid-body street workload at full size (2M points, 20,000 wire
    segments, the 50,000-triangle torus at rest; 256 placements of the
    25,000-vertex body = 6.4M queries) in the benchmark's launch: rigid
    transform, query ordering, ordered value + gradient, query-mesh
    log-sum-exp per placement (Eq. 6-8), adjoint of sum_k D_k.  2,000 sampled
    queries against the oracle's Barnes-Hut on the exported hierarchies; three
    whole placements through the oracle composite (D_k, and the adjoint in
    t_k and R_k from the oracle's weights and gradients); the reduction
    identity sum_j xbar_j = sum_k R_k^T tbar_k on every output."""
    require_gpu()
    from oracle import qmesh as QM
    from tests.gpu_common import oracle_scene, oracle_trees
    alpha, beta, alpha_q = 50.0, 0.5, 50.0
    sc, body = scenes.street_scene(1.0)
    scene = api.upload_scene(sc)
    R, t = scenes.rigid_transforms(256, seed=5)
    K, m = R.shape[0], body.shape[0]
    X, Rd, td = cuda(body), cuda(R), cuda(t)
    Q = api.sd_rigid_transform(X, Rd, td)
    perm = api.sd_query_order(scene, Q)
    d, g = api.sd_eval_grad_ordered(scene, Q, perm, alpha, beta)
    D, w, _ = api.sd_query_mesh_lse(d.reshape(K, m), None, alpha_q, want_vgrad=False)
    Rb, tb, Xb = api.sd_rigid_adjoint(X, Rd, w, g)
    torch.cuda.synchronize()
    Qn, dn, gn = Q.cpu().numpy().astype(np.float64), d.cpu().numpy(), g.cpu().numpy()
    D, Rb, tb, Xb = (a.cpu().numpy().astype(np.float64) for a in (D, Rb, tb, Xb))
    assert np.all(np.isfinite(dn)) and np.all(np.isfinite(gn)) and np.all(np.isfinite(D))
    osc, trees, floor = oracle_scene(sc), oracle_trees(scene), floor_of(sc)
    idx = np.sort(np.random.default_rng(8).choice(K * m, 2000, replace=False))
    dr, gr, _ = O.barnes_hut(osc, trees, Qn[idx], alpha, beta, cut_f32=True)
    dm = O.dmin(osc, Qn[idx])
    compare(dn[idx], gn[idx], dr, gr, floor, what="street full size", dmin=dm)
    assert np.all(dn[idx].astype(np.float64) <= dm)
    ks = np.array([0, 101, 255])
    rows = (ks[:, None] * m + np.arange(m)).reshape(-1)
    dk, gk, _ = O.barnes_hut(osc, trees, Qn[rows], alpha, beta, cut_f32=True)
    Dr, wr, _ = QM.query_mesh_lse(dk.reshape(3, m), gk.reshape(3, m, 3), alpha_q)
    assert np.all(np.abs(D[ks] - Dr) <= 1e-5 * np.maximum(np.abs(Dr), floor))
    Rr, tr, _ = O.rigid_adjoint(body, R[ks], wr.reshape(-1), gk)
    np.testing.assert_allclose(tb[ks], tr, atol=2e-4)          # |tbar_k| <= sum_j w_kj = 1
    np.testing.assert_allclose(Rb[ks], Rr, atol=2e-4 * max(1.0, np.abs(body).max()))
    lhs = Xb.sum(0)
    rhs = np.einsum("kab,ka->b", R.astype(np.float64), tb)
    np.testing.assert_allclose(lhs, rhs, atol=1e-3 * max(1.0, np.abs(rhs).max()))


def test_full_size_terrain_alpha_and_precision_modes():
    """The scale / precision workload at full size (20M terrain points, 1M
    torus triangles, 199,200 hemisphere edges; 32M queries in the box enlarged
    by 10 %), in the benchmark's launch, for alpha 10, 100, 1000 and 5000: 500
    sampled queries against the oracle's Barnes-Hut on the exported
    hierarchies, every output finite, the result at or below the minimum
    distance on the sample."""
    require_gpu()
    from tests.gpu_common import oracle_scene, oracle_trees
    beta = 0.5
    sc = scenes.terrain_scene(1.0)
    scene = api.upload_scene(sc)
    nq = 32_000_000
    Q = scenes.terrain_queries(sc, nq, seed=10)
    Qd = cuda(Q)
    perm = api.sd_query_order(scene, Qd)
    osc, trees, floor = oracle_scene(sc), oracle_trees(scene), floor_of(sc)
    for c in range(3):   # tight hierarchies at this size (40M nodes for the points)
        box, left, right, _ = api.sd_export_bvh(scene, c)
        internal = np.where(left >= 0)[0]
        l, r = left[internal], right[internal]
        assert np.array_equal(box[internal, :3], np.minimum(box[l, :3], box[r, :3]))
        assert np.array_equal(box[internal, 3:], np.maximum(box[l, 3:], box[r, 3:]))
        del box, left, right, internal, l, r
    idx = np.sort(np.random.default_rng(9).choice(nq, 500, replace=False))
    Qs = Q[idx].astype(np.float64)
    dm = O.dmin(osc, Qs)
    d = torch.empty(nq, device="cuda")
    g = torch.empty((nq, 3), device="cuda")
    for alpha in (10.0, 100.0, 1000.0, 5000.0):
        dr, gr, _ = O.barnes_hut(osc, trees, Qs, alpha, beta, cut_f32=True)
        api.sd_eval_grad_ordered(scene, Qd, perm, alpha, beta, out=d, grad_out=g)
        dn, gn = d.cpu().numpy(), g.cpu().numpy()
        assert np.all(np.isfinite(dn)) and np.all(np.isfinite(gn))
        compare(dn[idx], gn[idx], dr, gr, floor, what=f"terrain full size alpha={alpha:g}", dmin=dm)
        assert np.all(dn[idx].astype(np.float64) <= dm)


def test_full_size_surrogate_inference_and_routing():
    """The surrogate workload's inference at full size (16M uniform queries
    against the level-7 icosphere) in the benchmark's launch (the fused
    network kernel with routing, exact Barnes-Hut for the routed queries).
    The network's weights are the seeded initialisation scaled by 2 (the
    kernel's arithmetic does not depend on training): 1,000 sampled value +
    input-gradient outputs against the FP64 network oracle within the BF16
    rounding envelope; on every query the routing flag is |y| < band + eps
    and unrouted outputs are the network's bit for bit; 1,000 sampled routed
    queries against the oracle's Barnes-Hut on the exported hierarchy."""
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    from tests import surrogate_ref as R
    from tests.test_gpu_surrogate import K_ENV, _surrogate
    w = _workload()
    sc, scene = w["sc"], w["scene"]
    n = 16_000_000
    X = scenes.uniform_queries(n, 8, -1.5, 1.5)
    Xd = cuda(X)
    sur, th, B = _surrogate(seed=17, scale=2.0)
    y, gy = sur.forward(Xd)
    band, eps = 0.05, 0.02
    sur.load(th, eps_cert=eps)
    d, g, routed, nfb = S.sd_eval_surrogate(scene, sur, Xd, 50.0, 0.5, band=band)
    nfb = int(nfb)
    torch.cuda.synchronize()
    y, gy, d, g = y.cpu().numpy(), gy.cpu().numpy(), d.cpu().numpy(), g.cpu().numpy()
    routed = routed.cpu().numpy().astype(bool)
    assert np.all(np.isfinite(y)) and np.all(np.isfinite(gy))
    # network parity on a sample
    idx = np.sort(np.random.default_rng(19).choice(n, 1000, replace=False))
    Xs = X[idx].astype(np.float64)
    ref, dev = R.envelope(R.infer, R.effective_theta(th), B.astype(np.float64), Xs)
    yr, gr = ref[:1000], ref[1000:].reshape(1000, 3)
    yd, gd = dev[:1000], dev[1000:].reshape(1000, 3)
    fy = 2.0 ** -16 * (np.abs(yr) + np.abs(yr).mean())
    fg = 2.0 ** -16 * (np.abs(gr) + np.abs(gr).mean())
    assert np.all(np.abs(y[idx] - yr) <= K_ENV * yd + fy)
    assert np.all(np.abs(gy[idx] - gr) <= K_ENV * gd + fg)
    # routing on every query
    want = np.abs(y) < np.float32(band) + np.float32(eps)
    assert np.array_equal(routed, want) and nfb == int(want.sum()) and 0 < nfb < n
    assert np.array_equal(d[~routed], y[~routed]) and np.array_equal(g[~routed], gy[~routed])
    # routed queries: the exact path
    r = np.flatnonzero(routed)
    rs = np.sort(np.random.default_rng(20).choice(r, min(1000, len(r)), replace=False))
    Qs = X[rs].astype(np.float64)
    dr, grr, _ = O.barnes_hut(w["osc"], w["trees"], Qs, 50.0, 0.5, cut_f32=True)
    dm = O.dmin(w["osc"], Qs)
    assert np.all(d[rs].astype(np.float64) <= dm)      # conservative (App. A)
    compare(d[rs], g[rs], dr, grr, floor_of(sc), what="routed full size", dmin=dm)
