"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs, element by element.

* beta = 0 and the all-pairs kernel against the oracle's brute force (Eq. 3,
  Eq. 4 over every primitive);
* beta > 0 against the oracle's Alg. 1 on the hierarchy the library built
  (exported), every query: the oracle takes the open/accept decision of
  Sec. 3.5 in FP32 like the library (a discrete choice that decides which
  terms are summed), and evaluates every term in FP64;
* the default (conservative) output is the one compared; conservativeness
  d <= d_min (App. A, Sec. 3.5) on every query, and the unclamped output
  (SD_NO_CONSERVATIVE_ROUNDING) equal to it wherever the clamp does not act;
* edge cases: empty scene, single primitive, ragged sizes, NaN and on-surface
  queries, degenerate triangles, invalid arguments.
"""
import numpy as np
import pytest

from tests.gpu_common import (O, api, compare, cuda, floor_of, oracle_scene, oracle_trees,
                              require_gpu, scenes, torch)

pytestmark = pytest.mark.gpu


NOCONS = api.SD_NO_CONSERVATIVE_ROUNDING


def _run(scene, Q, alpha, beta, alpha_u=0.0, flags=0):
    """The library's evaluation with the given flags (by default the
    conservative output, which is what the parity gate judges)."""
    d, g = api.sd_eval_grad(scene, cuda(Q), alpha, beta, alpha_u, flags)
    torch.cuda.synchronize()
    return d.cpu().numpy(), g.cpu().numpy()


def _check_conservative(scene, Q, alpha, beta, dmin, d, alpha_u=0.0, flags=0, brute=False):
    """Default evaluation d: d <= d_min on every query (App. A, Sec. 3.5).  The
    unclamped evaluation runs the same arithmetic without the final clamp, so
    it equals d bit for bit except where the clamp acted, where it is larger."""
    if brute:
        dp = api.sd_eval_brute(scene, cuda(Q), alpha, alpha_u, flags | NOCONS, grad=False)
    else:
        dp = api.sd_eval(scene, cuda(Q), alpha, beta, alpha_u, flags | NOCONS)
    torch.cuda.synchronize()
    dp = dp.cpu().numpy()
    d = np.asarray(d, np.float32)
    bad = d.astype(np.float64) > dmin
    assert not bad.any(), f"conservativeness violated on {bad.sum()} queries"
    same = (d == dp) | (np.isnan(d) & np.isnan(dp))
    assert np.all(same | (d < dp)), "the clamp raised a result"
    return int((~same).sum())


def _mixed_scene(seed=40):
    ico = scenes.bumpy_icosphere(level=3, seed=seed)
    pl = scenes.random_polyline(300, seed=seed + 1, step=0.05)
    rng = np.random.default_rng(seed + 2)
    pts = rng.uniform(-1.2, 1.2, (700, 3)).astype(np.float32)
    nV1, nV2 = len(ico.V), len(pl.V)
    V = np.concatenate([ico.V, pl.V * np.float32(0.3) + np.float32(0.5), pts])
    return scenes.Scene(V=V, P=np.arange(nV1 + nV2, nV1 + nV2 + 700, dtype=np.int32),
                        E=(pl.E + nV1).astype(np.int32), T=ico.T, name="mixed")


CASES = {
    "points": lambda: scenes.point_sphere(2000, 10000)[0],
    "polyline": lambda: scenes.random_polyline(3000, seed=7),
    "icosphere_l4": lambda: scenes.bumpy_icosphere(level=4, seed=2),
    "mixed": _mixed_scene,
}


def _queries(sc, n, seed):
    if sc.T is not None and sc.P is None and sc.E is None:
        return scenes.icosphere_queries(sc, n, seed_box=seed, seed_surf=seed + 1)
    lo, hi = scenes.scene_aabb(sc)
    c, h = 0.5 * (lo + hi), 0.75 * (hi - lo)
    return scenes.uniform_queries(n, seed, c - h, c + h)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    require_gpu()
    sc = CASES[request.param]()
    scene = api.upload_scene(sc)
    return request.param, sc, scene, oracle_scene(sc), oracle_trees(scene)


@pytest.mark.parametrize("alpha", [50.0, 500.0])
def test_brute_kernel_matches_oracle(case, alpha):
    name, sc, scene, osc, _ = case
    Q = _queries(sc, 3001, seed=11)        # ragged: 3001 = 11 * 256 + 185
    d, g = api.sd_eval_brute(scene, cuda(Q), alpha)
    torch.cuda.synchronize()
    d, g = d.cpu().numpy(), g.cpu().numpy()
    dr, gr, dm = O.brute(osc, Q.astype(np.float64), alpha)
    compare(d, g, dr, gr, floor_of(sc), what=f"{name} brute", dmin=dm)
    _check_conservative(scene, Q, alpha, 0.0, dm, d, brute=True)


def test_beta_zero_traversal_matches_oracle_brute(case):
    name, sc, scene, osc, _ = case
    Q = _queries(sc, 2000, seed=12)
    d, g = _run(scene, Q, 80.0, 0.0)
    dr, gr, dm = O.brute(osc, Q.astype(np.float64), 80.0)
    compare(d, g, dr, gr, floor_of(sc), what=f"{name} beta=0", dmin=dm)
    _check_conservative(scene, Q, 80.0, 0.0, dm, d)


@pytest.mark.parametrize("alpha,beta,alpha_u", [(50.0, 0.5, 0.0), (500.0, 0.5, 0.0),
                                                (100.0, 1.0, 0.0), (50.0, 0.5, 300.0)])
def test_barnes_hut_matches_oracle_on_exported_tree(case, alpha, beta, alpha_u):
    name, sc, scene, osc, trees = case
    Q = _queries(sc, 10000, seed=13)
    d, g = _run(scene, Q, alpha, beta, alpha_u)
    dr, gr, st = O.barnes_hut(osc, trees, Q.astype(np.float64), alpha, beta, alpha_u=alpha_u, cut_f32=True)
    dm = O.dmin(osc, Q.astype(np.float64))
    compare(d, g, dr, gr, floor_of(sc), what=f"{name} BH a={alpha} b={beta}", dmin=dm)
    _check_conservative(scene, Q, alpha, beta, dm, d, alpha_u=alpha_u)


@pytest.mark.parametrize("alpha", [50.0, 500.0])
def test_compensated_f32_sums_match_oracle(case, alpha):
    """The compiled variant with the running sums in compensated FP32
    (SD_LSE_COMPENSATED_F32) meets the same gate against the oracle, keeps
    d <= d_min, and is refused where it is not compiled (value only,
    counters, all-pairs kernel, query primitives, tracing)."""
    name, sc, scene, osc, trees = case
    Q = _queries(sc, 10000, seed=15)
    C32 = api.SD_LSE_COMPENSATED_F32
    d, g = _run(scene, Q, alpha, 0.5, flags=C32)
    dr, gr, st = O.barnes_hut(osc, trees, Q.astype(np.float64), alpha, 0.5, cut_f32=True)
    dm = O.dmin(osc, Q.astype(np.float64))
    compare(d, g, dr, gr, floor_of(sc), what=f"{name} compensated-f32 a={alpha}", dmin=dm)
    assert not np.any(d.astype(np.float64) > dm)
    Qd = cuda(Q)
    for call in (lambda: api.sd_eval(scene, Qd, alpha, 0.5, 0.0, C32),
                 lambda: api.sd_eval_counters(scene, Qd, alpha, 0.5, flags=C32),
                 lambda: api.sd_eval_brute(scene, Qd, alpha, 0.0, C32)):
        with pytest.raises(api.SdError) as e:
            call()
        assert "COMPENSATED" in str(e.value)


def test_paper_metric_and_rootlog_flags(case):
    name, sc, scene, osc, trees = case
    Q = _queries(sc, 3000, seed=14)
    alpha = 60.0
    d, g = _run(scene, Q, alpha, 0.5, flags=api.SD_GRAD_PAPER_METRIC | api.SD_ROOTLOG_F64)
    # the final logarithm is always FP64: the flag is accepted and changes nothing
    d0, g0 = _run(scene, Q, alpha, 0.5, flags=api.SD_GRAD_PAPER_METRIC)
    assert np.array_equal(d, d0) and np.array_equal(g, g0)
    dr, gr, st = O.barnes_hut(osc, trees, Q.astype(np.float64), alpha, 0.5, metric_r2=True, cut_f32=True)
    compare(d, g, dr, gr, floor_of(sc), what=f"{name} metric+rootlog",
            dmin=O.dmin(osc, Q.astype(np.float64)))


def test_counters_are_consistent(case):
    name, sc, scene, osc, trees = case
    Q = _queries(sc, 2000, seed=15)
    c = api.sd_eval_counters(scene, cuda(Q), 50.0, 0.5, flags=api.SD_NO_PRUNE).cpu().numpy()
    _, _, st = O.barnes_hut(osc, trees, Q.astype(np.float64), 50.0, 0.5, cut_f32=True)
    np.testing.assert_array_equal(c[:, 0], st[:, 1])   # nodes visited
    np.testing.assert_array_equal(c[:, 1], st[:, 2])   # far-field terms
    np.testing.assert_array_equal(c[:, 2], st[:, 3])   # exact leaves


def test_exported_hierarchy_is_valid(case):
    """Every primitive sits in exactly one leaf, children boxes nest in their
    parent, and the depth-first order has each left child right after its
    parent."""
    name, sc, scene, osc, trees = case
    counts = sc.counts()
    for c in range(3):
        t = api.sd_export_bvh(scene, c)
        if counts[c] == 0:
            assert t is None
            continue
        box, left, right, prim = t
        n = counts[c]
        assert len(left) == 2 * n - 1
        leaves = prim[left < 0]
        assert np.array_equal(np.sort(leaves), np.arange(n))
        internal = np.where(left >= 0)[0]
        assert np.all(left[internal] == internal + 1)
        for ch in (left[internal], right[internal]):
            assert np.all(box[ch, :3] >= box[internal, :3]) and np.all(box[ch, 3:] <= box[internal, 3:])
        # tight: an internal box is exactly the union of its children's boxes
        # and a leaf box exactly its primitive's box (FP32 min / max are exact)
        l, r = left[internal], right[internal]
        assert np.array_equal(box[internal, :3], np.minimum(box[l, :3], box[r, :3]))
        assert np.array_equal(box[internal, 3:], np.maximum(box[l, 3:], box[r, 3:]))
        lv = np.where(left < 0)[0]
        xyz = (osc.Pxyz, osc.Exyz, osc.Txyz)[c].astype(np.float32).reshape(n, c + 1, 3)[prim[lv]]
        assert np.array_equal(box[lv, :3], xyz.min(1)) and np.array_equal(box[lv, 3:], xyz.max(1))


def test_weight_data_matches_oracle_valences(case):
    name, sc, scene, osc, trees = case
    info = scene.info()
    if sc.E is not None:
        w = api.sd_export_weights(scene, 1)
        n0, n1, amax = O.edge_valences(sc.E.astype(np.int64), len(sc.V))
        np.testing.assert_array_equal(w[:, 0], (1.0 / n0).astype(np.float32))
        np.testing.assert_array_equal(w[:, 1], (1.0 / n1).astype(np.float32))
        assert info["A"][1] == amax == osc.A_E
    if sc.T is not None:
        w = api.sd_export_weights(scene, 2)
        v, e = O.triangle_valences(sc.T.astype(np.int64), len(sc.V))
        np.testing.assert_array_equal(w[:, 0], (1.0 / v).astype(np.float32))
        np.testing.assert_array_equal(w[:, 1], (1.0 / e).astype(np.float32))
        assert abs(info["A"][2] - osc.A_T) < 1e-9 * osc.A_T
        assert info["A_T_literal"] == osc.A_T_literal


def test_deterministic(case):
    name, sc, scene, _, _ = case
    Q = cuda(_queries(sc, 5000, seed=16))
    a = api.sd_eval_grad(scene, Q, 50.0, 0.5)
    b = api.sd_eval_grad(scene, Q, 50.0, 0.5)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_concurrent_threads_and_streams(case):
    """One scene evaluated from two host threads at once, each on a stream of
    its own (the scene is read-only after the build; every call allocates its
    own scratch stream-ordered): every result equals the sequential one bit
    for bit."""
    import threading
    name, sc, scene, _, _ = case
    Qs = [cuda(_queries(sc, 7000 + 1000 * k, seed=30 + k)) for k in range(2)]
    ref = [api.sd_eval_grad(scene, Q, 50.0, 0.5) for Q in Qs]
    torch.cuda.synchronize()
    out, errors = [None, None], []

    def work(k):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                res = [api.sd_eval_grad(scene, Qs[k], 50.0, 0.5) for _ in range(4)]
            st.synchronize()
            out[k] = res
        except Exception as exc:   # reported below, in the test's own thread
            errors.append(exc)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k in range(2):
        for d, g in out[k]:
            assert torch.equal(d, ref[k][0]) and torch.equal(g, ref[k][1])


def test_value_only_equals_value_of_grad(case):
    name, sc, scene, _, _ = case
    Q = cuda(_queries(sc, 3000, seed=17))
    d1 = api.sd_eval(scene, Q, 50.0, 0.5)
    d2, _ = api.sd_eval_grad(scene, Q, 50.0, 0.5)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2)


def test_query_sorting_does_not_change_results(case):
    """The query order only changes when each lane's queued leaf terms are
    folded into its sums (the wave-cooperative leaf stage), i.e. the summation
    order: results agree to rounding, and the set of terms is identical."""
    name, sc, scene, _, _ = case
    Q = cuda(_queries(sc, 6000, seed=18))
    a = api.sd_eval_grad(scene, Q, 50.0, 0.5)
    b = api.sd_eval_grad(scene, Q, 50.0, 0.5, flags=api.SD_NO_QUERY_SORT)
    torch.cuda.synchronize()
    da, db = a[0].double(), b[0].double()
    assert torch.all((da - db).abs() <= 1e-6 * (da.abs() + 1e-3))
    assert torch.allclose(a[1], b[1], rtol=1e-5, atol=1e-6)
    ca = api.sd_eval_counters(scene, Q, 50.0, 0.5, flags=api.SD_NO_PRUNE)
    cb = api.sd_eval_counters(scene, Q, 50.0, 0.5, flags=api.SD_NO_PRUNE | api.SD_NO_QUERY_SORT)
    assert torch.equal(ca, cb)


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------
def test_literal_scale_flag():
    require_gpu()
    sc = scenes.bumpy_icosphere(level=2, seed=3)
    scene = api.upload_scene(sc, flags=api.SD_BUILD_A_PAPER_LITERAL)
    osc = oracle_scene(sc, a_literal=True)
    assert scene.info()["A"][2] == 6.0 == osc.A_T
    Q = _queries(sc, 1000, seed=19)
    # the printed A leaves some weights below 1, so the exact value itself may
    # exceed d_min (by at most log(6.00426 / 6) / alpha): the unclamped output
    # is the one that follows the oracle here
    d, g = _run(scene, Q, 40.0, 0.0, flags=NOCONS)
    dr, gr, dm = O.brute(osc, Q.astype(np.float64), 40.0)
    compare(d, g, dr, gr, floor_of(sc), what="literal A", dmin=dm)


def test_empty_scene_and_empty_queries():
    require_gpu()
    V = cuda(np.zeros((4, 3), np.float32))
    scene = api.sd_build_bvh(V)
    Q = cuda(np.random.default_rng(0).uniform(-1, 1, (300, 3)).astype(np.float32))
    d, g = api.sd_eval_grad(scene, Q, 10.0, 0.5)
    torch.cuda.synchronize()
    assert torch.all(torch.isinf(d)) and torch.all(d > 0) and torch.all(g == 0)
    d = api.sd_eval(scene, Q, 10.0, 0.5)
    assert torch.all(torch.isinf(d))
    c = api.sd_eval_counters(scene, Q, 10.0, 0.5)
    assert torch.all(c == 0)
    sc2 = api.upload_scene(scenes.point_sphere(50, 1)[0])
    d, g = api.sd_eval_grad(sc2, cuda(np.zeros((0, 3), np.float32)), 10.0, 0.5)
    assert d.numel() == 0


@pytest.mark.parametrize("kind", ["point", "edge", "triangle"])
def test_single_primitive(kind):
    require_gpu()
    rng = np.random.default_rng(5)
    V = rng.uniform(-1, 1, (3, 3)).astype(np.float32)
    sc = scenes.Scene(V=V, P=np.array([1], np.int32) if kind == "point" else None,
                      E=np.array([[0, 2]], np.int32) if kind == "edge" else None,
                      T=np.array([[0, 1, 2]], np.int32) if kind == "triangle" else None)
    scene = api.upload_scene(sc)
    Q = rng.uniform(-2, 2, (777, 3)).astype(np.float32)
    Q[0] = V[1] if kind != "edge" else V[0]      # a query on the primitive
    for beta in (0.0, 0.5):
        d, g = _run(scene, Q, 30.0, beta)
        dr, gr, _ = O.barnes_hut(oracle_scene(sc), oracle_trees(scene), Q.astype(np.float64), 30.0, beta,
                                 cut_f32=True)
        compare(d, g, dr, gr, 1e-3, what=f"single {kind} beta={beta}")
    d, g = _run(scene, Q, 30.0, 0.0)
    assert d[0] <= 0 and np.all(g[0] == 0)       # Eq. 11: zero gradient at d = 0


def test_nan_query_gives_nan():
    require_gpu()
    sc = scenes.bumpy_icosphere(level=2, seed=3)
    scene = api.upload_scene(sc)
    Q = np.zeros((5, 3), np.float32)
    Q[2, 1] = np.nan
    d, g = _run(scene, Q, 20.0, 0.5)
    assert np.isnan(d[2]) and np.all(np.isfinite(np.delete(d, 2)))


def test_degenerate_triangles():
    require_gpu()
    V = np.array([[0, 0, 0], [1, 1, 1], [2, 2, 2], [0, 1, 0], [1, 0, 0], [0, 0, 1]], np.float32)
    T = np.array([[0, 1, 2], [0, 4, 3], [0, 5, 4], [0, 3, 5], [3, 4, 5], [1, 1, 2]], np.int32)
    sc = scenes.Scene(V=V, T=T)
    scene = api.upload_scene(sc)
    Q = np.random.default_rng(6).uniform(-1, 3, (1000, 3)).astype(np.float32)
    d, g = _run(scene, Q, 25.0, 0.0)
    osc = oracle_scene(sc)
    dr, gr, dm = O.brute(osc, Q.astype(np.float64), 25.0)
    compare(d, g, dr, gr, 1e-3, what="degenerate", dmin=dm)
    _check_conservative(scene, Q, 25.0, 0.0, dm, d)


def test_invalid_arguments_raise():
    require_gpu()
    V = cuda(np.zeros((3, 3), np.float32))
    with pytest.raises(api.SdError) as e:
        api.sd_build_bvh(V, T=cuda(np.array([[0, 1, 5]], np.int32)))
    assert e.value.code == -1 and "index" in str(e.value)
    with pytest.raises(api.SdError):
        api.sd_build_bvh(V, E=cuda(np.array([[0, -1]], np.int32)))
    sc = api.upload_scene(scenes.point_sphere(20, 1)[0])
    Q = cuda(np.zeros((4, 3), np.float32))
    for bad in (dict(alpha=0.0), dict(alpha=-1.0), dict(alpha=float("nan")), dict(alpha=1.0, beta=-0.1),
                dict(alpha=1.0, alpha_u=-1.0)):
        with pytest.raises(api.SdError):
            api.sd_eval(sc, Q, **bad)


def test_huge_alpha_is_finite():
    """Large alpha d never overflows: the running maximum is factored out
    (the paper's FP64 sums would return inf far from the data)."""
    require_gpu()
    sc = scenes.point_sphere(500, 1)[0]
    scene = api.upload_scene(sc)
    Q = np.array([[40.0, 0, 0], [0, -30, 5], [0.1, 0.2, 0.3]], np.float32)
    dm = O.dmin(oracle_scene(sc), Q.astype(np.float64))
    for beta in (0.0, 0.5):
        d, g = _run(scene, Q, 5e4, beta)
        assert np.all(np.isfinite(d)) and np.all(np.isfinite(g))
        _check_conservative(scene, Q, 5e4, beta, dm, d)
        # App. A with unit weights: d_min - log|F|/alpha <= d (brute force, beta = 0);
        # the Barnes-Hut bound divides d_min by (1 + beta)
        assert np.all(d >= dm / (1 + beta) - np.log(500) / 5e4 - 1e-5)


@pytest.mark.parametrize("alpha", [10.0, 100.0, 1000.0, 5000.0])
def test_alpha_sweep_terrain_both_precision_modes(alpha):
    """Terrain points + torus + hemisphere net across the alpha range: the
    default output matches the oracle and is conservative, with and without
    the (now always-on) FP64 final logarithm flag."""
    require_gpu()
    sc = scenes.terrain_scene(scale=0.002, seed=9)
    scene = api.upload_scene(sc)
    Q = scenes.terrain_queries(sc, 3000, seed=10)
    Qd = cuda(Q)
    osc = oracle_scene(sc)
    dr, gr, st = O.barnes_hut(osc, oracle_trees(scene), Q.astype(np.float64), alpha, 0.5, cut_f32=True)
    dm = O.dmin(osc, Q.astype(np.float64))
    for fl in (0, api.SD_ROOTLOG_F64):
        d, g = api.sd_eval_grad(scene, Qd, alpha, 0.5, flags=fl)
        torch.cuda.synchronize()
        d, g = d.cpu().numpy(), g.cpu().numpy()
        compare(d, g, dr, gr, floor_of(sc), what=f"alpha {alpha} flags {fl}", dmin=dm)
        _check_conservative(scene, Q, alpha, 0.5, dm, d, flags=fl)


@pytest.mark.parametrize("nq", [1, 63, 64, 65, 4095, 4096, 4097])
def test_query_counts_around_the_wave_and_the_sort_threshold(nq):
    """The traversal is launched one wave (64 queries) per workgroup and sorts
    its queries by Morton code from 4,096 on: counts on both sides of each
    boundary, on the mixed three-class scene, against the oracle element by
    element, with value-only and value+gradient calls agreeing bit for bit."""
    require_gpu()
    sc = _mixed_scene()
    scene = api.upload_scene(sc)
    try:
        Q = _queries(sc, nq, seed=nq)
        d, g = _run(scene, Q, 50.0, 0.5)
        dv = api.sd_eval(scene, cuda(Q), 50.0, 0.5)
        torch.cuda.synchronize()
        assert np.array_equal(dv.cpu().numpy(), d)
        osc = oracle_scene(sc)
        dr, gr, _ = O.barnes_hut(osc, oracle_trees(scene), Q.astype(np.float64), 50.0, 0.5, cut_f32=True)
        dm = O.dmin(osc, Q.astype(np.float64))
        compare(d, g, dr, gr, floor_of(sc), what=f"mixed nq={nq}", dmin=dm)
        _check_conservative(scene, Q, 50.0, 0.5, dm, d)
    finally:
        scene.free()
