"""Pins of the oracle for edges and triangles as query primitives (Sec. 3.4):
simplex-simplex distances against an independent QP solve (App. B, Eq. 10),
reduction to the point query, exactness at beta = 0, conservativeness of the
far field with the halfspace box distance, and finite differences of the
rigid-translation gradient where the weights are constant."""
import numpy as np
import pytest
from scipy.optimize import minimize

from tests._trees import median_tree


def _qp_distance(A, B):
    """min |sum a_i A_i - sum b_j B_j| over two probability simplices (SLSQP),
    from several starts."""
    na, nb = len(A), len(B)

    def f(x):
        a, b = x[:na], x[na:]
        r = a @ A - b @ B
        return r @ r

    cons = [{"type": "eq", "fun": lambda x: x[:na].sum() - 1}, {"type": "eq", "fun": lambda x: x[na:].sum() - 1}]
    best = np.inf
    rng = np.random.default_rng(0)
    for _ in range(6):
        x0 = np.concatenate([rng.dirichlet(np.ones(na)), rng.dirichlet(np.ones(nb))])
        r = minimize(f, x0, method="SLSQP", bounds=[(0, 1)] * (na + nb), constraints=cons,
                     options={"ftol": 1e-16, "maxiter": 500})
        best = min(best, r.fun)
    return np.sqrt(max(best, 0.0))


@pytest.mark.parametrize("na,nb", [(1, 2), (1, 3), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_simplex_distance_matches_qp(oracle_mod, na, nb):
    O = oracle_mod
    rng = np.random.default_rng(10 * na + nb)
    for _ in range(25):
        A = rng.normal(size=(na, 3))
        B = rng.normal(size=(nb, 3)) + rng.normal(size=3) * 1.5
        d, y = O.simplex_distance(A, B)
        assert d == pytest.approx(_qp_distance(A, B), abs=2e-6)
        # y lies on B, and its distance to A is d
        dy, _ = O.simplex_distance(A, y[None])
        assert dy == pytest.approx(d, abs=1e-9)
        db, _ = O.simplex_distance(B, y[None])
        assert db < 1e-9


def test_parallel_and_crossing_cases(oracle_mod):
    O = oracle_mod
    # parallel segments 1 apart, overlapping in x
    d, _ = O.simplex_distance([[0, 0, 0], [2, 0, 0]], [[1, 1, 0], [3, 1, 0]])
    assert d == pytest.approx(1.0, abs=1e-15)
    # a segment piercing a triangle, and two crossing triangles
    d, y = O.simplex_distance([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0.2, 0.2, -1], [0.2, 0.2, 1]])
    assert d == 0.0 and np.allclose(y, [0.2, 0.2, 0.0])
    d, _ = O.simplex_distance([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0.2, 0.2, -1], [0.3, 0.2, 1], [0.2, 0.3, 1]])
    assert d == 0.0


def _scene(O, rng):
    V = rng.uniform(-1, 1, (40, 3)).astype(np.float32)
    T = np.array([rng.choice(40, 3, replace=False) for _ in range(12)], np.int32)
    E = np.array([rng.choice(40, 2, replace=False) for _ in range(10)], np.int32)
    return O.OracleScene(V, P=np.arange(6), E=E, T=T)


def _trees(O, sc):
    out = []
    for xyz, k in ((sc.Pxyz, 1), (sc.Exyz, 2), (sc.Txyz, 3)):
        out.append(O.OracleTree(*median_tree(xyz, k)) if len(xyz) else None)
    return out


def test_degenerate_query_is_the_point_query(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(1)
    sc = _scene(O, rng)
    Q = rng.uniform(-2, 2, (30, 3))
    d, g, dm = O.brute(sc, Q, 20.0)
    for nv in (2, 3):
        G = np.repeat(Q[:, None, :], nv, axis=1)
        d2, g2, dm2 = O.brute_prims(sc, G, 20.0)
        np.testing.assert_allclose(d2, d, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(g2, g, rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(dm2, dm, rtol=1e-12)
        db, gb, _ = O.barnes_hut_prims(sc, _trees(O, sc), G, 20.0, 0.5)
        dp, gp, _ = O.barnes_hut(sc, _trees(O, sc), Q, 20.0, 0.5)
        np.testing.assert_allclose(db, dp, rtol=1e-12, atol=1e-13)


def _random_prims(rng, n, nv, spread=2.0, size=0.3):
    c = rng.uniform(-spread, spread, (n, 1, 3))
    return c + rng.normal(size=(n, nv, 3)) * size


@pytest.mark.parametrize("nv", [2, 3])
def test_beta_zero_is_exact_and_far_field_is_conservative(oracle_mod, nv):
    O = oracle_mod
    rng = np.random.default_rng(2 + nv)
    sc = _scene(O, rng)
    trees = _trees(O, sc)
    G = _random_prims(rng, 60, nv)
    d, g, dm = O.brute_prims(sc, G, 15.0)
    d0, g0, _ = O.barnes_hut_prims(sc, trees, G, 15.0, 0.0)
    np.testing.assert_allclose(d0, d, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g0, g, rtol=1e-9, atol=1e-11)
    for beta in (0.5, 1.0, 2.0):
        db, _, st = O.barnes_hut_prims(sc, trees, G, 15.0, beta)
        assert np.all(db <= dm + 1e-12)                 # App. A: never above the minimum distance
        assert np.all(st[:, 2] > 0) or beta < 1.0       # the far field is used
        # FP32 decisions agree with FP64 ones away from ties
        d32, _, _ = O.barnes_hut_prims(sc, trees, G, 15.0, beta, cut_f32=True)
        ok = st[:, 0] > 1e-5
        np.testing.assert_array_equal(d32[ok], db[ok])


@pytest.mark.parametrize("nv", [2, 3])
def test_translation_gradient_matches_finite_differences_for_points(oracle_mod, nv):
    """Point data (weight 1): the value's derivative in a rigid translation of
    g is the gradient (the closest pair moves without changing weights)."""
    O = oracle_mod
    rng = np.random.default_rng(7 + nv)
    P = rng.uniform(-1, 1, (25, 3)).astype(np.float32)
    sc = O.OracleScene(P, P=np.arange(25))
    G = _random_prims(rng, 20, nv, spread=1.6, size=0.2)
    d, g, _ = O.brute_prims(sc, G, 12.0)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        dp, _, _ = O.brute_prims(sc, G + e, 12.0)
        dm_, _, _ = O.brute_prims(sc, G - e, 12.0)
        np.testing.assert_allclose((dp - dm_) / (2 * h), g[:, a], atol=2e-6)
