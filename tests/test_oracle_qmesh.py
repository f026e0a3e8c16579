"""Pins of the query-mesh oracle (Sec. 3.6, Eq. 6-8) against closed forms, a
library log-sum-exp, finite differences and the rigid-translation identity."""
import numpy as np
import pytest
from scipy.special import logsumexp

from oracle import qmesh as QM


def _mixed_mesh(rng, nV=30, n_pts=8, n_edges=15, n_tris=12):
    prim = -np.ones((n_pts + n_edges + n_tris, 3), np.int64)
    prim[:n_pts, 0] = rng.choice(nV, n_pts, replace=False)
    for i in range(n_edges):
        prim[n_pts + i, :2] = rng.choice(nV, 2, replace=False)
    for i in range(n_tris):
        prim[n_pts + n_edges + i] = rng.choice(nV, 3, replace=False)
    return prim


def test_single_primitive_is_its_own_distance():
    g = np.array([[[0.3, -0.4, 0.866]]])
    for prim, nV, share in ((None, 1, 1.0), (np.array([[0, 1, -1]]), 2, 0.5), (np.array([[2, 0, 1]]), 3, 1 / 3)):
        D, w, vg = QM.query_mesh_lse(np.array([[0.7]]), g, 25.0, prim, nV)
        assert D[0] == pytest.approx(0.7, abs=1e-15)
        assert w[0, 0] == 1.0
        # the primitive's gradient is a rigid translation split equally between its vertices
        np.testing.assert_allclose(vg[0], np.repeat(g[0] * share, nV, axis=0), rtol=1e-15)


def test_two_points_closed_form():
    rng = np.random.default_rng(1)
    for a in (1.0, 30.0, 400.0):
        d = rng.uniform(-0.2, 1.0, (5, 2))
        D, w, _ = QM.query_mesh_lse(d, np.zeros((5, 2, 3)), a)
        lo, gap = d.min(1), np.abs(d[:, 0] - d[:, 1])
        np.testing.assert_allclose(D, lo - np.log1p(np.exp(-a * gap)) / a, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(w.sum(1), 1.0, rtol=1e-15)


def test_vertex_split_sum_equals_plain_logsumexp():
    """Eq. 7 (vertex form) equals Eq. 6, checked against scipy's logsumexp."""
    rng = np.random.default_rng(2)
    prim = _mixed_mesh(rng)
    d = rng.uniform(0.0, 2.0, (4, len(prim)))
    for a in (2.0, 50.0, 1e3):
        D, _, _ = QM.query_mesh_lse(d, np.zeros(d.shape + (3,)), a, prim, 30)
        np.testing.assert_allclose(D, -logsumexp(-a * d, axis=1) / a, rtol=1e-13, atol=1e-15)


def test_weights_are_the_derivative_of_D():
    rng = np.random.default_rng(3)
    d = rng.uniform(0.0, 1.0, (2, 9))
    a, h = 20.0, 1e-6
    D, w, _ = QM.query_mesh_lse(d, np.zeros((2, 9, 3)), a)
    for j in range(9):
        dp, dm_ = d.copy(), d.copy()
        dp[:, j] += h
        dm_[:, j] -= h
        fd = (QM.query_mesh_lse(dp, np.zeros((2, 9, 3)), a)[0] - QM.query_mesh_lse(dm_, np.zeros((2, 9, 3)), a)[0]) / (2 * h)
        np.testing.assert_allclose(w[:, j], fd, rtol=1e-7, atol=1e-9)


def test_vertex_gradients_sum_to_the_translation_derivative():
    """Translating the whole query mesh moves every primitive rigidly: the
    vertex gradients of Eq. 8 add up to sum_j w_j grad d_j."""
    rng = np.random.default_rng(4)
    prim = _mixed_mesh(rng)
    d = rng.uniform(0.0, 1.0, (3, len(prim)))
    g = rng.normal(size=(3, len(prim), 3))
    D, w, vg = QM.query_mesh_lse(d, g, 15.0, prim, 30)
    np.testing.assert_allclose(vg.sum(1), np.einsum("kj,kjc->kc", w, g), rtol=1e-12, atol=1e-14)


def test_point_query_mesh_gradient_matches_finite_differences(oracle_mod):
    """A point query mesh over a real data mesh: with d_j and grad d_j from the
    oracle's exact evaluation, Eq. 8 is the exact derivative of D in each query
    vertex (central differences of the whole composite)."""
    O = oracle_mod
    rng = np.random.default_rng(5)
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32)
    T = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
    sc = O.OracleScene(V, T=T)
    Q = rng.uniform(-0.6, 1.4, (7, 3))
    alpha, aq, h = 20.0, 8.0, 1e-5

    def total(Qx):
        d, g, _ = O.brute(sc, Qx, alpha)
        return QM.query_mesh_lse(d[None], g[None], aq)

    D, w, vg = total(Q)
    for v in range(len(Q)):
        for c in range(3):
            Qp, Qm = Q.copy(), Q.copy()
            Qp[v, c] += h
            Qm[v, c] -= h
            fd = (total(Qp)[0][0] - total(Qm)[0][0]) / (2 * h)
            assert vg[0, v, c] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_sharp_limit_and_monotonicity():
    rng = np.random.default_rng(6)
    d = rng.uniform(0.1, 1.0, (3, 40))
    prev = None
    for a in (1.0, 10.0, 100.0, 1e4):
        D, _, _ = QM.query_mesh_lse(d, np.zeros(d.shape + (3,)), a)
        assert np.all(D <= d.min(1) + 1e-15)                  # a smooth minimum lies below the minimum
        if prev is not None:
            assert np.all(D >= prev - 1e-15)                  # and rises toward it with alpha_q
        prev = D
    np.testing.assert_allclose(prev, d.min(1), atol=np.log(40) / 1e4 + 1e-12)


def test_infinite_and_nan_rows():
    d = np.array([[np.inf, np.inf], [0.5, np.inf], [0.5, np.nan]])
    D, w, vg = QM.query_mesh_lse(d, np.ones((3, 2, 3)), 10.0)
    assert np.isposinf(D[0]) and np.all(w[0] == 0) and np.all(vg[0] == 0)
    assert D[1] == 0.5 and w[1, 0] == 1.0 and w[1, 1] == 0.0
    assert np.isnan(D[2])
