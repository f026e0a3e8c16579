"""Pins of the oracle's valence counting (App. C.1-C.3) on meshes whose
valences are known by construction or counted by brute force, and of the
query-primitive gradient (Sec. 3.4) on edge and triangle data by finite
differences, wherever the closest point g(lambda) of every term is a vertex
of the query primitive (a rigid translation of g then moves every closest
pair rigidly, so the point-query gradient at that vertex is the exact
derivative)."""
import itertools

import numpy as np
import pytest

from paper_2108_10480_amd import scenes


# --------------------------------------------------------------------------
# edges (App. C.2): N_k = number of edges at vertex k, A_E = max_k N_k
# --------------------------------------------------------------------------
def test_edge_valences_of_known_graphs(oracle_mod):
    O = oracle_mod
    # open polyline 0-1-2-3-4: ends 1, interior 2
    E = np.array([[0, 1], [1, 2], [2, 3], [3, 4]])
    n0, n1, amax = O.edge_valences(E, 5)
    assert list(n0) == [1, 2, 2, 2] and list(n1) == [2, 2, 2, 1] and amax == 2
    # closed loop: every vertex 2
    E = np.array([[0, 1], [1, 2], [2, 3], [3, 0]])
    n0, n1, amax = O.edge_valences(E, 4)
    assert np.all(n0 == 2) and np.all(n1 == 2) and amax == 2
    # star: hub 0 with 7 spokes, leaves 1
    E = np.array([[0, k] for k in range(1, 8)])
    n0, n1, amax = O.edge_valences(E, 8)
    assert np.all(n0 == 7) and np.all(n1 == 1) and amax == 7
    # the hemisphere net of the terrain workload: the pole has one edge per
    # longitude, rim vertices 3 (two along the rim, one up), the rest 4
    sc = scenes.terrain_scene(0.002)
    E = sc.E - sc.E.min()
    n0, n1, amax = O.edge_valences(E, int(E.max()) + 1)
    deg = np.bincount(E.reshape(-1))
    assert amax == deg.max() == deg[0]
    assert set(np.unique(deg[1:])) <= {3, 4}


# --------------------------------------------------------------------------
# triangles (App. C.3): v_i = largest vertex valence of triangle i, e_i =
# largest number of triangles sharing one of its edges
# --------------------------------------------------------------------------
def _brute_triangle_valences(T):
    T = [tuple(int(x) for x in t) for t in T]
    v, e = [], []
    for t in T:
        v.append(max(sum(1 for u in T if a in u) for a in t))
        e.append(max(sum(1 for u in T if a in u and b in u) for a, b in itertools.combinations(t, 2)))
    return np.array(v), np.array(e)


def test_triangle_valences_of_known_meshes(oracle_mod):
    O = oracle_mod
    # closed tetrahedron: every vertex in 3 triangles, every edge in 2
    T = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]])
    v, e = O.triangle_valences(T, 4)
    assert np.all(v == 3) and np.all(e == 2)
    # icosahedron: every vertex in 5 triangles
    V, F = scenes.icosphere(0)
    v, e = O.triangle_valences(F, len(V))
    assert np.all(v == 5) and np.all(e == 2)
    # subdivided: the 12 original vertices keep valence 5, the new ones have 6,
    # and every triangle has a new vertex
    V, F = scenes.icosphere(2)
    deg = np.bincount(F.reshape(-1))
    assert (deg == 5).sum() == 12 and (deg == 6).sum() == len(V) - 12
    v, e = O.triangle_valences(F, len(V))
    assert np.all(v == 6) and np.all(e == 2)
    # torus grid: valence 6 everywhere
    tv, tf = scenes.torus_grid(12, 8, 1.0, 0.3)
    v, e = O.triangle_valences(tf, len(tv))
    assert np.all(v == 6) and np.all(e == 2)
    # an isolated triangle, and two triangles sharing an edge
    v, e = O.triangle_valences(np.array([[0, 1, 2]]), 3)
    assert list(v) == [1] and list(e) == [1]
    v, e = O.triangle_valences(np.array([[0, 1, 2], [2, 1, 3]]), 4)
    assert list(v) == [2, 2] and list(e) == [2, 2]
    # a non-manifold edge shared by three triangles
    v, e = O.triangle_valences(np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]]), 5)
    assert list(v) == [3, 3, 3] and list(e) == [3, 3, 3]


def test_triangle_valences_match_brute_force_on_open_patches(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    V, F = scenes.icosphere(2)
    for trial in range(4):
        keep = rng.random(len(F)) < 0.6          # open, with boundary edges (e = 1)
        T = F[keep]
        v, e = O.triangle_valences(T, len(V))
        vb, eb = _brute_triangle_valences(T)
        np.testing.assert_array_equal(v, vb)
        np.testing.assert_array_equal(e, eb)
        assert (eb == 1).any() or trial > 0


# --------------------------------------------------------------------------
# Sec. 3.4: edge and triangle data, the closest point of g at its vertex g0
# --------------------------------------------------------------------------
def _data_scene(O):
    """Edges (an open polyline: end valences 1 and 2, so the weight varies
    along the end edges) and an open triangle fan (valences 2-6), all with
    x > 0.4 and y > 0.4."""
    rng = np.random.default_rng(11)
    c = np.array([0.9, 0.9, 0.0])
    ring = [c + 0.35 * np.array([np.cos(t), np.sin(t), 0.3 * np.sin(3 * t)]) for t in np.linspace(0, 5.2, 6)]
    Vt = np.array([c] + ring)
    Tt = np.array([[0, k, k + 1] for k in range(1, 6)])
    Vp = np.array([[0.6 + 0.15 * k, 1.5 + 0.1 * np.sin(k), 0.2 * np.cos(k)] for k in range(6)])
    Ep = np.array([[k, k + 1] for k in range(5)]) + len(Vt)
    V = np.concatenate([Vt, Vp]).astype(np.float32)
    V += rng.normal(0, 0.01, V.shape).astype(np.float32)
    assert np.all(V[:, 0] > 0.4) and np.all(V[:, 1] > 0.4)
    return O.OracleScene(V, E=Ep, T=Tt)


@pytest.mark.parametrize("nv", [2, 3])
@pytest.mark.parametrize("alpha", [6.0, 30.0])
def test_translation_gradient_matches_finite_differences_for_edge_and_triangle_data(oracle_mod, nv, alpha):
    """g's other vertices point away from the data ((p - g0).(g_k - g0) < 0
    for every data point p), so g0 is the closest point of g to every data
    primitive; the weights vary along the data primitives (App. C)."""
    O = oracle_mod
    sc = _data_scene(O)
    rng = np.random.default_rng(int(alpha) + nv)
    G = []
    for _ in range(12):
        g0 = rng.uniform(-0.3, 0.3, 3)
        others = [g0 + np.array([-rng.uniform(0.2, 0.6), -rng.uniform(0.0, 0.1), rng.uniform(-0.1, 0.1)]),
                  g0 + np.array([-rng.uniform(0.0, 0.1), -rng.uniform(0.2, 0.6), rng.uniform(-0.1, 0.1)])]
        G.append([g0] + others[: nv - 1])
    G = np.array(G)
    V = sc.V.astype(np.float64)
    for g in G:
        for k in range(1, nv):
            assert np.all((V - g[0]) @ (g[k] - g[0]) < 0)
    d, grad, _ = O.brute_prims(sc, G, alpha)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        dp, _, _ = O.brute_prims(sc, G + e, alpha)
        dm_, _, _ = O.brute_prims(sc, G - e, alpha)
        np.testing.assert_allclose((dp - dm_) / (2 * h), grad[:, a], atol=2e-6)
    # and the same terms as a point query at g0 (the closest point of g)
    dq, gq, _ = O.brute(sc, G[:, 0, :].copy(), alpha)
    np.testing.assert_allclose(d, dq, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(grad, gq, rtol=1e-10, atol=1e-12)
