"""The synthetic input recipes (no GPU): sizes and structure of the benchmark
workloads as stated for them, so that a change of a generator cannot silently
change what the benchmark measures."""
import numpy as np

from paper_2108_10480_amd import scenes


def test_bumpy_icosphere_workload():
    sc = scenes.bumpy_icosphere(level=7, seed=2)
    assert sc.V.shape == (163842, 3) and sc.T.shape == (327680, 3) and sc.P is None and sc.E is None
    r = np.linalg.norm(sc.V.astype(np.float64), axis=1)
    assert 0.6 <= r.min() and r.max() <= 1.4                  # star-shaped radial bumps
    # closed manifold: every edge shared by exactly two triangles; valences 5 or 6
    e = np.sort(np.concatenate([sc.T[:, [0, 1]], sc.T[:, [1, 2]], sc.T[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e[:, 0].astype(np.int64) * len(sc.V) + e[:, 1], return_counts=True)
    assert np.all(cnt == 2)
    val = np.bincount(sc.T.ravel(), minlength=len(sc.V))
    assert set(np.unique(val)) == {5, 6}
    Q = scenes.icosphere_queries(sc, 100_000, seed_box=3, seed_surf=4)
    assert Q.shape == (100_000, 3) and Q.dtype == np.float32
    assert np.all(np.abs(Q[:50_000]) <= 1.5)                  # half uniform in the box
    rq = np.linalg.norm(Q[50_000:].astype(np.float64), axis=1)
    assert 0.55 < rq.min() and rq.max() < 1.45                 # half within the band around the surface


def test_street_workload():
    sc, body = scenes.street_scene(1.0)
    assert sc.counts() == (2_000_000, 20_000, 50_000)
    assert body.shape == (25_000, 3)
    lo, hi = scenes.scene_aabb(sc)
    assert lo[0] >= -0.5 and hi[0] <= 100.5 and lo[1] >= -14.5 and hi[1] <= 14.5
    R, t = scenes.rigid_transforms(256, seed=5)
    assert R.shape == (256, 3, 3) and t.shape == (256, 3)
    np.testing.assert_allclose(R @ R.transpose(0, 2, 1), np.broadcast_to(np.eye(3), (256, 3, 3)), atol=1e-6)
    assert np.allclose(np.linalg.det(R.astype(np.float64)), 1.0, atol=1e-5)
    assert np.all(t >= [5, -8, 0.2]) and np.all(t <= [95, 8, 6])


def test_terrain_workload_structure():
    """At one hundredth of the size (the full size holds 20M points, 1M
    triangles, about 200k edges): every class present, counts scaling."""
    sc = scenes.terrain_scene(0.01)
    nP, nE, nT = sc.counts()
    assert nP == 200_000 and nT == 2 * 100 * 50 and nE > 1000
    Q = scenes.terrain_queries(sc, 10_000, seed=10)
    lo, hi = scenes.scene_aabb(sc)
    ext = hi - lo
    assert np.all(Q >= lo - 0.1 * ext - 1e-6) and np.all(Q <= hi + 0.1 * ext + 1e-6)
