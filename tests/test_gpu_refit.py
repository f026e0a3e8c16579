"""GPU: the bottom-up box refit at the sizes where its work splits.

The refit runs in two launches: the nodes whose leaves lie inside one
workgroup's unit of 16,384 consecutive leaves, then the nodes that span units,
by one workgroup from a list of their finished children.  Point clouds of
sizes around the unit (and tiny ones) are built and the exported hierarchy is
checked exactly: every internal box is the union of its children's boxes (FP32
min / max are exact), every leaf box is its point, the depth-first layout puts
each left child right after its parent, and every point sits in one leaf.
Uniform, clustered and duplicated points give shallow and deep Karras trees.
"""
import numpy as np
import pytest

from tests.gpu_common import api, cuda, require_gpu, torch

pytestmark = pytest.mark.gpu

UNIT = 16_384


def _points(n, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    if kind == "clustered":
        c = rng.uniform(-1, 1, (max(1, n // 500), 3))
        return (c[rng.integers(0, len(c), n)] + rng.normal(0, 1e-3, (n, 3))).astype(np.float32)
    # duplicated: a few distinct points repeated (equal Morton codes)
    d = rng.uniform(-1, 1, (7, 3))
    return d[rng.integers(0, 7, n)].astype(np.float32)


def _check_points_hierarchy(P, scene):
    n = len(P)
    box, left, right, prim = api.sd_export_bvh(scene, 0)
    assert len(left) == 2 * n - 1
    lv = np.where(left < 0)[0]
    assert len(lv) == n
    assert np.array_equal(np.sort(prim[lv]), np.arange(n))
    assert np.array_equal(box[lv, :3], P[prim[lv]]) and np.array_equal(box[lv, 3:], P[prim[lv]])
    internal = np.where(left >= 0)[0]
    assert np.all(left[internal] == internal + 1)
    l, r = left[internal], right[internal]
    assert np.array_equal(box[internal, :3], np.minimum(box[l, :3], box[r, :3]))
    assert np.array_equal(box[internal, 3:], np.maximum(box[l, 3:], box[r, 3:]))
    # every node except the root is the child of exactly one node
    ch = np.concatenate([l, r])
    assert np.array_equal(np.sort(ch), np.arange(1, 2 * n - 1))


@pytest.mark.parametrize("n", [1, 2, 3, 1023, 1025, UNIT - 1, UNIT, UNIT + 1, 2 * UNIT + 1, 100_003])
@pytest.mark.parametrize("kind", ["uniform", "clustered", "duplicated"])
def test_refit_exact_around_the_unit(n, kind):
    require_gpu()
    P = _points(n, kind, seed=n + len(kind))
    print(f"refit check: n={n} kind={kind}", flush=True)
    scene = api.sd_build_bvh(cuda(P), P=torch.arange(n, dtype=torch.int32, device="cuda"))
    try:
        _check_points_hierarchy(P, scene)
    finally:
        scene.free()


def test_refit_repeated_builds_agree():
    """Two builds of the same 300,000 clustered points export the same
    hierarchy (the refit's order of work does not change the boxes)."""
    require_gpu()
    P = _points(300_000, "clustered", seed=5)
    Pd = cuda(P)
    idx = torch.arange(len(P), dtype=torch.int32, device="cuda")
    a = api.sd_build_bvh(Pd, P=idx)
    b = api.sd_build_bvh(Pd, P=idx)
    try:
        ta, tb = api.sd_export_bvh(a, 0), api.sd_export_bvh(b, 0)
        for x, y in zip(ta, tb):
            assert np.array_equal(x, y)
        _check_points_hierarchy(P, a)
    finally:
        a.free()
        b.free()
