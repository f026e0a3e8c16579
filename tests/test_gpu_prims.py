"""GPU parity for edges and triangles as query primitives (Sec. 3.4): the HIP
library through the C ABI against the FP64 oracle on the exported
hierarchies (opening decisions in FP32 on both sides), every query, plus
reduction to point queries, conservativeness and argument errors.

Queries that touch or cross the data mesh are left out of the element-wise
comparison: there the distance is 0 and the weight is taken at one point of
the intersection, which is not unique (both sides are still checked to give
a value at or below 0 + rounding)."""
import numpy as np
import pytest

from tests.gpu_common import (O, api, compare, cuda, floor_of, oracle_scene, oracle_trees, require_gpu, scenes,
                              torch)

pytestmark = pytest.mark.gpu


def _scenes():
    rng = np.random.default_rng(21)
    ico = scenes.bumpy_icosphere(level=2, seed=4)
    out = {"triangles": ico}
    V = rng.uniform(-1, 1, (300, 3)).astype(np.float32)
    out["points"] = scenes.Scene(V=V, P=np.arange(300, dtype=np.int32))
    t = np.linspace(0, 6 * np.pi, 201)
    W = np.column_stack([np.cos(t), np.sin(t), t / (3 * np.pi) - 1]).astype(np.float32)
    out["edges"] = scenes.Scene(V=W, E=np.column_stack([np.arange(200), np.arange(1, 201)]).astype(np.int32))
    Vm = np.concatenate([ico.V, V[:100] * 1.6, W]).astype(np.float32)
    nI = len(ico.V)
    out["mixed"] = scenes.Scene(V=Vm, P=np.arange(nI, nI + 100, dtype=np.int32), T=ico.T,
                                E=(np.column_stack([np.arange(200), np.arange(1, 201)]) + nI + 100).astype(np.int32))
    return out


SCENES = _scenes()


def _prims(rng, n, nv, spread=1.7, size=0.25):
    c = rng.uniform(-spread, spread, (n, 1, 3))
    return (c + rng.normal(size=(n, nv, 3)) * size).astype(np.float32)


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("nv", [2, 3])
@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_query_primitives_match_oracle(name, nv, beta):
    require_gpu()
    sc = SCENES[name]
    scene = api.upload_scene(sc)
    osc, trees = oracle_scene(sc), oracle_trees(scene)
    rng = np.random.default_rng(100 + 10 * nv + int(beta * 10))
    G = _prims(rng, 3000, nv)
    alpha = 40.0
    d, g = api.sd_eval_grad_prims(scene, cuda(G), alpha, beta)
    torch.cuda.synchronize()
    d, g = d.cpu().numpy(), g.cpu().numpy()
    dc = d
    dr, gr, st = O.barnes_hut_prims(osc, trees, G.astype(np.float64), alpha, beta, cut_f32=True)
    _, _, dm = O.brute_prims(osc, G.astype(np.float64), alpha)
    sep = dm > 1e-3
    assert sep.mean() > 0.6
    # The point-query gate for value and gradient (1e-5, relative; value floor
    # 1e-3 of the diagonal, gradient floor 1e-2): the closest point g(lambda)
    # is formed in FP64, so the terms at it are as exact as the point-query
    # terms (an FP32 g(lambda) moved the distance at first order wherever a
    # vertex or an edge of g is closest: errors up to 2.4e-5 in value and
    # 4e-4 in gradient).
    floor = floor_of(sc)
    compare(d, g, dr, gr, floor, mask=sep, what=f"{name} nv={nv} beta={beta}", dmin=dm)
    # the default (conservative) result never exceeds the minimum distance
    assert np.all(dc[sep] <= dm[sep])
    assert np.all(dc[~sep] <= dm[~sep] + 1e-5)


def test_degenerate_primitives_are_point_queries():
    require_gpu()
    sc = SCENES["mixed"]
    scene = api.upload_scene(sc)
    rng = np.random.default_rng(3)
    Q = rng.uniform(-1.8, 1.8, (5000, 3)).astype(np.float32)
    fl = api.SD_NO_CONSERVATIVE_ROUNDING
    d0, g0 = api.sd_eval_grad(scene, cuda(Q), 40.0, 0.5, flags=fl)
    for nv in (1, 2, 3):
        G = np.repeat(Q[:, None, :], nv, axis=1)
        d, g = api.sd_eval_grad_prims(scene, cuda(G), 40.0, 0.5, flags=fl)
        np.testing.assert_allclose(d.cpu().numpy(), d0.cpu().numpy(), rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(g.cpu().numpy(), g0.cpu().numpy(), rtol=1e-5, atol=1e-6)


def test_prims_edge_cases():
    require_gpu()
    scene = api.upload_scene(SCENES["edges"])
    G = cuda(np.zeros((0, 2, 3), np.float32))
    d, g = api.sd_eval_grad_prims(scene, G, 40.0)
    assert d.numel() == 0
    empty = api.upload_scene(scenes.Scene(V=np.zeros((3, 3), np.float32)))
    d, g = api.sd_eval_grad_prims(empty, cuda(np.ones((5, 3, 3), np.float32)), 40.0)
    assert torch.all(torch.isposinf(d)) and torch.all(g == 0)
    with pytest.raises(api.SdError):
        api.sd_eval_grad_prims(scene, cuda(np.ones((5, 2, 3), np.float32)), 40.0, beta=-1.0)
    p = api.params(40.0, 0.5)
    rc = api.lib().sd_eval_grad_prims(scene.handle, api._c_p(0), api.ctypes.c_int32(4), api._i64(1),
                                      api.ctypes.byref(p), api._c_p(0), api._c_p(0), api._stream())
    assert rc == -1   # SD_EINVAL
