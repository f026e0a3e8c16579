"""GPU: sphere tracing of the smooth distance's level sets (Sec. 4.2) through
the C ABI, against closed forms and the FP64 reference tracer driven by the
oracle's Barnes-Hut evaluation (FP32 opening decisions) on the exported
hierarchies."""
import numpy as np
import pytest

from oracle import trace as TR
from tests.gpu_common import O, api, cuda, oracle_scene, oracle_trees, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu


def test_single_point_closed_form():
    """One point at the origin: d = |x| exactly, so a ray from (3, b, 0) along
    -x meets the level 0.5 at 3 - sqrt(0.25 - b^2) for b < 0.5 and misses
    otherwise; a ray starting inside the level set hits at t = 0."""
    require_gpu()
    sc = scenes.Scene(V=np.zeros((1, 3), np.float32), P=np.array([0], np.int32))
    scene = api.upload_scene(sc)
    b = np.array([0.0, 0.1, 0.3, 0.45, 0.6, 0.9, 0.0], np.float32)
    Oo = np.stack([np.full_like(b, 3.0), b, np.zeros_like(b)], 1)
    Oo[-1] = [0.2, 0.0, 0.0]
    U = np.tile(np.array([-1.0, 0.0, 0.0], np.float32), (len(b), 1))
    t, steps = api.sd_sphere_trace(scene, cuda(Oo), cuda(U), alpha=50.0, beta=0.5, level=0.5, eps=1e-5,
                                   t_max=8.0, max_steps=2000)
    t = t.cpu().numpy()
    hit = b[:-1] < 0.5
    np.testing.assert_allclose(t[:-1][hit], 3 - np.sqrt(0.25 - b[:-1][hit].astype(np.float64) ** 2), atol=2e-5)
    assert np.all(np.isposinf(t[:-1][~hit]))
    assert t[-1] == 0.0 and steps.cpu().numpy()[-1] == 1


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_icosphere_trace_matches_oracle_tracer(beta):
    """Triangles of a bumpy icosphere with the ablation parameters
    (alpha 200, alpha_U 1200): hit distances against the FP64 tracer."""
    require_gpu()
    sc = scenes.bumpy_icosphere(level=3, seed=2)
    scene = api.upload_scene(sc)
    osc, trees = oracle_scene(sc), oracle_trees(scene)
    rng = np.random.default_rng(5)
    n = 96
    Oo = rng.normal(size=(n, 3))
    Oo = (2.5 * Oo / np.linalg.norm(Oo, axis=1, keepdims=True)).astype(np.float32)
    target = rng.uniform(-0.5, 0.5, (n, 3))
    U = target - Oo
    U = (U / np.linalg.norm(U, axis=1, keepdims=True)).astype(np.float32)
    kw = dict(level=0.0, eps=1e-4, t_max=6.0, max_steps=512)
    t, _ = api.sd_sphere_trace(scene, cuda(Oo), cuda(U), alpha=200.0, beta=beta, alpha_u=1200.0, **kw)
    t = t.cpu().numpy().astype(np.float64)
    dist = lambda X: O.barnes_hut(osc, trees, X, 200.0, beta, alpha_u=1200.0, cut_f32=True)[0]
    tr, _ = TR.sphere_trace(dist, Oo, U, **kw)
    assert np.array_equal(np.isposinf(t), np.isposinf(tr))
    fin = np.isfinite(tr)
    assert fin.sum() > n // 2
    # both stop within eps of the level set; their last steps differ by rounding
    np.testing.assert_allclose(t[fin], tr[fin], atol=3 * kw["eps"])


def test_trace_edge_cases():
    require_gpu()
    sc = scenes.bumpy_icosphere(level=1, seed=2)
    scene = api.upload_scene(sc)
    e = torch.empty((0, 3), device="cuda")
    t, s = api.sd_sphere_trace(scene, e, e, alpha=50.0)
    assert t.numel() == 0
    Oo = cuda(np.array([[3.0, 0.0, 0.0], [np.nan, 0.0, 0.0]], np.float32))
    U = cuda(np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]], np.float32))
    t, s = api.sd_sphere_trace(scene, Oo, U, alpha=50.0, t_max=5.0)
    assert torch.all(torch.isposinf(t))            # pointing away; a NaN ray
    for kw in (dict(eps=0.0), dict(t_max=-1.0), dict(max_steps=0), dict(level=float("nan"))):
        with pytest.raises(api.SdError):
            api.sd_sphere_trace(scene, Oo, U, alpha=50.0, **kw)
    with pytest.raises(api.SdError):
        api.sd_sphere_trace(scene, Oo, U, alpha=-1.0)
