"""The allocation-free entry point (sd_eval_grad_noalloc) against the
allocating one (sd_eval_grad) through the C ABI: two calls in a row on one GPU,
the second with fewer queries (both take the Morton-ordered path, so the
second reuses the static scratch the first filled), then a call below the
ordering threshold and the size limit."""
import numpy as np
import pytest

from tests.gpu_common import O, api, compare, cuda, floor_of, oracle_scene, oracle_trees, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu


def test_noalloc_equals_allocating_entry_point():
    require_gpu()
    sc = scenes.bumpy_icosphere(level=4, seed=2)
    scene = api.upload_scene(sc)
    osc, trees = oracle_scene(sc), oracle_trees(scene)
    for n, seed in ((300_001, 41), (5_003, 42), (777, 43)):
        Qh = scenes.icosphere_queries(sc, n, seed_box=seed, seed_surf=seed + 100)
        Q = cuda(Qh)
        d = torch.empty(n, dtype=torch.float32, device="cuda")
        g = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        api.sd_eval_grad_noalloc(scene, Q, 50.0, 0.5, out=d, grad_out=g)
        d_ref, g_ref = api.sd_eval_grad(scene, Q, 50.0, 0.5)
        torch.cuda.synchronize()
        assert torch.equal(d, d_ref) and torch.equal(g, g_ref), n
        # and the oracle's bar on a sample of the outputs
        idx = np.sort(np.random.default_rng(seed).choice(n, min(n, 1500), replace=False))
        dr, gr, _ = O.barnes_hut(osc, trees, Qh[idx].astype(np.float64), 50.0, 0.5, cut_f32=True)
        compare(d.cpu().numpy()[idx], g.cpu().numpy()[idx], dr, gr, floor_of(sc), what=f"noalloc n={n}")


def test_noalloc_limit_and_arguments():
    require_gpu()
    sc = scenes.bumpy_icosphere(level=2, seed=2)
    scene = api.upload_scene(sc)
    n = api.SD_NOALLOC_MAX_QUERIES + 1
    Q = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(api.SdError) as e:
        api.sd_eval_grad_noalloc(scene, Q, 50.0, 0.5)
    assert e.value.code == -1 and "limit" in str(e.value)
    d, g = api.sd_eval_grad_noalloc(scene, Q[:0], 50.0, 0.5)
    assert d.numel() == 0
    with pytest.raises(api.SdError):
        api.sd_eval_grad_noalloc(scene, Q[:10], -1.0, 0.5)
