"""GPU: what the trained surrogate gains over the method without it.

On the bumpy level-7 icosphere (alpha = 50, beta = 0.5) a surrogate is trained
on labels from the exact evaluation (reduced budget: 8M samples, 30 epochs),
certified locally on held-out uniform queries, and used with routing on 8M
uniform queries.  Checked: training reduces the error of the network by more
than 10x; the certified routing leaves most queries to the network; routed
queries carry the exact results; the errors outside the band stay within the
certified margins on fresh queries except for a small fraction (an empirical
certificate).  The measured speed of the routed path against Barnes-Hut alone
is printed (the benchmark reports it at full size).
"""
import time

import numpy as np
import pytest

from tests.gpu_common import api, cuda, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu


def _ms(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def test_trained_surrogate_gain():
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    alpha, beta, band = 50.0, 0.5, 0.05
    sc = scenes.bumpy_icosphere(level=7, seed=2)
    scene = api.upload_scene(sc)
    Xtr = torch.as_tensor(scenes.surrogate_samples(sc, 8_000_000, seed=6), device="cuda")
    ytr = api.sd_eval(scene, Xtr, alpha, beta)
    Xva = torch.as_tensor(scenes.uniform_queries(1_000_000, 7, -1.5, 1.5), device="cuda")
    yva = api.sd_eval(scene, Xva, alpha, beta)
    sur = S.Surrogate(scenes.fourier_matrix(11, sigma=[0.5, 1.0, 2.0, 4.0]), scenes.surrogate_init(12),
                      max_batch=65536)
    rmse = lambda: float(((sur.forward(Xva, grad=False) - yva) ** 2).mean().sqrt())
    rmse0 = rmse()
    losses = S.train(sur, Xtr, ytr, 30, batch=65536, lr0=3e-3, lr_min=1e-5, seed=13)
    rmse1 = rmse()
    print(f"validation RMSE untrained {rmse0:.3e} -> trained {rmse1:.3e} ({len(losses)} steps)")
    assert rmse1 < rmse0 / 10

    lo, hi = (-1.5, -1.5, -1.5), (1.5, 1.5, 1.5)
    eps = sur.certify_cells(Xva, yva, lo, hi, grid=32, safety=1.5)
    n = 8_000_000
    Xin = torch.as_tensor(scenes.uniform_queries(n, 8, -1.5, 1.5), device="cuda")
    d, g, routed, nfb = S.sd_eval_surrogate(scene, sur, Xin, alpha, beta, band=band)
    nfb = int(nfb)
    de, ge = api.sd_eval_grad(scene, Xin, alpha, beta)
    r = routed.bool()
    frac = nfb / n
    err_out = (d - de).abs()[~r]
    print(f"global margin {eps:.3e}; routed fraction {frac:.3f}; max error outside the band "
          f"{float(err_out.max()):.3e}, p99 {float(torch.quantile(err_out[:1_000_000], 0.99)):.3e}")
    assert 0.0 < frac < 0.5
    # routed queries: exact Barnes-Hut (same terms; summation order may differ)
    rel = (d - de).abs()[r] / de.abs()[r].clamp_min(1e-3 * 3.0)
    assert float(rel.max()) < 2e-6
    # an empirical certificate: nearly every fresh query outside the band is
    # within the margin of its cell (plus the band it was tested against)
    yq = sur.forward(Xin, grad=False)
    assert torch.equal(yq[~r], d[~r])
    within = (d - de).abs()[~r] <= torch.as_tensor(float(eps), device="cuda")
    assert float(within.float().mean()) > 0.999

    t_sur = _ms(lambda: S.sd_eval_surrogate(scene, sur, Xin, alpha, beta, band=band))
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    t_bh = _ms(lambda: (api.sd_query_order(scene, Xin, out=perm),
                        api.sd_eval_grad_ordered(scene, Xin, perm, alpha, beta)))
    print(f"value+gradient on {n} uniform queries: surrogate path {t_sur:.2f} ms "
          f"({n / t_sur / 1e3:.0f} Mq/s), Barnes-Hut {t_bh:.2f} ms ({n / t_bh / 1e3:.0f} Mq/s), "
          f"ratio {t_bh / t_sur:.2f}")
