"""GPU: out-of-memory paths and the library's device-memory accounting.

An allocation refused by the memory budget (sd_set_memory_budget) takes the
same path as a failed device allocation: the call returns SD_ENOMEM with a
message, and releases everything it had taken.  Checked where the refusal
comes first (scene build, surrogate creation) and in the middle of a call
(the query ordering's scratch after its permutation buffer); afterwards the
library holds exactly the bytes it held before, and the same calls succeed,
with the same results, once the budget is lifted."""
import gc

import numpy as np
import pytest

from tests.gpu_common import api, cuda, require_gpu, scenes, torch

pytestmark = pytest.mark.gpu

SD_ENOMEM = -2


@pytest.fixture
def no_budget_after():
    yield
    api.sd_set_memory_budget(None)


def _settle():
    gc.collect()
    torch.cuda.synchronize()


def test_scene_build_refused_by_the_budget_leaks_nothing(no_budget_after):
    require_gpu()
    _settle()
    base = api.sd_memory_in_use()
    sc = scenes.bumpy_icosphere(level=3, seed=1)
    scene = api.upload_scene(sc)
    held = api.sd_memory_in_use() - base
    assert held >= scene.info()["device_bytes"] > 0
    scene.free()
    assert api.sd_memory_in_use() == base
    # every budget below what the build needs fails cleanly, wherever the
    # refusal falls among its allocations
    for frac in (0.0, 0.3, 0.7, 0.99):
        api.sd_set_memory_budget(base + int(frac * held))
        with pytest.raises(api.SdError) as e:
            api.upload_scene(sc)
        assert e.value.code == SD_ENOMEM and "budget" in str(e.value)
        _settle()
        assert api.sd_memory_in_use() == base
    api.sd_set_memory_budget(None)
    scene = api.upload_scene(sc)
    assert api.sd_memory_in_use() - base == held
    scene.free()
    assert api.sd_memory_in_use() == base


def test_evaluation_scratch_refused_midway_leaks_nothing(no_budget_after):
    require_gpu()
    sc = scenes.bumpy_icosphere(level=3, seed=2)
    scene = api.upload_scene(sc)
    rng = np.random.default_rng(3)
    nq = 100_000                                  # ordered by Morton code (>= 4096 queries)
    Q = cuda(rng.uniform(-1.5, 1.5, (nq, 3)).astype(np.float32))
    d0, g0 = api.sd_eval_grad(scene, Q, 50.0, 0.5)
    _settle()
    base = api.sd_memory_in_use()
    # room for the permutation (4 bytes a query) but not for the sort's scratch
    api.sd_set_memory_budget(base + 4 * nq + 4096)
    with pytest.raises(api.SdError) as e:
        api.sd_eval_grad(scene, Q, 50.0, 0.5)
    assert e.value.code == SD_ENOMEM
    _settle()
    assert api.sd_memory_in_use() == base
    api.sd_set_memory_budget(None)
    d1, g1 = api.sd_eval_grad(scene, Q, 50.0, 0.5)
    assert torch.equal(d0, d1) and torch.equal(g0, g1)
    _settle()
    assert api.sd_memory_in_use() == base
    scene.free()


def test_surrogate_creation_refused_by_the_budget_leaks_nothing(no_budget_after):
    require_gpu()
    from paper_2108_10480_amd import surrogate as S
    _settle()
    base = api.sd_memory_in_use()
    B = np.random.default_rng(4).normal(size=(S.N_FREQ, 3)).astype(np.float32)
    theta = np.zeros(S.N_PARAMS, np.float32)
    sur = S.Surrogate(B, theta, max_batch=4096)
    held = api.sd_memory_in_use() - base
    sur.free()
    assert held > 0 and api.sd_memory_in_use() == base
    for frac in (0.0, 0.5, 0.95):
        api.sd_set_memory_budget(base + int(frac * held))
        with pytest.raises(api.SdError) as e:
            S.Surrogate(B, theta, max_batch=4096)
        assert e.value.code == SD_ENOMEM
        _settle()
        assert api.sd_memory_in_use() == base
