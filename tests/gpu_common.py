"""Shared helpers for the GPU parity tests (HIP library vs FP64 oracle)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O                      # noqa: E402
from paper_2108_10480_amd import api, scenes        # noqa: E402

VALUE_TOL = 1e-5        # |d - d_ref| / max(|d_ref|, 1e-3 scene diagonal)
GRAD_TOL = 1e-5         # |g - g_ref| / max(|g_ref|, 1e-2)


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test needs an MI355X")


def cuda(a, dt=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dt is not None:
        t = t.to(dt)
    return t.cuda()


def oracle_scene(sc, a_literal=False):
    return O.OracleScene(sc.V, P=sc.P, E=sc.E, T=sc.T, a_literal=a_literal)


def oracle_trees(scene):
    out = []
    for c in range(3):
        t = api.sd_export_bvh(scene, c)
        out.append(None if t is None else O.OracleTree(*t))
    return out


def floor_of(sc):
    lo, hi = scenes.scene_aabb(sc)
    return 1e-3 * float(np.linalg.norm(hi - lo))


def compare(d, g, dr, gr, floor, mask=None, vtol=VALUE_TOL, gtol=GRAD_TOL, what="", dmin=None):
    """Element-by-element comparison with the oracle; dmin (optional) is only
    printed for the worst query."""
    d = np.asarray(d, np.float64)
    ev = O.value_error(d, dr, floor)
    if mask is None:
        mask = np.ones(len(d), bool)
    bad = np.isnan(d) != np.isnan(dr)
    assert not bad.any(), f"{what}: NaN mismatch"
    fin = np.isfinite(dr) & mask
    assert np.all(np.isposinf(d[np.isposinf(dr) & mask])), f"{what}: +inf mismatch"
    emax = ev[fin].max() if fin.any() else 0.0
    if emax > vtol:
        k = int(np.argmax(np.where(fin, ev, 0)))
        extra = "" if dmin is None else f" dmin={np.asarray(dmin)[k]:.9g}"
        print(f"{what}: worst query {k}: d={d[k]:.9g} ref={dr[k]:.9g}{extra} floor={floor:.3g}")
    assert emax <= vtol, f"{what}: value err {emax:.3e}"
    if g is not None:
        eg = O.grad_error(g, gr)[fin]
        gm = eg.max() if len(eg) else 0.0
        if gm > gtol:
            k = int(np.flatnonzero(fin)[np.argmax(eg)])
            print(f"{what}: worst gradient query {k}: g={np.asarray(g)[k]} ref={gr[k]} d={d[k]:.9g}")
        assert gm <= gtol, f"{what}: grad err {gm:.3e}"
        return emax, gm
    return emax, None
