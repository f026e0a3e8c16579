"""Pins of the oracle's exact nearest distance by branch and bound (Eq. 2 over
a hierarchy) against the brute-force minimum over every primitive, which is
Eq. 2 as written.  The branch and bound serves the conservativeness checks of
large workloads (d <= d_min on every query)."""
import numpy as np

from paper_2108_10480_amd import scenes
from tests._trees import median_tree


def _mixed(seed):
    rng = np.random.default_rng(seed)
    ico = scenes.bumpy_icosphere(level=2, seed=seed)
    pl = scenes.random_polyline(120, seed=seed + 1, step=0.08)
    pts = rng.uniform(-1.3, 1.3, (150, 3)).astype(np.float32)
    nI, nL = len(ico.V), len(pl.V)
    V = np.concatenate([ico.V, pl.V, pts]).astype(np.float32)
    return V, np.arange(nI + nL, nI + nL + 150, dtype=np.int32), (pl.E + nI).astype(np.int32), ico.T


def test_branch_and_bound_equals_brute_force(oracle_mod):
    O = oracle_mod
    for seed in (1, 2):
        V, P, E, T = _mixed(seed)
        osc = O.OracleScene(V, P=P, E=E, T=T)
        trees = []
        for xyz, k in ((osc.Pxyz, 1), (osc.Exyz, 2), (osc.Txyz, 3)):
            t = median_tree(xyz, k)
            trees.append(None if t is None else O.OracleTree(*t))
        rng = np.random.default_rng(10 + seed)
        Q = np.concatenate([rng.uniform(-2, 2, (600, 3)),
                            V[rng.integers(0, len(V), 50)].astype(np.float64)])   # some on the data
        np.testing.assert_array_equal(O.dmin_tree(osc, trees, Q), O.dmin(osc, Q))
        # one class alone, and an empty class list entry
        only_t = [None, None, trees[2]]
        np.testing.assert_array_equal(O.dmin_tree(O.OracleScene(V, T=T), only_t, Q),
                                      O.dmin(O.OracleScene(V, T=T), Q))
