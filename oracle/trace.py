"""FP64 reference sphere tracer (Sec. 4.2; Hart 1996) over any distance.

TEST INFRASTRUCTURE ONLY: used by the tests to check the library's tracer.

Per ray: x = o + t u from t = 0, step r = d(x) - level until r <= eps (hit
at t) or t > t_max or max_steps evaluations (miss, +inf).  ``dist`` maps an
(n, 3) array of points to their distances (e.g. the oracle's Barnes-Hut or
exact evaluation); all rays advance together, finished rays drop out.
"""
from __future__ import annotations

import numpy as np


def sphere_trace(dist, O, U, level=0.0, eps=1e-4, t_max=10.0, max_steps=256):
    O = np.asarray(O, np.float64)
    U = np.asarray(U, np.float64)
    n = len(O)
    t = np.zeros(n)
    hit = np.full(n, np.inf)
    steps = np.zeros(n, np.int64)
    live = np.ones(n, bool)
    while live.any():
        idx = np.nonzero(live)[0]
        r = dist(O[idx] + t[idx, None] * U[idx]) - level
        steps[idx] += 1
        done = r <= eps
        hit[idx[done]] = t[idx[done]]
        live[idx[done]] = False
        go = idx[~done]
        t[go] += r[~done]
        stop = ~(t[go] <= t_max) | (steps[go] >= max_steps)
        live[go[stop]] = False
    return hit, steps
