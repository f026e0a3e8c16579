"""FP64 reference for the smooth distance to a query mesh (Sec. 3.6).

TEST INFRASTRUCTURE ONLY.  Only the tests and the benchmark import this
module; it shares no code with the HIP library and never calls it.

The data-to-query-mesh distance combines per-query-primitive smooth distances
d_j = d(M_d, g_j) with an outer log-sum-exp of sharpness alpha_q (Eq. 6):

    D = -(1/alpha_q) log sum_j exp(-alpha_q d_j),

rewritten by splitting each exponential equally between the n(g_j) + 1
vertices of g_j and summing over vertices and their one-rings (Eq. 7); the
gradient with respect to query vertex q_k collects the split shares of the
primitives around it, each moving its primitive rigidly (Eq. 8):

    dD/dq_k = sum_{g_j in N_k} exp(-alpha_q d_j) / (n(g_j) + 1) grad d_j
              / sum_j exp(-alpha_q d_j).

Both sums are evaluated here as written (with the largest exponential
factored out, which cancels), the value from the vertex form of Eq. 7.
"""
from __future__ import annotations

import numpy as np


def one_rings(prim, nV):
    """N_k: the query primitives incident to each vertex (prim: m x 3 vertex
    ids, -1 for unused corners)."""
    rings = [[] for _ in range(nV)]
    for j, row in enumerate(prim):
        for v in row:
            if v >= 0:
                rings[int(v)].append(j)
    return rings


def point_prims(m):
    """Primitive j is query vertex j (a point query mesh)."""
    p = -np.ones((m, 3), np.int64)
    p[:, 0] = np.arange(m)
    return p


def query_mesh_lse(d, grad, alpha_q, prim=None, nV=None):
    """Eq. 6-8 for K instances of one query mesh.

    d: K x m per-primitive smooth distances, grad: K x m x 3 their gradients,
    prim: m x 3 vertex ids (-1 unused) or None for points (nV = m).
    Returns (D (K,), w (K, m) = dD/dd_kj, vgrad (K, nV, 3)).
    An instance with every d = +inf gives D = +inf, w = 0, vgrad = 0."""
    d = np.asarray(d, np.float64)
    grad = np.asarray(grad, np.float64)
    K, m = d.shape
    if prim is None:
        prim = point_prims(m)
        nV = m
    prim = np.asarray(prim, np.int64)
    size = (prim >= 0).sum(1)                       # n(g_j) + 1
    rings = one_rings(prim, nV)
    D = np.empty(K)
    w = np.zeros((K, m))
    vgrad = np.zeros((K, nV, 3))
    for k in range(K):
        dk = d[k]
        if m == 0 or np.all(np.isposinf(dk)):
            D[k] = np.inf
            continue
        if np.any(np.isnan(dk)):
            D[k] = np.nan
            w[k] = np.nan
            vgrad[k] = np.nan
            continue
        dm = dk.min()
        e = np.exp(-alpha_q * (dk - dm))             # exp(-alpha_q d_j) / exp(-alpha_q d_min)
        # Eq. 7: sum over vertices of the split shares of their one-rings
        s7 = 0.0
        for v in range(nV):
            for j in rings[v]:
                s7 += e[j] / size[j]
        D[k] = dm - np.log(s7) / alpha_q
        # Eq. 8: denominator is the plain sum of Eq. 6
        s6 = e.sum()
        w[k] = e / s6
        for v in range(nV):
            acc = np.zeros(3)
            for j in rings[v]:
                acc += e[j] / size[j] * grad[k, j]
            vgrad[k, v] = acc / s6
    return D, w, vgrad
