"""A plain top-down median-split hierarchy for the oracle's Barnes-Hut pins.

It is written independently of the library's LBVH: the oracle evaluates
Alg. 1 on whatever binary box hierarchy it is given, so the CPU pin tests
build their own trees here.
"""
import numpy as np


def prim_boxes(xyz, k):
    """xyz: (n, 3k) float32 vertex coordinates of each primitive."""
    pts = np.asarray(xyz, np.float32).reshape(len(xyz), k, 3)
    return pts.min(1), pts.max(1)


def median_tree(xyz, k, leaf_order_seed=None):
    lo, hi = prim_boxes(xyz, k)
    n = len(lo)
    if n == 0:
        return None
    cen = 0.5 * (lo.astype(np.float64) + hi)
    box, left, right, prim = [], [], [], []

    def rec(ids):
        me = len(left)
        box.append(np.concatenate([lo[ids].min(0), hi[ids].max(0)]))
        left.append(-1); right.append(-1); prim.append(-1)
        if len(ids) == 1:
            prim[me] = int(ids[0])
            return me
        ext = cen[ids].max(0) - cen[ids].min(0)
        ax = int(np.argmax(ext))
        order = ids[np.argsort(cen[ids, ax], kind="stable")]
        h = len(order) // 2
        l = rec(order[:h])
        r = rec(order[h:])
        left[me], right[me] = l, r
        return me

    rec(np.arange(n))
    return (np.asarray(box, np.float32), np.asarray(left, np.int32),
            np.asarray(right, np.int32), np.asarray(prim, np.int32))
