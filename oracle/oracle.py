"""FP64 reference ("oracle") for the smooth distance — Python side.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg import this module.  It shares no code with the
HIP library and never calls it: everything here is numpy (FP64) plus the
plain C routines in ``sd_oracle.c`` (loaded with ctypes).

What lives here (each function cites the passage it follows):

* valences per primitive class .................. App. C.1, App. C.2, App. C.3
* edge weight polynomial (5x5 solve) ............ App. C.2
* triangle weight polynomial (pseudoinverse) .... App. C.3
* global weight scale A per class ............... Sec. 3.3, App. C.2, App. C.3
* brute-force and Barnes-Hut evaluation ......... Eq. 3, Eq. 4, Alg. 1, Alg. 2
  (in C, see sd_oracle.c); edges and triangles as query primitives (Sec. 3.4)
  with the simplex-simplex distances of App. B
* the surrogate network in FP64 (forward, backward, input gradient, Adam):
  see ``mlp.py``

Readings of ambiguous passages:
* App. C.2's derivative constraints are read as w'(0) = w'(1) = 0.
* App. C.3's "A = max_i v_i" is strengthened to A_T = max(max_i v_i,
  max_i 1/min w~_i) so that A w~_i >= 1 holds everywhere as Sec. 3.3 requires
  ("strict"); ``a_literal=True`` gives the printed max_i v_i.
* A triangle whose largest vertex valence is 1 (an isolated triangle) uses
  w~ = 1: the App. C.3 construction has no meaningful solution there.
* Valences are counted within each primitive class.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile sd_oracle.c with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               _SRC, "-o", _LIB, "-lm"])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


# --------------------------------------------------------------------------
# ctypes structures (mirror sd_oracle.c)
# --------------------------------------------------------------------------
_P = ctypes.c_void_p


class _OrScene(ctypes.Structure):
    _fields_ = [("nP", ctypes.c_int64), ("P", _P),
                ("nE", ctypes.c_int64), ("E", _P), ("Ecls", _P), ("Ecoef", _P),
                ("nT", ctypes.c_int64), ("T", _P), ("Tcls", _P), ("Tcoef", _P),
                ("logA_E", ctypes.c_double), ("logA_T", ctypes.c_double)]


class _OrParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("alpha_u", ctypes.c_double),
                ("beta", ctypes.c_double), ("metric_r2", ctypes.c_int32),
                ("cut_f32", ctypes.c_int32)]


class _OrTree(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("box", _P), ("left", _P),
                ("right", _P), ("prim", _P)]


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0)


# --------------------------------------------------------------------------
# App. C.2: edge weights
# --------------------------------------------------------------------------
def edge_weight_coeffs(n0, n1):
    """Quartic w~(phi) = sum_k c_k phi^k with w~(0) = 1/N_i0, w~(1) = 1/N_i1,
    w~(1/2) = 1 and zero slope at phi = 0 and phi = 1 (App. C.2)."""
    M = np.array([[1, 0, 0, 0, 0],
                  [1, 1, 1, 1, 1],
                  [1, .5, .25, .125, .0625],
                  [0, 1, 0, 0, 0],
                  [0, 1, 2, 3, 4]], dtype=np.float64)
    r = np.array([1.0 / n0, 1.0 / n1, 1.0, 0.0, 0.0])
    return np.linalg.solve(M, r)


# --------------------------------------------------------------------------
# App. C.3: triangle weights
# --------------------------------------------------------------------------
TRI_MONOMIALS = [(a, b) for a in range(8) for b in range(8 - a)]   # 36 monomials phi1^a phi2^b

TRI_POINTS_VERTEX = [(0, 0), (1, 0), (0, 1)]
TRI_POINTS_EDGE = [(1 / 3, 0), (2 / 3, 0), (1 / 3, 2 / 3), (2 / 3, 1 / 3), (0, 1 / 3), (0, 2 / 3)]
TRI_POINT_CENTER = (1 / 3, 1 / 3)


def _poly_compose_line(a, b, x0, x1, y0, y1):
    """Coefficients (in t) of x^a y^b along x = x0 + x1 t, y = y0 + y1 t."""
    px = np.polynomial.polynomial.polypow([x0, x1], a) if a else np.array([1.0])
    py = np.polynomial.polynomial.polypow([y0, y1], b) if b else np.array([1.0])
    return np.polynomial.polynomial.polymul(px, py)


def triangle_constraint_matrix():
    """The linear system of App. C.3: 10 point constraints, then the
    coefficient rows of the four normal-derivative identities (7 each; the
    duplicated rows the paper mentions are kept, which leaves the
    minimum-norm solution unchanged)."""
    rows = []
    pts = TRI_POINTS_VERTEX + TRI_POINTS_EDGE + [TRI_POINT_CENTER]
    for (x, y) in pts:
        rows.append([x ** a * y ** b for (a, b) in TRI_MONOMIALS])

    def deriv_rows(kind):
        out = np.zeros((7, len(TRI_MONOMIALS)))
        for j, (a, b) in enumerate(TRI_MONOMIALS):
            # derivative monomials: d/dx x^a y^b = a x^(a-1) y^b, d/dy = b x^a y^(b-1)
            terms = []
            if kind in ("dx_on_x0", "sum_on_diag", "sum_on_diag_rev") and a > 0:
                terms.append((a, a - 1, b))
            if kind in ("dy_on_y0", "sum_on_diag", "sum_on_diag_rev") and b > 0:
                terms.append((b, a, b - 1))
            for (k, aa, bb) in terms:
                if kind == "dx_on_x0":          # line (0, t)
                    c = _poly_compose_line(aa, bb, 0, 0, 0, 1)
                elif kind == "dy_on_y0":        # line (t, 0)
                    c = _poly_compose_line(aa, bb, 0, 1, 0, 0)
                elif kind == "sum_on_diag":     # line (t, 1 - t)
                    c = _poly_compose_line(aa, bb, 0, 1, 1, -1)
                else:                           # line (1 - t, t)
                    c = _poly_compose_line(aa, bb, 1, -1, 0, 1)
                c = np.asarray(c, dtype=np.float64)
                out[:len(c), j] += k * c[:7]
        return out

    for kind in ("dx_on_x0", "dy_on_y0", "sum_on_diag", "sum_on_diag_rev"):
        rows.extend(deriv_rows(kind))
    return np.array(rows, dtype=np.float64)


def triangle_rhs(v, e):
    return np.array([1.0 / v] * 3 + [1.0 / e] * 6 + [(v - 1.0) / v] + [0.0] * 28)


_TRI_PINV = None


def triangle_weight_coeffs(v, e):
    """36 monomial coefficients of w~ for max vertex valence v and max edge
    valence e, as the pseudoinverse solution of App. C.3 (monomial basis,
    unscaled columns).  Returned as an (8, 8) table, entry [a, b] multiplying
    phi1^a phi2^b.  v == 1 (isolated triangle) gives the constant 1."""
    global _TRI_PINV
    out = np.zeros((8, 8))
    if v <= 1:
        out[0, 0] = 1.0
        return out
    if _TRI_PINV is None:
        _TRI_PINV = np.linalg.pinv(triangle_constraint_matrix(), rcond=1e-12)
    c = _TRI_PINV @ triangle_rhs(float(v), float(e))
    for j, (a, b) in enumerate(TRI_MONOMIALS):
        out[a, b] = c[j]
    return out


def eval_poly2(C, x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    v = np.zeros(np.broadcast(x, y).shape)
    for a in range(8):
        for b in range(8 - a):
            if C[a, b] != 0.0:
                v = v + C[a, b] * x ** a * y ** b
    return v


def triangle_weight_min(C, n_grid=400):
    """Minimum of w~ over the barycentric triangle: dense grid, then a bounded
    local refinement from the best grid points (scipy, FP64)."""
    from scipy.optimize import minimize
    g = np.linspace(0.0, 1.0, n_grid + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    m = X + Y <= 1.0 + 1e-15
    xs, ys = X[m], Y[m]
    vals = eval_poly2(C, xs, ys)
    order = np.argsort(vals)[:8]
    best = vals[order[0]]

    def f(z):
        x, y = z
        # penalised projection onto the simplex keeps the search feasible
        x, y = max(x, 0.0), max(y, 0.0)
        s = x + y
        if s > 1.0:
            x, y = x / s, y / s
        return float(eval_poly2(C, x, y))

    for i in order:
        r = minimize(f, [xs[i], ys[i]], method="Nelder-Mead",
                     options=dict(xatol=1e-13, fatol=1e-15, maxiter=4000))
        best = min(best, r.fun)
    # one-dimensional refinement along the three boundary lines
    from scipy.optimize import minimize_scalar
    for line in ((lambda t: (t, 0.0)), (lambda t: (0.0, t)), (lambda t: (1 - t, t))):
        tt = np.linspace(0, 1, 4001)
        vv = np.array([eval_poly2(C, *line(t)) for t in tt])
        k = int(np.argmin(vv))
        lo, hi = tt[max(k - 1, 0)], tt[min(k + 1, len(tt) - 1)]
        r = minimize_scalar(lambda t: float(eval_poly2(C, *line(t))), bounds=(lo, hi),
                            method="bounded", options=dict(xatol=1e-14))
        best = min(best, r.fun, vv[k])
    return float(best)


# --------------------------------------------------------------------------
# Valences (App. C.1-C.3), counted within each class
# --------------------------------------------------------------------------
def edge_valences(E, nV):
    N = np.bincount(E.reshape(-1), minlength=nV)
    return N[E[:, 0]], N[E[:, 1]], int(N.max()) if len(E) else 1


def triangle_valences(T, nV):
    Nv = np.bincount(T.reshape(-1), minlength=nV)
    v = Nv[T].max(axis=1)
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    e = np.sort(e, axis=1)
    _, inv, cnt = np.unique(e, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    ev = cnt[inv].reshape(3, len(T)).T.max(axis=1)
    return v.astype(np.int64), ev.astype(np.int64)


# --------------------------------------------------------------------------
# Oracle scene
# --------------------------------------------------------------------------
class OracleScene:
    """The data mesh M_d split into its point, edge and triangle primitives,
    with per-class weights.  Arrays are FP32 (promoted to FP64 in C)."""

    def __init__(self, V, P=None, E=None, T=None, a_literal=False):
        V = np.ascontiguousarray(V, np.float32)
        self.V = V
        nV = len(V)
        if P is None:
            self.Pxyz = np.zeros((0, 3), np.float32)
        else:
            self.Pxyz = np.ascontiguousarray(V[np.asarray(P)], np.float32)
        # edges
        if E is None or len(E) == 0:
            self.Exyz = np.zeros((0, 6), np.float32)
            self.Ecls = np.zeros(0, np.int32)
            self.Ecoef = np.zeros((1, 5))
            self.A_E = 1.0
        else:
            E = np.asarray(E, np.int64)
            self.Exyz = np.ascontiguousarray(V[E].reshape(-1, 6), np.float32)
            n0, n1, amax = edge_valences(E, nV)
            keys, cls = np.unique(np.stack([n0, n1], 1), axis=0, return_inverse=True)
            self.Ecls = np.ascontiguousarray(cls.reshape(-1), np.int32)
            self.Ecoef = np.ascontiguousarray([edge_weight_coeffs(a, b) for a, b in keys])
            self.A_E = float(amax)            # App. C.2: A = max_k |N_k|
        # triangles
        if T is None or len(T) == 0:
            self.Txyz = np.zeros((0, 9), np.float32)
            self.Tcls = np.zeros(0, np.int32)
            self.Tcoef = np.zeros((1, 8, 8))
            self.A_T = 1.0
            self.A_T_literal = 1.0
            self.tri_classes = []
        else:
            T = np.asarray(T, np.int64)
            self.Txyz = np.ascontiguousarray(V[T].reshape(-1, 9), np.float32)
            v, e = triangle_valences(T, nV)
            keys, cls = np.unique(np.stack([v, e], 1), axis=0, return_inverse=True)
            self.Tcls = np.ascontiguousarray(cls.reshape(-1), np.int32)
            coefs, A = [], float(v.max())
            self.tri_classes = []
            for (vv, ee) in keys:
                C = triangle_weight_coeffs(int(vv), int(ee))
                coefs.append(C)
                wmin = triangle_weight_min(C) if vv > 1 else 1.0
                if wmin <= 0:
                    raise ValueError(f"triangle weight not positive for valences {(vv, ee)}")
                self.tri_classes.append((int(vv), int(ee), wmin))
                A = max(A, 1.0 / wmin)
            self.Tcoef = np.ascontiguousarray(coefs)
            self.A_T_literal = float(v.max())
            self.A_T = self.A_T_literal if a_literal else A
        self._keep = []

    @property
    def n_prims(self):
        return len(self.Pxyz) + len(self.Exyz) + len(self.Txyz)

    def _struct(self):
        s = _OrScene()
        s.nP, s.P = len(self.Pxyz), _ptr(self.Pxyz)
        s.nE, s.E, s.Ecls, s.Ecoef = len(self.Exyz), _ptr(self.Exyz), _ptr(self.Ecls), _ptr(self.Ecoef)
        s.nT, s.T, s.Tcls, s.Tcoef = len(self.Txyz), _ptr(self.Txyz), _ptr(self.Tcls), _ptr(self.Tcoef)
        s.logA_E, s.logA_T = np.log(self.A_E), np.log(self.A_T)
        return s


def _params(alpha, alpha_u=0.0, beta=0.0, metric_r2=False, cut_f32=False):
    p = _OrParams()
    p.alpha, p.alpha_u, p.beta, p.metric_r2, p.cut_f32 = alpha, alpha_u, beta, int(metric_r2), int(cut_f32)
    return p


def brute(scene: OracleScene, Q, alpha, alpha_u=0.0, metric_r2=False):
    """Eq. 3 and Eq. 4 summed over every primitive.  Returns (d, grad, d_min)."""
    Q = np.ascontiguousarray(Q, np.float64)
    n = len(Q)
    d, g, dm = np.empty(n), np.empty((n, 3)), np.empty(n)
    s, p = scene._struct(), _params(alpha, alpha_u, 0.0, metric_r2)
    rc = lib().or_brute(ctypes.byref(s), ctypes.byref(p), ctypes.c_int64(n), _ptr(Q),
                        _ptr(d), _ptr(g), _ptr(dm))
    if rc != 0:
        raise ValueError("oracle brute: bad parameters")
    return d, g, dm


def dmin(scene: OracleScene, Q):
    """Eq. 2: exact minimum distance over all primitives."""
    Q = np.ascontiguousarray(Q, np.float64)
    out = np.empty(len(Q))
    s = scene._struct()
    lib().or_dmin(ctypes.byref(s), ctypes.c_int64(len(Q)), _ptr(Q), _ptr(out))
    return out


def dmin_tree(scene: OracleScene, trees, Q):
    """Eq. 2 by branch and bound over hierarchies whose boxes contain their
    primitives (``trees`` as for barnes_hut): equal to ``dmin``, at a cost
    that allows every query of a large workload to be checked."""
    Q = np.ascontiguousarray(Q, np.float64)
    out = np.empty(len(Q))
    s = scene._struct()
    ts = (_OrTree * 3)()
    for c in range(3):
        if trees[c] is None:
            ts[c].n_nodes = 0
        else:
            ts[c] = trees[c]._struct()
    lib().or_dmin_tree(ctypes.byref(s), ts, ctypes.c_int64(len(Q)), _ptr(Q), _ptr(out))
    return out


def closest(cls, prim, q):
    """Closest point of one primitive (0 point, 1 segment, 2 triangle) to q.
    Returns dict(d, c, phi, dphi, region)."""
    prim = np.ascontiguousarray(prim, np.float32).reshape(-1)
    q = np.ascontiguousarray(q, np.float64).reshape(3)
    o = np.empty(13)
    lib().or_closest(ctypes.c_int(cls), _ptr(prim), _ptr(q), _ptr(o))
    return dict(d=o[0], c=o[1:4], phi=o[4:6], dphi=o[6:12].reshape(2, 3), region=int(o[12]))


class OracleTree:
    """A hierarchy given as explicit children (left/right = -1 at leaves) with
    float32 boxes, over the primitives of one class (``prim`` = primitive id)."""

    def __init__(self, box, left, right, prim):
        self.box = np.ascontiguousarray(box, np.float32).reshape(-1, 6)
        self.left = np.ascontiguousarray(left, np.int32)
        self.right = np.ascontiguousarray(right, np.int32)
        self.prim = np.ascontiguousarray(prim, np.int32)

    def _struct(self):
        t = _OrTree()
        t.n_nodes = len(self.left)
        t.box, t.left, t.right, t.prim = (_ptr(self.box), _ptr(self.left),
                                          _ptr(self.right), _ptr(self.prim))
        return t


def barnes_hut(scene: OracleScene, trees, Q, alpha, beta, alpha_u=0.0, metric_r2=False, cut_f32=False):
    """Alg. 1 + Alg. 2 with the conservative far field of App. D on given
    hierarchies (``trees`` = [points, edges, triangles], None for an empty
    class).  Returns (d, grad, stats) with stats[:, 0] the smallest relative
    opening-criterion margin |beta D - |B|| / D met by each query and
    stats[:, 1:4] = nodes visited, far-field terms, exact leaves.

    ``cut_f32``: take the open/accept decision |B| < beta D (Sec. 3.5) in
    FP32 on squared lengths, as a single-precision evaluator takes it, so that
    both pick the same terms; the terms themselves stay FP64.  Queries should
    then be FP32 values (they are rounded to FP32 for the decision)."""
    Q = np.ascontiguousarray(Q, np.float64)
    n = len(Q)
    arr = (_OrTree * 3)()
    for c in range(3):
        if trees[c] is None:
            arr[c].n_nodes = 0
        else:
            arr[c] = trees[c]._struct()
    d, g, st = np.empty(n), np.empty((n, 3)), np.empty((n, 4))
    s, p = scene._struct(), _params(alpha, alpha_u, beta, metric_r2, cut_f32)
    rc = lib().or_barnes_hut(ctypes.byref(s), ctypes.byref(p), arr, ctypes.c_int64(n), _ptr(Q),
                             _ptr(d), _ptr(g), _ptr(st))
    if rc != 0:
        raise ValueError("oracle barnes_hut: bad parameters")
    return d, g, st


def _prims(G):
    G = np.ascontiguousarray(G, np.float64)
    if G.ndim != 3 or G.shape[2] != 3 or not 1 <= G.shape[1] <= 3:
        raise ValueError("query primitives must be (n, nv, 3) with nv in 1..3")
    return G, G.shape[0], G.shape[1]


def brute_prims(scene: OracleScene, G, alpha, alpha_u=0.0, metric_r2=False):
    """Eq. 3 and Eq. 4 over every primitive for query primitives G (n, nv, 3):
    nv = 1 points, 2 edges, 3 triangles (Sec. 3.4).  Returns (d, grad, d_min)."""
    G, n, nv = _prims(G)
    d, g, dm = np.empty(n), np.empty((n, 3)), np.empty(n)
    s, p = scene._struct(), _params(alpha, alpha_u, 0.0, metric_r2)
    rc = lib().or_brute_prims(ctypes.byref(s), ctypes.byref(p), ctypes.c_int64(n), _ptr(G), ctypes.c_int(nv),
                              _ptr(d), _ptr(g), _ptr(dm))
    if rc != 0:
        raise ValueError("oracle brute_prims: bad parameters")
    return d, g, dm


def barnes_hut_prims(scene: OracleScene, trees, G, alpha, beta, alpha_u=0.0, metric_r2=False, cut_f32=False):
    """Alg. 1 + Alg. 2 for query primitives G (n, nv, 3) with the box distance
    from the per-axis gaps of the halfspaces g lies outside of (App. D for
    general primitives); stats as in barnes_hut."""
    G, n, nv = _prims(G)
    arr = (_OrTree * 3)()
    for c in range(3):
        if trees[c] is None:
            arr[c].n_nodes = 0
        else:
            arr[c] = trees[c]._struct()
    d, g, st = np.empty(n), np.empty((n, 3)), np.empty((n, 4))
    s, p = scene._struct(), _params(alpha, alpha_u, beta, metric_r2, cut_f32)
    rc = lib().or_barnes_hut_prims(ctypes.byref(s), ctypes.byref(p), arr, ctypes.c_int64(n), _ptr(G),
                                   ctypes.c_int(nv), _ptr(d), _ptr(g), _ptr(st))
    if rc != 0:
        raise ValueError("oracle barnes_hut_prims: bad parameters")
    return d, g, st


def simplex_distance(A, B):
    """Distance between two simplices (1-3 vertices each, rows xyz) and the
    closest point on B (App. B, Eq. 10)."""
    A = np.ascontiguousarray(A, np.float64).reshape(-1, 3)
    B = np.ascontiguousarray(B, np.float64).reshape(-1, 3)
    out = np.empty(4)
    lib().or_simplex_distance(_ptr(A), ctypes.c_int(len(A)), _ptr(B), ctypes.c_int(len(B)), _ptr(out))
    return out[0], out[1:]


def rigid_apply(X, R, t):
    X = np.ascontiguousarray(X, np.float32)
    R = np.ascontiguousarray(R, np.float32).reshape(-1, 9)
    t = np.ascontiguousarray(t, np.float32).reshape(-1, 3)
    K, m = len(R), len(X)
    out = np.empty((K * m, 3))
    lib().or_rigid_apply(_ptr(X), ctypes.c_int64(m), _ptr(R), _ptr(t), ctypes.c_int64(K), _ptr(out))
    return out


def rigid_adjoint(X, R, gbar, grad):
    """tbar_k = sum_j u_kj, Rbar_k = sum_j u_kj x_j^T, xbar_j = sum_k R_k^T u_kj
    with u_kj = gbar_kj grad d(R_k x_j + t_k)."""
    X = np.ascontiguousarray(X, np.float32)
    R = np.ascontiguousarray(R, np.float32).reshape(-1, 9)
    K, m = len(R), len(X)
    gbar = np.ascontiguousarray(gbar, np.float64).reshape(K * m)
    grad = np.ascontiguousarray(grad, np.float64).reshape(K * m, 3)
    Rb, tb, Xb = np.empty((K, 9)), np.empty((K, 3)), np.empty((m, 3))
    lib().or_rigid_adjoint(_ptr(X), ctypes.c_int64(m), _ptr(R), ctypes.c_int64(K),
                           _ptr(gbar), _ptr(grad), _ptr(Rb), _ptr(tb), _ptr(Xb))
    return Rb.reshape(K, 3, 3), tb, Xb


# --------------------------------------------------------------------------
# Error measures used by the parity tests
# --------------------------------------------------------------------------
def value_error(d, d_ref, floor):
    """|d - d_ref| / max(|d_ref|, floor): the relative error of the value,
    with an absolute floor (1e-3 of the scene diagonal in the tests) where the
    reference crosses zero, i.e. near the zero isosurface and on the data."""
    den = np.maximum(np.abs(d_ref), floor)
    return np.abs(np.asarray(d, np.float64) - d_ref) / den


def grad_error(g, g_ref, floor=1e-2):
    g = np.asarray(g, np.float64)
    return np.linalg.norm(g - g_ref, axis=1) / np.maximum(np.linalg.norm(g_ref, axis=1), floor)
