"""Python binding of libsd (ctypes).  Argument marshalling only: every step of
the computation runs in the HIP kernels behind the C ABI (include/sd.h).

PyTorch supplies device memory and the current HIP stream.  Functions keep the
C names: sd_build_bvh, sd_eval, sd_eval_grad, sd_eval_brute, sd_eval_counters,
sd_export_bvh, sd_export_weights, sd_rigid_transform, sd_rigid_adjoint,
sd_rigid_qmesh_adjoint, sd_query_mesh_lse, sd_eval_grad_prims, sd_sphere_trace, plus
the surrogate entry points in ``surrogate.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsd.so")

SD_BUILD_A_PAPER_LITERAL = 0x1
SD_GRAD_PAPER_METRIC = 0x1
SD_ROOTLOG_F64 = 0x2
SD_NO_QUERY_SORT = 0x4
SD_NO_CONSERVATIVE_ROUNDING = 0x8
SD_NO_PRUNE = 0x10
SD_COUNTERS_BY_CLASS = 0x20
SD_LSE_COMPENSATED_F32 = 0x40

_c_p = ctypes.c_void_p
_i64 = ctypes.c_int64


class SdParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("alpha_u", ctypes.c_float),
                ("beta", ctypes.c_float), ("flags", ctypes.c_uint32)]


class SdSceneInfo(ctypes.Structure):
    _fields_ = [("n_prims", _i64 * 3), ("n_nodes", _i64 * 3), ("A", ctypes.c_double * 3),
                ("A_T_literal", ctypes.c_double), ("diam_max", ctypes.c_double),
                ("device_bytes", _i64), ("n_tri_classes", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class SdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsd error {code}: {msg}")
        self.code = code


_lib = None

EXPORTED = ["sd_build_bvh", "sd_free_scene", "sd_scene_info_get", "sd_eval", "sd_eval_grad",
            "sd_eval_brute", "sd_eval_counters", "sd_export_bvh", "sd_export_weights",
            "sd_query_order", "sd_eval_grad_ordered", "sd_eval_grad_noalloc",
            "sd_triangle_weight_basis", "sd_rigid_transform", "sd_rigid_adjoint", "sd_rigid_qmesh_adjoint", "sd_query_mesh_lse", "sd_sphere_trace", "sd_eval_grad_prims",
            "sd_surrogate_create", "sd_surrogate_free", "sd_surrogate_forward",
            "sd_surrogate_loss_grad", "sd_surrogate_adam", "sd_surrogate_train_step",
            "sd_surrogate_certify", "sd_surrogate_certify_cells", "sd_surrogate_save", "sd_surrogate_load", "sd_eval_surrogate",
            "sd_set_memory_budget", "sd_memory_in_use", "sd_last_error"]


def lib():
    """Load libsd.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_2108_10480_amd.csrc.build)")
        L = ctypes.CDLL(LIB_PATH)
        L.sd_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name != "sd_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SdError(rc, lib().sd_last_error().decode())


def _stream():
    return _c_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, dtype, name, shape_last=None):
    if t is None:
        return _c_p(0), 0
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"{name} must have shape (n, {shape_last})")
    return _c_p(t.data_ptr()), t.shape[0]


class Scene:
    """Owns an sd_scene handle (device hierarchies, leaf records, weights)."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("scene already freed")
        return self._h

    def info(self):
        inf = SdSceneInfo()
        _check(lib().sd_scene_info_get(self.handle, ctypes.byref(inf)))
        return dict(n_prims=list(inf.n_prims), n_nodes=list(inf.n_nodes), A=list(inf.A),
                    A_T_literal=inf.A_T_literal, diam_max=inf.diam_max,
                    device_bytes=inf.device_bytes, n_tri_classes=inf.n_tri_classes)

    def free(self):
        if self._h is not None and _lib is not None:
            lib().sd_free_scene(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sd_build_bvh(V, P=None, E=None, T=None, flags=0, all_points=False):
    """Build the per-class hierarchies for the data mesh (V, P, E, T).
    ``all_points=True`` makes every vertex a point (P must be None)."""
    Vp, nV = _dptr(V, torch.float32, "V", 3)
    Pp, nP = _dptr(P, torch.int32, "P")
    Ep, nE = _dptr(E, torch.int32, "E", 2)
    Tp, nT = _dptr(T, torch.int32, "T", 3)
    if all_points:
        if P is not None:
            raise ValueError("all_points=True needs P=None")
        nP = -1
    h = _c_p()
    _check(lib().sd_build_bvh(Vp, _i64(nV), Pp, _i64(nP), Ep, _i64(nE), Tp, _i64(nT),
                              ctypes.c_uint32(flags), _stream(), ctypes.byref(h)))
    return Scene(h)


def sd_set_memory_budget(nbytes):
    """Budget of the library's device memory in bytes (None or < 0: none)."""
    _check(lib().sd_set_memory_budget(_i64(-1 if nbytes is None else int(nbytes))))


def sd_memory_in_use():
    """Device bytes the library holds now."""
    out = ctypes.c_int64()
    _check(lib().sd_memory_in_use(ctypes.byref(out)))
    return out.value


def params(alpha, beta=0.5, alpha_u=0.0, flags=0):
    return SdParams(float(alpha), float(alpha_u), float(beta), int(flags))


def _queries(Q):
    Qp, n = _dptr(Q, torch.float32, "Q", 3)
    return Qp, n


def sd_eval(scene, Q, alpha, beta=0.5, alpha_u=0.0, flags=0, out=None):
    Qp, n = _queries(Q)
    d = out if out is not None else torch.empty(n, dtype=torch.float32, device=Q.device)
    p = params(alpha, beta, alpha_u, flags)
    _check(lib().sd_eval(scene.handle, Qp, _i64(n), ctypes.byref(p), _c_p(d.data_ptr()), _stream()))
    return d


def sd_eval_grad(scene, Q, alpha, beta=0.5, alpha_u=0.0, flags=0, out=None, grad_out=None):
    Qp, n = _queries(Q)
    d = out if out is not None else torch.empty(n, dtype=torch.float32, device=Q.device)
    g = grad_out if grad_out is not None else torch.empty((n, 3), dtype=torch.float32, device=Q.device)
    p = params(alpha, beta, alpha_u, flags)
    _check(lib().sd_eval_grad(scene.handle, Qp, _i64(n), ctypes.byref(p), _c_p(d.data_ptr()),
                              _c_p(g.data_ptr()), _stream()))
    return d, g


SD_NOALLOC_MAX_QUERIES = 1 << 20


def sd_eval_grad_noalloc(scene, Q, alpha, beta=0.5, alpha_u=0.0, flags=0, out=None, grad_out=None):
    """sd_eval_grad through the entry point that allocates no device memory
    (at most SD_NOALLOC_MAX_QUERIES queries per call).  Pass `out` and
    `grad_out` to keep the call itself free of allocations."""
    Qp, n = _queries(Q)
    d = out if out is not None else torch.empty(n, dtype=torch.float32, device=Q.device)
    g = grad_out if grad_out is not None else torch.empty((n, 3), dtype=torch.float32, device=Q.device)
    p = params(alpha, beta, alpha_u, flags)
    _check(lib().sd_eval_grad_noalloc(scene.handle, Qp, _i64(n), ctypes.byref(p), _c_p(d.data_ptr()),
                                      _c_p(g.data_ptr()), _stream()))
    return d, g


def sd_query_order(scene, Q, out=None):
    """Morton order of the queries (uint32 permutation, stored as int32)."""
    Qp, n = _queries(Q)
    perm = out if out is not None else torch.empty(n, dtype=torch.int32, device=Q.device)
    _check(lib().sd_query_order(scene.handle, Qp, _i64(n), _c_p(perm.data_ptr()), _stream()))
    return perm


def sd_eval_grad_ordered(scene, Q, perm, alpha, beta=0.5, alpha_u=0.0, flags=0, out=None,
                         grad_out=None):
    Qp, n = _queries(Q)
    if perm is not None and (perm.dtype != torch.int32 or perm.numel() != n or not perm.is_cuda):
        raise ValueError("perm must be a CUDA int32 tensor with one entry per query")
    d = out if out is not None else torch.empty(n, dtype=torch.float32, device=Q.device)
    g = grad_out if grad_out is not None else torch.empty((n, 3), dtype=torch.float32, device=Q.device)
    p = params(alpha, beta, alpha_u, flags)
    _check(lib().sd_eval_grad_ordered(scene.handle, Qp, _c_p(perm.data_ptr() if perm is not None else 0),
                                      _i64(n), ctypes.byref(p), _c_p(d.data_ptr()), _c_p(g.data_ptr()),
                                      _stream()))
    return d, g


def sd_eval_brute(scene, Q, alpha, alpha_u=0.0, flags=0, grad=True):
    Qp, n = _queries(Q)
    d = torch.empty(n, dtype=torch.float32, device=Q.device)
    g = torch.empty((n, 3), dtype=torch.float32, device=Q.device) if grad else None
    p = params(alpha, 0.0, alpha_u, flags)
    _check(lib().sd_eval_brute(scene.handle, Qp, _i64(n), ctypes.byref(p), _c_p(d.data_ptr()),
                               _c_p(g.data_ptr() if g is not None else 0), _stream()))
    return (d, g) if grad else d


def sd_eval_counters(scene, Q, alpha, beta=0.5, alpha_u=0.0, flags=0):
    """Per-query (nodes visited, far-field terms, exact leaves); with
    SD_COUNTERS_BY_CLASS the leaves split into points, edges, triangles."""
    Qp, n = _queries(Q)
    k = 5 if flags & SD_COUNTERS_BY_CLASS else 3
    c = torch.empty((n, k), dtype=torch.int32, device=Q.device)
    p = params(alpha, beta, alpha_u, flags)
    _check(lib().sd_eval_counters(scene.handle, Qp, _i64(n), ctypes.byref(p), _c_p(c.data_ptr()),
                                  _stream()))
    return c


def sd_export_bvh(scene, cls):
    """Host copy of one class hierarchy: (box (n,6) f32, left, right, prim) int32."""
    nn = scene.info()["n_nodes"][cls]
    if nn == 0:
        return None
    box = np.empty((nn, 6), np.float32)
    left, right, prim = (np.empty(nn, np.int32) for _ in range(3))
    f = lambda a: _c_p(a.ctypes.data)
    _check(lib().sd_export_bvh(scene.handle, ctypes.c_int(cls), f(box), f(left), f(right), f(prim),
                               _stream()))
    return box, left, right, prim


def sd_export_weights(scene, cls):
    n = scene.info()["n_prims"][cls]
    k = 2 if cls == 1 else 3
    out = np.empty((n, k), np.float32)
    if n:
        _check(lib().sd_export_weights(scene.handle, ctypes.c_int(cls), _c_p(out.ctypes.data), _stream()))
    return out


def sd_triangle_weight_basis():
    out = np.empty((3, 8, 8), np.float64)
    _check(lib().sd_triangle_weight_basis(_c_p(out.ctypes.data)))
    return out


def sd_rigid_transform(X, R, t):
    Xp, m = _dptr(X, torch.float32, "X", 3)
    Rp, K = _dptr(R.reshape(-1, 9), torch.float32, "R", 9)
    tp, K2 = _dptr(t, torch.float32, "t", 3)
    if K2 != K:
        raise ValueError("R and t disagree on the number of transforms")
    Q = torch.empty((K * m, 3), dtype=torch.float32, device=X.device)
    _check(lib().sd_rigid_transform(Xp, _i64(m), Rp, tp, _i64(K), _c_p(Q.data_ptr()), _stream()))
    return Q


def sd_rigid_adjoint(X, R, gbar, grad, want_x=True):
    Xp, m = _dptr(X, torch.float32, "X", 3)
    Rf = R.reshape(-1, 9).contiguous()
    Rp, K = _dptr(Rf, torch.float32, "R", 9)
    gb = gbar.reshape(-1).contiguous()
    gd = grad.reshape(-1, 3).contiguous()
    if gb.numel() != K * m or gd.shape[0] != K * m:
        raise ValueError("gbar / grad must have K*m entries")
    Rbar = torch.empty((K, 9), dtype=torch.float32, device=X.device)
    tbar = torch.empty((K, 3), dtype=torch.float32, device=X.device)
    Xbar = torch.empty((m, 3), dtype=torch.float32, device=X.device) if want_x else None
    _check(lib().sd_rigid_adjoint(Xp, _i64(m), Rp, _i64(K), _c_p(gb.data_ptr()), _c_p(gd.data_ptr()),
                                  _c_p(Rbar.data_ptr()), _c_p(tbar.data_ptr()),
                                  _c_p(Xbar.data_ptr() if Xbar is not None else 0), _stream()))
    return Rbar.reshape(K, 3, 3), tbar, Xbar


def sd_rigid_qmesh_adjoint(X, R, w, Dbar, grad, want_x=True):
    """sd_rigid_adjoint with gbar_kj = w_kj Dbar_k formed in the kernels."""
    Xp, m = _dptr(X, torch.float32, "X", 3)
    Rf = R.reshape(-1, 9).contiguous()
    Rp, K = _dptr(Rf, torch.float32, "R", 9)
    wc = w.reshape(-1).contiguous()
    Db = Dbar.reshape(-1).contiguous()
    _dptr(Db.reshape(-1, 1), torch.float32, "Dbar", 1)
    gd = grad.reshape(-1, 3).contiguous()
    if wc.numel() != K * m or gd.shape[0] != K * m or Db.numel() != K:
        raise ValueError("w / grad must have K*m entries and Dbar K")
    Rbar = torch.empty((K, 9), dtype=torch.float32, device=X.device)
    tbar = torch.empty((K, 3), dtype=torch.float32, device=X.device)
    Xbar = torch.empty((m, 3), dtype=torch.float32, device=X.device) if want_x else None
    _check(lib().sd_rigid_qmesh_adjoint(Xp, _i64(m), Rp, _i64(K), _c_p(wc.data_ptr()), _c_p(Db.data_ptr()),
                                        _c_p(gd.data_ptr()), _c_p(Rbar.data_ptr()), _c_p(tbar.data_ptr()),
                                        _c_p(Xbar.data_ptr() if Xbar is not None else 0), _stream()))
    return Rbar.reshape(K, 3, 3), tbar, Xbar


class RigidSmoothDistance(torch.autograd.Function):
    """d_kj = smooth distance of R_k x_j + t_k, differentiable in (R, t, X) by the
    hand-written adjoint (sd_rigid_adjoint), the forward gradient from
    sd_eval_grad."""

    @staticmethod
    def forward(ctx, X, R, t, scene, alpha, beta, alpha_u, flags):
        Xc, Rc, tc = X.detach().contiguous(), R.detach().contiguous(), t.detach().contiguous()
        Q = sd_rigid_transform(Xc, Rc, tc)
        d, g = sd_eval_grad(scene, Q, alpha, beta, alpha_u, flags)
        ctx.save_for_backward(Xc, Rc, g)
        K, m = Rc.reshape(-1, 9).shape[0], Xc.shape[0]
        return d.reshape(K, m)

    @staticmethod
    def backward(ctx, gbar):
        X, R, g = ctx.saved_tensors
        Rbar, tbar, Xbar = sd_rigid_adjoint(X, R, gbar.contiguous(), g,
                                            want_x=ctx.needs_input_grad[0])
        return (Xbar, Rbar.reshape(R.shape), tbar, None, None, None, None, None)


def rigid_smooth_distance(X, R, t, scene, alpha, beta=0.5, alpha_u=0.0, flags=0):
    return RigidSmoothDistance.apply(X, R, t, scene, alpha, beta, alpha_u, flags)


def sd_eval_grad_prims(scene, G, alpha, beta=0.5, alpha_u=0.0, flags=0):
    """Value and gradient (rigid translation) for query primitives G (n, nv, 3):
    nv = 2 edges, 3 triangles, 1 points (Sec. 3.4)."""
    if not (isinstance(G, torch.Tensor) and G.is_cuda and G.dtype == torch.float32):
        raise TypeError("G must be a float32 CUDA tensor")
    if G.dim() != 3 or G.shape[2] != 3 or not 1 <= G.shape[1] <= 3:
        raise ValueError("G must have shape (n, nv, 3) with nv in 1..3")
    Gc = G.contiguous()
    n, nv = Gc.shape[0], Gc.shape[1]
    p = params(alpha, beta, alpha_u, flags)
    d = torch.empty(n, dtype=torch.float32, device=G.device)
    g = torch.empty((n, 3), dtype=torch.float32, device=G.device)
    _check(lib().sd_eval_grad_prims(scene.handle, _c_p(Gc.data_ptr()), ctypes.c_int32(nv), _i64(n),
                                    ctypes.byref(p), _c_p(d.data_ptr()), _c_p(g.data_ptr()), _stream()))
    return d, g


def sd_sphere_trace(scene, O, U, alpha, beta=0.5, alpha_u=0.0, flags=0, level=0.0, eps=1e-4, t_max=10.0,
                    max_steps=256, want_steps=True):
    """Sphere tracing of the level set d = level along rays (O, U) (n x 3
    each, U unit): (t (n,) with +inf for a miss, steps (n,) int32 or None)."""
    Op, n = _dptr(O, torch.float32, "O", 3)
    Up, n2 = _dptr(U, torch.float32, "U", 3)
    if n2 != n:
        raise ValueError("O and U must have the same number of rays")
    p = params(alpha, beta, alpha_u, flags)
    t = torch.empty(n, dtype=torch.float32, device=O.device)
    st = torch.empty(n, dtype=torch.int32, device=O.device) if want_steps else None
    _check(lib().sd_sphere_trace(scene.handle, Op, Up, _i64(n), ctypes.byref(p), ctypes.c_float(level),
                                 ctypes.c_float(eps), ctypes.c_float(t_max), ctypes.c_int32(max_steps),
                                 _c_p(t.data_ptr()), _c_p(st.data_ptr() if st is not None else 0), _stream()))
    return t, st


def sd_query_mesh_lse(d, grad, alpha_q, prim=None, nV=None, want_w=True, want_vgrad=True):
    """Smooth distance to a query mesh (Sec. 3.6, Eq. 6-8) for K instances:
    d (K, m) per-primitive distances, grad (K, m, 3) their gradients, prim
    (m, 3) int32 vertex ids (-1 unused) or None for a point query mesh.
    Returns (D (K,), w (K, m) or None, vgrad (K, nV, 3) or None)."""
    if d.dim() != 2:
        raise ValueError("d must be K x m")
    K, m = d.shape
    dc = d.contiguous()
    if dc.dtype != torch.float32 or not dc.is_cuda:
        raise ValueError("d must be a float32 CUDA tensor")
    gp = 0
    if want_vgrad:
        gc = grad.reshape(K, m, 3).contiguous()
        if gc.dtype != torch.float32 or not gc.is_cuda:
            raise ValueError("grad must be a float32 CUDA tensor")
        gp = gc.data_ptr()
    pp = 0
    if prim is not None:
        pc = prim.contiguous()
        if pc.dtype != torch.int32 or not pc.is_cuda or pc.shape != (m, 3):
            raise ValueError("prim must be an m x 3 int32 CUDA tensor")
        pp = pc.data_ptr()
        if nV is None:
            raise ValueError("nV is required with prim")
    else:
        nV = m
    D = torch.empty(K, dtype=torch.float32, device=d.device)
    w = torch.empty((K, m), dtype=torch.float32, device=d.device) if want_w else None
    vg = torch.empty((K, nV, 3), dtype=torch.float32, device=d.device) if want_vgrad else None
    _check(lib().sd_query_mesh_lse(_c_p(dc.data_ptr()), _c_p(gp), _i64(K), _i64(m), _c_p(pp), _i64(nV),
                                   ctypes.c_float(alpha_q), _c_p(D.data_ptr()),
                                   _c_p(w.data_ptr() if w is not None else 0),
                                   _c_p(vg.data_ptr() if vg is not None else 0), _stream()))
    return D, w, vg


class RigidQueryMeshDistance(torch.autograd.Function):
    """D_k = smooth distance between the data mesh and the point query mesh
    {R_k x_j + t_k} (Eq. 6 with alpha_q), differentiable in (R, t, X): the
    upstream dL/dD_k times the weights w_kj = dD_k/dd_kj feeds the rigid
    adjoint (sd_rigid_qmesh_adjoint forms that product on the GPU)."""

    @staticmethod
    def forward(ctx, X, R, t, scene, alpha, beta, alpha_u, flags, alpha_q):
        Xc, Rc, tc = X.detach().contiguous(), R.detach().contiguous(), t.detach().contiguous()
        Q = sd_rigid_transform(Xc, Rc, tc)
        d, g = sd_eval_grad(scene, Q, alpha, beta, alpha_u, flags)
        K, m = Rc.reshape(-1, 9).shape[0], Xc.shape[0]
        D, w, _ = sd_query_mesh_lse(d.reshape(K, m), None, alpha_q, want_vgrad=False)
        ctx.save_for_backward(Xc, Rc, g, w)
        return D

    @staticmethod
    def backward(ctx, Dbar):
        X, R, g, w = ctx.saved_tensors
        Rbar, tbar, Xbar = sd_rigid_qmesh_adjoint(X, R, w, Dbar, g, want_x=ctx.needs_input_grad[0])
        return (Xbar, Rbar.reshape(R.shape), tbar, None, None, None, None, None, None)


def rigid_query_mesh_distance(X, R, t, scene, alpha, alpha_q, beta=0.5, alpha_u=0.0, flags=0):
    return RigidQueryMeshDistance.apply(X, R, t, scene, alpha, beta, alpha_u, flags, alpha_q)


def upload_scene(sc, device="cuda", flags=0):
    """Build from a scenes.Scene (numpy arrays)."""
    f = lambda a, dt: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    return sd_build_bvh(f(sc.V, torch.float32), f(sc.P, torch.int32), f(sc.E, torch.int32),
                        f(sc.T, torch.int32), flags=flags)
