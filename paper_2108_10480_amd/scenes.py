"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only builds geometry and query sets: vertices, primitive index
tuples, query points.  It holds none of the smooth-distance arithmetic (no
distances, weights, log-sum-exp or hierarchy), so both the HIP path and the
FP64 reference read identical FP32 arrays produced here.

The paper's own data (Thingi10K meshes, the Stanford bunny, Toronto-3D street
lidar, OpenTopography terrain) is not available, so every scene below is a
synthetic stand-in with the shapes and sizes of the paper's workloads
(Sec. 4.4 benchmark, Table 1 lidar scenes).

All arrays are numpy: vertices ``V`` float32 (n, 3); point ids ``P`` int32
(n,), edges ``E`` int32 (n, 2), triangles ``T`` int32 (n, 3); queries ``Q``
float32 (n, 3).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Scene:
    V: np.ndarray                      # (nV, 3) float32
    P: np.ndarray | None = None        # (nP,) int32 vertex ids used as points
    E: np.ndarray | None = None        # (nE, 2) int32
    T: np.ndarray | None = None        # (nT, 3) int32
    name: str = ""

    def counts(self):
        return (0 if self.P is None else len(self.P),
                0 if self.E is None else len(self.E),
                0 if self.T is None else len(self.T))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


# --------------------------------------------------------------------------
# basic shapes
# --------------------------------------------------------------------------
_PHI = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = np.array([
    [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
    [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
    [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1]], dtype=np.float64)
_ICO_F = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)


def icosphere(level: int):
    """Unit icosphere after ``level`` midpoint subdivisions (float64 V, int64 F).

    V = 10*4^level + 2, F = 20*4^level, E = 30*4^level.
    """
    V = _ICO_V / np.linalg.norm(_ICO_V, axis=1, keepdims=True)
    F = _ICO_F.copy()
    for _ in range(level):
        nV, nF = len(V), len(F)
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
        es = np.sort(e, axis=1)
        uniq, inv = np.unique(es, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = 0.5 * (V[uniq[:, 0]] + V[uniq[:, 1]])
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        m = inv.reshape(3, nF).T + nV          # midpoints of (01, 12, 20)
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        m01, m12, m20 = m[:, 0], m[:, 1], m[:, 2]
        F = np.concatenate([
            np.stack([a, m01, m20], 1), np.stack([m01, b, m12], 1),
            np.stack([m20, m12, c], 1), np.stack([m01, m12, m20], 1)])
        V = np.concatenate([V, mid])
    return V, F


def torus_grid(nu: int, nv: int, R: float, r: float):
    """Closed torus triangulated on an nu x nv grid (every vertex has valence 6)."""
    u = 2 * np.pi * np.arange(nu) / nu
    v = 2 * np.pi * np.arange(nv) / nv
    uu, vv = np.meshgrid(u, v, indexing="ij")
    X = np.stack([(R + r * np.cos(vv)) * np.cos(uu),
                  (R + r * np.cos(vv)) * np.sin(uu),
                  r * np.sin(vv)], -1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i, j = i.reshape(-1), j.reshape(-1)
    a = i * nv + j
    b = ((i + 1) % nu) * nv + j
    c = ((i + 1) % nu) * nv + (j + 1) % nv
    d = i * nv + (j + 1) % nv
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return X, F


def grid_edges_of(F):
    """Unique undirected edges of a triangle list, sorted (helper for edge scenes)."""
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    return np.unique(np.sort(e, axis=1), axis=0)


# --------------------------------------------------------------------------
# point sphere (point-cloud workload, 2,000 points)
# --------------------------------------------------------------------------
def point_sphere(n_points=2000, n_queries=10000, seed_data=0, seed_query=1):
    rng = np.random.default_rng(seed_data)
    d = rng.standard_normal((n_points, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = 1.0 + rng.normal(0.0, 0.005, n_points)
    V = _f32(d * rad[:, None])
    Q = _f32(np.random.default_rng(seed_query).uniform(-1.5, 1.5, (n_queries, 3)))
    return Scene(V=V, P=_i32(np.arange(n_points)), name="point_sphere"), Q


# --------------------------------------------------------------------------
# bumpy icosphere (triangle-mesh workload: level 7 = 327,680 triangles)
# --------------------------------------------------------------------------
def bumpy_icosphere(level=7, seed=2):
    V, F = icosphere(level)
    rng = np.random.default_rng(seed)
    dirs = rng.standard_normal((8, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    k = rng.uniform(1.0, 6.0, 8)
    ph = rng.uniform(0.0, 2 * np.pi, 8)
    r = 1.0 + 0.05 * np.sin(V @ dirs.T * k + ph).sum(1)
    V = V * r[:, None]
    return Scene(V=_f32(V), T=_i32(F), name=f"bumpy_icosphere_l{level}")


def triangle_areas_normals(V, T):
    """Float64 areas and unit normals of the triangles (sampling helper)."""
    V = V.astype(np.float64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, c - a)
    ln = np.linalg.norm(n, axis=1)
    return 0.5 * ln, n / np.maximum(ln, 1e-300)[:, None]


def surface_samples(V, T, n, rng, offset_lo, offset_hi):
    """Area-weighted uniform points on the triangles, moved along the face
    normal by U[offset_lo, offset_hi]."""
    area, nrm = triangle_areas_normals(V, T)
    cdf = np.cumsum(area)
    cdf /= cdf[-1]
    tri = np.minimum(np.searchsorted(cdf, rng.random(n)), len(T) - 1)
    r1, r2 = rng.random(n), rng.random(n)
    flip = r1 + r2 > 1.0
    r1[flip], r2[flip] = 1.0 - r1[flip], 1.0 - r2[flip]
    Vd = V.astype(np.float64)
    a, b, c = Vd[T[tri, 0]], Vd[T[tri, 1]], Vd[T[tri, 2]]
    p = a + r1[:, None] * (b - a) + r2[:, None] * (c - a)
    off = rng.uniform(offset_lo, offset_hi, n)
    return p + off[:, None] * nrm[tri]


def icosphere_queries(scene, n_queries=1_000_000, seed_box=3, seed_surf=4, box=1.5,
                      band=0.02):
    """Half uniform in [-box, box]^3, half within +-band of the surface."""
    n_box = n_queries // 2
    n_surf = n_queries - n_box
    qb = np.random.default_rng(seed_box).uniform(-box, box, (n_box, 3))
    qs = surface_samples(scene.V, scene.T, n_surf, np.random.default_rng(seed_surf),
                         -band, band)
    return _f32(np.concatenate([qb, qs]))


# --------------------------------------------------------------------------
# small random scenes for unit tests
# --------------------------------------------------------------------------
def random_points(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    V = _f32(rng.uniform(-scale, scale, (n, 3)))
    return Scene(V=V, P=_i32(np.arange(n)), name=f"rand_points_{n}")


def random_polyline(n_seg, seed, closed=False, step=0.3):
    """A random-walk polyline (interior vertices have edge valence 2)."""
    rng = np.random.default_rng(seed)
    steps = rng.normal(0.0, step, (n_seg + 1, 3))
    V = np.cumsum(steps, axis=0)
    nv = n_seg if closed else n_seg + 1
    V = V[:nv]
    E = np.stack([np.arange(n_seg), (np.arange(n_seg) + 1) % nv], 1)
    return Scene(V=_f32(V), E=_i32(E), name=f"polyline_{n_seg}")


def uniform_queries(n, seed, lo, hi):
    return _f32(np.random.default_rng(seed).uniform(lo, hi, (n, 3)))


def scene_aabb(scene):
    V = scene.V
    used = []
    if scene.P is not None:
        used.append(V[scene.P])
    if scene.E is not None:
        used.append(V[scene.E.reshape(-1)])
    if scene.T is not None:
        used.append(V[scene.T.reshape(-1)])
    X = np.concatenate(used) if used else np.zeros((1, 3), np.float32)
    return X.min(0).astype(np.float64), X.max(0).astype(np.float64)


# --------------------------------------------------------------------------
# inputs of the learned surrogate: frequencies, initial weights, sample sets
# --------------------------------------------------------------------------
SURR_N_FREQ = 64
SURR_WIDTH = 256
SURR_DEPTH = 4


def surrogate_param_shapes():
    """Flat parameter order of the surrogate network: W1 (256x128), b1,
    W2..W4 (256x256) with their biases, w5 (256), b5 (1); matrices are
    out x in, row-major."""
    shapes = [(SURR_WIDTH, 2 * SURR_N_FREQ), (SURR_WIDTH,)]
    for _ in range(SURR_DEPTH - 1):
        shapes += [(SURR_WIDTH, SURR_WIDTH), (SURR_WIDTH,)]
    return shapes + [(SURR_WIDTH,), (1,)]


def fourier_matrix(seed=11, sigma=2.0, n_freq=SURR_N_FREQ):
    """Random Fourier frequencies B ~ N(0, sigma^2), n_freq x 3, float32.
    sigma may be a sequence: equal groups of rows use each scale."""
    rng = np.random.default_rng(seed)
    sig = np.repeat(np.atleast_1d(np.asarray(sigma, np.float64)), -(-n_freq // np.size(sigma)))[:n_freq]
    return _f32(rng.normal(0.0, 1.0, (n_freq, 3)) * sig[:, None])


def surrogate_init(seed=12):
    """Initial parameters, flat float32: every matrix and bias of a layer with
    fan-in k drawn from U(-1/sqrt(k), 1/sqrt(k)); the output bias is 0."""
    rng = np.random.default_rng(seed)
    fan_in = [2 * SURR_N_FREQ] * 2 + [SURR_WIDTH] * (2 * (SURR_DEPTH - 1) + 1)
    parts = []
    for shp, k in zip(surrogate_param_shapes()[:-1], fan_in):
        lim = 1.0 / np.sqrt(k)
        parts.append(rng.uniform(-lim, lim, int(np.prod(shp))))
    parts.append(np.zeros(1))
    return _f32(np.concatenate(parts))


def surrogate_samples(scene, n, seed=6, near_frac=0.7, offset=0.5, box=1.5):
    """Training points: a fraction near_frac on area-weighted random triangle
    points moved along the face normal by U[-offset, offset], the rest uniform
    in [-box, box]^3."""
    rng = np.random.default_rng(seed)
    n_near = int(round(n * near_frac))
    near = surface_samples(scene.V, scene.T, n_near, rng, -offset, offset)
    far = rng.uniform(-box, box, (n - n_near, 3))
    X = np.concatenate([near, far])
    return _f32(X[rng.permutation(n)])


def terrain_surrogate_samples(scene, n, seed=6, near_frac=0.7, sigma=(0.01, 0.05, 0.2)):
    """Training points for the terrain scene: a fraction near_frac at random
    scene vertices (terrain points, net and torus vertices) moved by an
    isotropic Gaussian offset whose scale is drawn from `sigma`, the rest
    uniform in the query box (the scene box enlarged by 10 % of its extent on
    every side, as terrain_queries)."""
    rng = np.random.default_rng(seed)
    n_near = int(round(n * near_frac))
    V = scene.V
    base = V[rng.integers(0, len(V), n_near)].astype(np.float64)
    s = np.asarray(sigma, np.float64)[rng.integers(0, len(sigma), n_near)]
    near = base + rng.standard_normal((n_near, 3)) * s[:, None]
    lo, hi = scene_aabb(scene)
    far = rng.uniform(lo - 0.1 * (hi - lo), hi + 0.1 * (hi - lo), (n - n_near, 3))
    X = np.concatenate([near, far])
    return _f32(X[rng.permutation(n)])


def epoch_order(n, epoch, seed=13):
    """Shuffled sample order of one training epoch, int32."""
    return _i32(np.random.default_rng([seed, epoch]).permutation(n))


# --------------------------------------------------------------------------
# mixed co-dimensional street scene with a rigid body (differentiation workload)
# --------------------------------------------------------------------------
def street_scene(scale=1.0, seed=0):
    """Synthetic lidar street (metres; x in [0, 100], y in [-10, 10]) with every
    primitive class: ground points (z ~ N(0, 0.01^2)), 50 poles sampled as point
    columns (radius 0.1, height 8), two rows of box buildings whose facades are
    sampled on a 5 cm grid with 20 % dropout, four catenary wires through the
    pole tops (polylines, 5,000 segments each), and a 250 x 100 torus (R = 1,
    r = 0.35; 50,000 triangles) resting at (50, 0, 2).  At scale = 1 the point
    cloud holds exactly 2,000,000 points; smaller scales shrink every count.
    Returns (Scene, body_vertices) with the body in its own frame."""
    rng = np.random.default_rng(seed)
    n_ground = int(round(1_000_000 * scale))
    n_pole = max(int(round(2000 * scale)), 8)
    n_total = int(round(2_000_000 * scale))
    ground = np.stack([rng.uniform(0, 100, n_ground), rng.uniform(-10, 10, n_ground),
                       rng.normal(0, 0.01, n_ground)], 1)
    poles = []
    for k in range(50):
        th = rng.uniform(0, 2 * np.pi, n_pole)
        poles.append(np.stack([1 + 2 * k + 0.1 * np.cos(th), 8 + 0.1 * np.sin(th),
                               rng.uniform(0, 8, n_pole)], 1))
    poles = np.concatenate(poles)
    # building rows: 10 buildings of 10 m along x per row, heights U[6, 14];
    # facades at |y| = 10 and |y| = 14, 5 cm grid (coarser when scale < 1)
    h = 0.05 / np.sqrt(max(scale, 1e-6)) if scale < 1 else 0.05
    heights = rng.uniform(6, 14, (2, 10))
    fac = []
    for row, sgn in enumerate((1.0, -1.0)):
        for b in range(10):
            xs = np.arange(10 * b, 10 * b + 10, h) + 0.5 * h
            zs = np.arange(0, heights[row, b], h) + 0.5 * h
            gx, gz = np.meshgrid(xs, zs, indexing="ij")
            for yy in (10.0, 14.0):
                fac.append(np.stack([gx.ravel(), np.full(gx.size, sgn * yy), gz.ravel()], 1))
    fac = np.concatenate(fac)
    fac = fac[rng.random(len(fac)) < 0.8]
    need = n_total - n_ground - len(poles)
    fac = fac[rng.permutation(len(fac))[:max(need, 0)]]
    pts = np.concatenate([ground, poles, fac])
    # wires: catenaries z = z0 + c (cosh((x - xm)/c) - 1) - sag between consecutive
    # pole tops, 4 heights, 5,000 segments each along x in [1, 99]
    n_seg = max(int(round(5000 * scale)), 50)
    wires_v, wires_e = [], []
    base = len(pts)
    for z0 in (7.4, 7.6, 7.8, 8.0):
        x = np.linspace(1, 99, n_seg + 1)
        span = 2.0
        xm = 1 + span * (np.floor((x - 1) / span) + 0.5)
        c = 5.0
        z = z0 + c * (np.cosh((x - xm) / c) - 1) - c * (np.cosh(span / 2 / c) - 1)
        v = np.stack([x, np.full_like(x, 8.0), z], 1)
        e = np.stack([np.arange(n_seg), np.arange(n_seg) + 1], 1) + base
        wires_v.append(v)
        wires_e.append(e)
        base += len(v)
    wv = np.concatenate(wires_v)
    we = np.concatenate(wires_e)
    nu, nv = (250, 100) if scale >= 1 else (max(int(250 * np.sqrt(scale)), 12), max(int(100 * np.sqrt(scale)), 6))
    body, F = torus_grid(nu, nv, 1.0, 0.35)
    tv = body + np.array([50.0, 0.0, 2.0])
    V = np.concatenate([pts, wv, tv])
    T = F + base
    sc = Scene(V=_f32(V), P=_i32(np.arange(len(pts))), E=_i32(we), T=_i32(T), name=f"street_{scale:g}")
    return sc, _f32(body)


def rigid_transforms(K, seed=5, lo=(5.0, -8.0, 0.2), hi=(95.0, 8.0, 6.0)):
    """K random rigid transforms: rotations from unit quaternions, translations
    uniform in the box [lo, hi]; R (K, 3, 3) and t (K, 3), float32."""
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(K, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                  2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                  2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1)
    t = rng.uniform(lo, hi, (K, 3))
    return _f32(R.reshape(K, 3, 3)), _f32(t)


# --------------------------------------------------------------------------
# terrain + mesh scene for the alpha / precision sweep
# --------------------------------------------------------------------------
def _gradient_table(rng, period=256):
    """Random unit gradients on a period x period integer lattice."""
    ang = rng.uniform(0, 2 * np.pi, (period, period))
    return np.cos(ang), np.sin(ang)


def _gradient_noise_2d(x, y, table):
    """Seeded 2D gradient (Perlin-style) noise: the lattice gradients of
    `table`, quintic fade, bilinear blend of the corner dot products."""
    gx, gy = table
    period = gx.shape[0]
    xi, yi = np.floor(x).astype(np.int64), np.floor(y).astype(np.int64)
    fx, fy = x - xi, y - yi
    fade = lambda t: t * t * t * (t * (6 * t - 15) + 10)
    u, v = fade(fx), fade(fy)
    out = 0.0
    for dx in (0, 1):
        for dy in (0, 1):
            ix, iy = (xi + dx) % period, (yi + dy) % period
            dot = gx[ix, iy] * (fx - dx) + gy[ix, iy] * (fy - dy)
            wgt = (u if dx else 1 - u) * (v if dy else 1 - v)
            out = out + wgt * dot
    return out


def _terrain_heights(x, y, tables, chunk=1 << 20):
    """z = 0.25 sum_{o<6} 0.5^o n(2^o 2 (x, y)), elementwise, in chunks on a
    thread pool (numpy releases the interpreter lock in its array loops; the
    per-element arithmetic does not depend on the chunking)."""
    import concurrent.futures as cf
    import os
    z = np.zeros(len(x))

    def work(lo):
        hi = min(lo + chunk, len(x))
        xs, ys = x[lo:hi], y[lo:hi]
        acc = np.zeros(hi - lo)
        for o in range(6):
            f = 2.0 ** o * 2.0
            acc += 0.25 * 0.5 ** o * _gradient_noise_2d(f * xs + 37.0, f * ys + 91.0, tables[o])
        z[lo:hi] = acc

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, len(x), chunk)))
    return z


def terrain_scene(scale=1.0, seed=9):
    """Heightfield point cloud over [-1, 1]^2 (z = 0.25 sum_{o<6} 0.5^o
    n(2^o 2 (x, y)) with seeded gradient noise n, plus N(0, 0.005^2)), a torus
    (R = 0.5, r = 0.15, axis z, centred at (0, 0, 0.7)) and a hemispherical
    latitude-longitude net of edges (radius 0.4, centred at (-0.5, 0.5, 0.3)).
    At scale = 1: 20M points, 1M triangles (1000 x 500 grid), about 200,000
    edges; smaller scales shrink every count."""
    rng = np.random.default_rng(seed)
    n = max(int(round(20_000_000 * scale)), 100)
    x, y = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    noise_rng = np.random.default_rng(seed + 1000)
    tables = [_gradient_table(noise_rng) for _ in range(6)]
    z = _terrain_heights(x, y, tables)
    z += rng.normal(0, 0.005, n)
    pts = np.stack([x, y, z], 1)
    k = np.sqrt(scale)
    tv, tf = torus_grid(max(int(round(1000 * k)), 8), max(int(round(500 * k)), 4), 0.5, 0.15)
    tv = tv + np.array([0.0, 0.0, 0.7])
    n_lat = max(int(round(250 * k)), 4)
    n_lon = max(int(round(400 * k)), 8)
    th = np.linspace(0, 0.5 * np.pi, n_lat, endpoint=False)       # from the pole down to the rim
    ph = 2 * np.pi * np.arange(n_lon) / n_lon
    T_, P_ = np.meshgrid(th[1:], ph, indexing="ij")
    hv = np.stack([np.sin(T_) * np.cos(P_), np.sin(T_) * np.sin(P_), np.cos(T_)], -1).reshape(-1, 3)
    hv = np.concatenate([[[0.0, 0.0, 1.0]], hv]) * 0.4 + np.array([-0.5, 0.5, 0.3])
    idx = lambda i, j: 1 + i * n_lon + (j % n_lon)
    E = [[0, idx(0, j)] for j in range(n_lon)]
    for i in range(n_lat - 1):
        for j in range(n_lon):
            E.append([idx(i, j), idx(i, j + 1)])
            if i + 1 < n_lat - 1:
                E.append([idx(i, j), idx(i + 1, j)])
    E = np.asarray(E, np.int64)
    V = np.concatenate([pts, tv, hv])
    sc = Scene(V=_f32(V), P=_i32(np.arange(n)), E=_i32(E + n + len(tv)), T=_i32(tf + n),
               name=f"terrain_{scale:g}")
    return sc


def terrain_queries(scene, n, seed=10, grow=0.1):
    """Queries uniform in the scene's bounding box enlarged by `grow` of its
    extent on every side."""
    lo, hi = scene_aabb(scene)
    ext = hi - lo
    return uniform_queries(n, seed, lo - grow * ext, hi + grow * ext)
