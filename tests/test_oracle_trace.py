"""Pins of the reference sphere tracer: closed-form hits and misses on the
distance to a sphere, and agreement with a root of the exact distance."""
import numpy as np
from scipy.optimize import brentq

from oracle import trace as TR


def test_sphere_closed_form():
    """Distance to the origin minus nothing, level 0.5: a ray from (3, b, 0)
    along -x hits the sphere of radius 0.5 at 3 - sqrt(0.25 - b^2) when
    b < 0.5 and misses otherwise."""
    b = np.array([0.0, 0.1, 0.3, 0.45, 0.6, 0.9])
    O = np.stack([np.full_like(b, 3.0), b, np.zeros_like(b)], 1)
    U = np.tile([-1.0, 0.0, 0.0], (len(b), 1))
    t, steps = TR.sphere_trace(lambda X: np.linalg.norm(X, axis=1), O, U, level=0.5, eps=1e-9, t_max=8.0,
                               max_steps=10000)
    hit = b < 0.5
    np.testing.assert_allclose(t[hit], 3 - np.sqrt(0.25 - b[hit] ** 2), atol=1e-8)
    assert np.all(np.isposinf(t[~hit]))
    assert steps[0] == 2          # straight on: one step lands exactly on the sphere


def test_root_of_a_smooth_distance():
    """On the distance to a segment the hit is the first root of d - level along
    the ray (bracketed and solved independently)."""
    a, c = np.array([-1.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0])

    def seg(X):
        e = c - a
        s = np.clip(((X - a) @ e) / (e @ e), 0, 1)
        return np.linalg.norm(X - (a + s[:, None] * e), axis=1)

    rng = np.random.default_rng(3)
    O = np.column_stack([rng.uniform(-0.8, 0.8, 20), np.full(20, 2.0), rng.uniform(-0.2, 0.2, 20)])
    U = np.tile([0.0, -1.0, 0.0], (20, 1))
    t, _ = TR.sphere_trace(seg, O, U, level=0.25, eps=1e-10, t_max=5.0, max_steps=10000)
    for k in range(20):
        f = lambda s: seg((O[k] + s * U[k])[None])[0] - 0.25
        assert abs(t[k] - brentq(f, 0.0, 2.0)) < 1e-7
