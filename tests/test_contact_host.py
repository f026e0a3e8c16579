"""Host-side pieces of the rigid-body contact step (Sec. 4.5): the rotation
exponential and its left Jacobian against finite differences."""
import numpy as np
from scipy.spatial.transform import Rotation

from paper_2108_10480_amd import contact as C


def test_rotation_exponential_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(20):
        w = rng.normal(size=3) * rng.uniform(0, 3)
        np.testing.assert_allclose(C.rotvec_to_matrix(w), Rotation.from_rotvec(w).as_matrix(), atol=1e-12)


def test_left_jacobian_by_finite_differences():
    """exp([w + e]) exp([w])^T = exp([J_l(w) e]) to first order."""
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(10):
        w = rng.normal(size=3)
        J = C.left_jacobian(w)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            D = C.rotvec_to_matrix(w + e) @ C.rotvec_to_matrix(w).T
            axial = np.array([D[2, 1] - D[1, 2], D[0, 2] - D[2, 0], D[1, 0] - D[0, 1]]) / 2
            np.testing.assert_allclose(axial / h, J[:, k], atol=1e-6)


def _plane_step(jump=0.0, h0=0.0, width=1e-5):
    """A ContactStep whose constraint is a stand-in: the height of the body's
    centre above the plane z = h0, minus d_safe, with an optional downward
    jump of `jump` within `width` of the boundary (the kind of small
    discontinuity the Barnes-Hut constraint has there), where the returned
    gradient is zero (no model of the constraint there predicts the jump)."""
    step = C.ContactStep(scene=None, alpha=50.0, alpha_q=50.0, d_safe=0.05, h=0.01)

    def constraint(body, x, R0, grad=True):
        step.evals += 1
        c = x[2] - h0 - step.d_safe
        if jump > 0.0 and 0.0 < c < width:
            return c - jump, np.zeros(6)
        return c, np.array([0.0, 0.0, 1.0, 0.0, 0.0, 0.0])

    step.constraint = constraint
    return step


def _cube():
    g = np.array([-0.1, 0.1])
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.column_stack([X.ravel(), Y.ravel(), Z.ravel()])


def test_falling_body_rests_on_a_smooth_constraint():
    step = _plane_step()
    body = C.RigidBody(_cube(), mass=1.0, p=(0.0, 0.0, 0.3), omega=(0.0, 0.0, 1.0))
    for _ in range(80):
        it, c = step.step(body)
        assert c > 0 and it < step.max_iter
    assert 0.0 < body.p[2] - 0.05 < 1e-3            # on the constraint, not hovering
    assert abs(body.v[2]) < 1e-2
    np.testing.assert_allclose(body.omega, [0.0, 0.0, 1.0], atol=1e-9)   # no torque from a central constraint
    assert step.stalls == 0


def test_jump_next_to_the_boundary_ends_at_a_feasible_iterate():
    """When the solve ends at an infeasible point (here: the target c_res
    lies inside a jump that takes the constraint below zero), the step
    returns its feasible start instead, and the solve is counted."""
    step = _plane_step(jump=2e-5)
    body = C.RigidBody(_cube(), mass=1.0, p=(0.0, 0.0, 0.3))
    for _ in range(80):
        it, c = step.step(body)
        assert c > 0 and step.c_res < 1e-5
        assert body.p[2] - 0.05 > 0.0
    assert step.stalls > 0
