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
