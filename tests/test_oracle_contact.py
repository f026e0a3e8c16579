"""Pins of the oracle's contact step (Sec. 4.5, Eq. 9): the rotation and its
derivative against finite differences and a library rotation, the constraint
gradient against finite differences of its value, free flight equal to the
implicit / exponential Euler step, a single-vertex body against a single data
point equal to the closed-form projection onto the sphere |p - P| = d_safe,
and the KKT conditions at a general contact."""
import numpy as np
from scipy.spatial.transform import Rotation


def _cube(n=3, side=0.2):
    g = (np.arange(n) / (n - 1) - 0.5) * side
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.column_stack([X.ravel(), Y.ravel(), Z.ravel()])


def _plane(O, step=0.1):
    g = np.arange(-0.5, 0.5001, step)
    X, Y = np.meshgrid(g, g)
    P = np.column_stack([X.ravel(), Y.ravel(), np.zeros(X.size)]).astype(np.float32)
    return O.OracleScene(P, P=np.arange(len(P)))


def test_rotation_and_its_derivative(oracle_mod):
    from oracle import contact as OC
    rng = np.random.default_rng(1)
    for _ in range(10):
        th = rng.normal(size=3) * rng.uniform(0.0, 2.5)
        np.testing.assert_allclose(OC.rotation(th), Rotation.from_rotvec(th).as_matrix(), atol=1e-13)
        dR = OC.rotation_derivative(th)
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd = (OC.rotation(th + e) - OC.rotation(th - e)) / (2 * h)
            np.testing.assert_allclose(dR[k], fd, atol=1e-8)
    # near zero (series branch)
    th = np.array([1e-9, -2e-9, 3e-9])
    np.testing.assert_allclose(OC.rotation_derivative(th)[0], OC._hat(np.eye(3)[0]), atol=1e-8)


def test_constraint_gradient_by_finite_differences(oracle_mod):
    from oracle import contact as OC
    O = oracle_mod
    sc = _plane(O)
    X = _cube()
    R0 = OC.rotation([0.3, -0.2, 0.5])
    rng = np.random.default_rng(2)
    for _ in range(3):
        x = np.concatenate([rng.uniform(-0.1, 0.1, 2), [rng.uniform(0.15, 0.3)], rng.normal(size=3) * 0.3])
        c, g = OC.constraint(sc, X, R0, x, alpha=40.0, alpha_q=40.0, d_safe=0.05)
        h = 1e-6
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            cp, _ = OC.constraint(sc, X, R0, x + e, 40.0, 40.0, 0.05)
            cm, _ = OC.constraint(sc, X, R0, x - e, 40.0, 40.0, 0.05)
            assert abs((cp - cm) / (2 * h) - g[k]) < 1e-7 * max(1.0, abs(g[k]))


def test_free_flight_is_the_euler_step(oracle_mod):
    from oracle import contact as OC
    O = oracle_mod
    sc = O.OracleScene(np.array([[0.0, 0.0, -50.0]], np.float32), P=np.array([0]))
    X = _cube()
    p0, v0, w0 = np.array([0.0, 0.0, 1.0]), np.array([0.5, 0.0, 1.0]), np.array([0.3, -0.2, 2.0])
    r = OC.contact_step(sc, X, 2.0, p0, np.eye(3), v0, w0, 0.01, (0, 0, -9.81), 50.0, 50.0, 0.05)
    np.testing.assert_allclose(r["p"], p0 + 0.01 * v0 + 1e-4 * np.array([0, 0, -9.81]), atol=1e-12)
    np.testing.assert_allclose(r["omega"], w0, atol=1e-10)
    np.testing.assert_allclose(r["R"], OC.rotation(0.01 * w0), atol=1e-12)


def test_single_vertex_on_a_single_point_is_the_sphere_projection(oracle_mod):
    """One data point P, a one-vertex body: D = |p - P| (one term of weight 1
    in both sums), so the step is the projection of p^ onto |p - P| >= d_safe."""
    from oracle import contact as OC
    O = oracle_mod
    P = np.array([0.1, -0.2, 0.0])
    sc = O.OracleScene(P.astype(np.float32)[None], P=np.array([0]))
    X = np.zeros((1, 3))
    p0, v0 = np.array([0.12, -0.19, 0.08]), np.array([0.3, 0.1, -5.0])
    h, d_safe = 0.01, 0.05
    r = OC.contact_step(sc, X, 1.0, p0, np.eye(3), v0, np.zeros(3), h, (0, 0, -9.81), 30.0, 30.0, d_safe)
    p_hat = p0 + h * v0 + h * h * np.array([0, 0, -9.81])
    assert np.linalg.norm(p_hat - P) < d_safe            # the constraint is active
    np.testing.assert_allclose(r["p"], P + d_safe * (p_hat - P) / np.linalg.norm(p_hat - P), atol=1e-9)


def test_kkt_at_a_general_contact(oracle_mod):
    """A tilted cube pressed onto a point-sampled plane: the constraint is
    active (c = 0) and the energy gradient is lambda times the constraint
    gradient with lambda >= 0, both gradients by finite differences."""
    from oracle import contact as OC
    O = oracle_mod
    sc = _plane(O)
    X = _cube()
    R0 = OC.rotation([0.2, 0.4, 0.1])
    p0, v0, w0 = np.array([0.02, -0.01, 0.16]), np.array([0.1, 0.0, -3.0]), np.array([1.0, -0.5, 0.3])
    h, m, d_safe, a = 0.01, 1.0, 0.05, 40.0
    r = OC.contact_step(sc, X, m, p0, R0, v0, w0, h, (0, 0, -9.81), a, a, d_safe)
    x = r["x"]
    assert abs(r["c"]) < 1e-9 and r["lambda"] > 0
    Xc = X - X.mean(0)
    I = R0 @ OC.body_inertia(Xc, m) @ R0.T
    p_hat, th_hat = p0 + h * v0 + h * h * np.array([0, 0, -9.81]), h * w0
    E = lambda y: 0.5 * m / h ** 2 * np.sum((y[:3] - p_hat) ** 2) + 0.5 / h ** 2 * (y[3:] - th_hat) @ I @ (y[3:] - th_hat)
    C = lambda y: OC.constraint(sc, Xc, R0, y, a, a, d_safe)[0]
    hstep = 1e-6
    gE, gC = np.zeros(6), np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = hstep
        gE[k] = (E(x + e) - E(x - e)) / (2 * hstep)
        gC[k] = (C(x + e) - C(x - e)) / (2 * hstep)
    lam = gE @ gC / (gC @ gC)
    assert lam > 0
    assert np.linalg.norm(gE - lam * gC) < 1e-5 * np.linalg.norm(gE)
