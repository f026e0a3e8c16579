"""FP64 reference for one rigid-body contact time step (Sec. 4.5, Eq. 9).

TEST INFRASTRUCTURE ONLY.  Only the tests import this module; it shares no
code with the library (in particular not with its interior-point solver) and
never calls it.

One step of a rigid body of point masses (the body's vertices X, body frame,
centred at the centre of mass) against a static data mesh is the constrained
minimisation

    min_x  E(x) = (m / 2h^2) |p - p^|^2 + (1 / 2h^2) (th - th^)^T I (th - th^)
    s.t.   c(x) = D(M_d, M_q(p, th)) - d_safe >= 0                    (Eq. 9)

over x = (p, th): p the new position, th a rotation vector applied on the
left of the step's start orientation R0, p^ = p0 + h v0 + h^2 g and
th^ = h omega0 (the unconstrained minimiser is the implicit Euler step in
position and the exponential Euler step in orientation), I = R0 I_body R0^T
the world inertia of the point masses.  D is the query-mesh distance of the
moved vertices (Sec. 3.6, Eq. 6): the outer log-sum-exp with alpha_q of their
smooth distances to the data (Eq. 3, every primitive exact, i.e. beta = 0).
The minimiser does not depend on how it is found; here it is found by a
library SQP solver (scipy SLSQP) on the FP64 constraint and its gradient,
which follows from Eq. 4, Eq. 8 and the derivative of the rotation.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

from oracle import oracle as O
from oracle import qmesh as QM


def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def rotation(th):
    """exp([th]): the rotation by |th| about th / |th| (Rodrigues)."""
    th = np.asarray(th, np.float64)
    a = float(np.linalg.norm(th))
    K = _hat(th)
    if a == 0.0:
        return np.eye(3)
    return np.eye(3) + np.sin(a) / a * K + (1.0 - np.cos(a)) / a ** 2 * (K @ K)


def rotation_derivative(th):
    """d exp([th]) / d th_k for k = 0, 1, 2 (3 x 3 x 3), from the closed form
    of Rodrigues' formula differentiated term by term."""
    th = np.asarray(th, np.float64)
    a = float(np.linalg.norm(th))
    K = _hat(th)
    E = [_hat(np.eye(3)[k]) for k in range(3)]
    if a < 1e-8:   # first order: exp([th]) = I + [th] + [th]^2 / 2
        return np.array([E[k] + 0.5 * (E[k] @ K + K @ E[k]) for k in range(3)])
    s, c = np.sin(a), np.cos(a)
    f1, f2 = s / a, (1.0 - c) / a ** 2
    df1 = (a * c - s) / a ** 2          # d f1 / d a
    df2 = (a * s - 2.0 * (1.0 - c)) / a ** 3
    out = []
    for k in range(3):
        da = th[k] / a
        out.append(df1 * da * K + f1 * E[k] + df2 * da * (K @ K) + f2 * (E[k] @ K + K @ E[k]))
    return np.array(out)


def body_inertia(X, mass):
    """Inertia tensor of len(X) equal point masses about their mean."""
    X = np.asarray(X, np.float64)
    r = X - X.mean(0)
    m = mass / len(X)
    return m * (np.sum(r * r) * np.eye(3) - r.T @ r)


def constraint(scene, Xb, R0, x, alpha, alpha_q, d_safe):
    """c(x) and dc/dx for x = (p, th): vertices q_j = exp([th]) R0 X_j + p."""
    p, th = x[:3], x[3:]
    Rth = rotation(th)
    Y = Xb @ R0.T                      # R0 X_j
    Q = Y @ Rth.T + p
    d, g, _ = O.brute(scene, Q, alpha)
    D, w, _ = QM.query_mesh_lse(d.reshape(1, -1), g.reshape(1, -1, 3), alpha_q)
    w = w.reshape(-1)
    u = w[:, None] * g                 # dD/dq_j
    dp = u.sum(0)
    dR = rotation_derivative(th)       # d q_j / d th_k = (dExp_k) Y_j
    dth = np.array([np.sum(u * (Y @ dR[k].T)) for k in range(3)])
    return float(D[0]) - d_safe, np.concatenate([dp, dth])


def contact_step(scene, Xb, mass, p0, R0, v0, w0, h, gravity, alpha, alpha_q, d_safe):
    """The constrained minimiser x* = (p, th) of one step and the new state
    (p, R, v, omega) = (p, exp([th]) R0, (p - p0) / h, th / h)."""
    Xb = np.asarray(Xb, np.float64)
    Xb = Xb - Xb.mean(0)
    p0, v0, w0 = (np.asarray(a, np.float64) for a in (p0, v0, w0))
    R0 = np.asarray(R0, np.float64)
    Iw = R0 @ body_inertia(Xb, mass) @ R0.T
    p_hat = p0 + h * v0 + h * h * np.asarray(gravity, np.float64)
    th_hat = h * w0
    Hp, Hth = mass / h ** 2, Iw / h ** 2

    def energy(x):
        dp, dt = x[:3] - p_hat, x[3:] - th_hat
        return 0.5 * Hp * dp @ dp + 0.5 * dt @ Hth @ dt, np.concatenate([Hp * dp, Hth @ dt])

    # scale the variables so that the energy's Hessian is the identity (the
    # solver's tolerances then mean the same thing in every coordinate)
    L = np.linalg.cholesky(Hth + 1e-12 * np.eye(3))
    S = np.zeros((6, 6))
    S[:3, :3] = np.eye(3) / np.sqrt(Hp)
    S[3:, 3:] = np.linalg.inv(L).T
    x_hat = np.concatenate([p_hat, th_hat])
    c0 = lambda y: constraint(scene, Xb, R0, x_hat + S @ y, alpha, alpha_q, d_safe)
    cache = {}

    def cfun(y):
        k = y.tobytes()
        if k not in cache:
            cache[k] = c0(y)
        return cache[k]

    res = minimize(lambda y: (0.5 * y @ y, y), np.zeros(6), jac=True, method="SLSQP",
                   constraints=[{"type": "ineq", "fun": lambda y: cfun(y)[0],
                                 "jac": lambda y: cfun(y)[1] @ S}],
                   options={"ftol": 1e-15, "maxiter": 500})
    x = x_hat + S @ res.x
    c, gc = constraint(scene, Xb, R0, x, alpha, alpha_q, d_safe)
    e, ge = energy(x)
    lam = float(ge @ gc / (gc @ gc)) if c < 1e-6 else 0.0
    return {"x": x, "p": x[:3], "R": rotation(x[3:]) @ R0, "v": (x[:3] - p0) / h, "omega": x[3:] / h,
            "c": c, "lambda": lam, "kkt": float(np.linalg.norm(ge - lam * gc)), "success": bool(res.success)}
