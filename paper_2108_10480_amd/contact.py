"""Frictionless rigid-body contact with one smooth-distance constraint (Sec. 4.5).

Each time step minimises an incremental potential whose unconstrained
minimiser is an implicit Euler step in position and an exponential Euler step
in orientation, subject to the single constraint

    D(M_d, M_q(p, theta)) - d_safe >= 0                       (Eq. 9)

where D is the smooth distance between the data mesh and the body's query
mesh (its vertices, outer log-sum-exp of Sec. 3.6).  The problem is solved
with a primal-dual interior-point method whose Hessian block is replaced by
the (constant) Hessian of the potential, the mass matrix, as a stand-in for
the paper's identity (it is exact for the quadratic potential and keeps the
units consistent); every accepted iterate is feasible (a backtracking line
search keeps the constraint >= 0).

The constraint value and gradient come from the library: the body vertices
are moved rigidly on the GPU, their smooth distances and gradients are
evaluated by Barnes-Hut, combined by the query-mesh log-sum-exp, and pulled
back to (p, theta) through the rigid adjoint.  Only the 6 x 6 solve runs on
the host.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


def rotvec_to_matrix(w):
    """exp([w]x) by Rodrigues' formula (FP64)."""
    w = np.asarray(w, np.float64)
    a = np.linalg.norm(w)
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if a < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(a) / a * K + (1 - np.cos(a)) / a ** 2 * (K @ K)


def left_jacobian(w):
    """J_l(w) of SO(3): I + (1 - cos a)/a^2 [w] + (a - sin a)/a^3 [w]^2."""
    w = np.asarray(w, np.float64)
    a = np.linalg.norm(w)
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if a < 1e-8:
        return np.eye(3) + 0.5 * K
    return np.eye(3) + (1 - np.cos(a)) / a ** 2 * K + (a - np.sin(a)) / a ** 3 * (K @ K)


class RigidBody:
    """A rigid body given by its vertices in the body frame (centred at the
    centre of mass, unit mass per vertex scaled to `mass`)."""

    def __init__(self, X, mass=1.0, p=(0.0, 0.0, 0.0), R=None, v=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0)):
        X = np.asarray(X, np.float64)
        c = X.mean(0)
        self.X = (X - c).astype(np.float32)
        self.mass = float(mass)
        m = self.mass / len(X)
        r = self.X.astype(np.float64)
        self.I_body = m * (np.sum(r * r) * np.eye(3) - r.T @ r)      # inertia of point masses
        self.p = np.asarray(p, np.float64) + 0.0
        self.R = np.eye(3) if R is None else np.asarray(R, np.float64)
        self.v = np.asarray(v, np.float64) + 0.0
        self.omega = np.asarray(omega, np.float64) + 0.0
        self._Xd = None

    @property
    def Xd(self):
        """The body-frame vertices in device memory (copied on first use)."""
        if self._Xd is None:
            self._Xd = torch.as_tensor(self.X, device="cuda")
        return self._Xd


class ContactStep:
    """One implicit time step of a body against a static scene."""

    def __init__(self, scene, alpha, alpha_q, beta=0.5, d_safe=0.0, h=1e-2, gravity=(0.0, 0.0, -9.81),
                 max_iter=50, tol=1e-8):
        self.scene, self.alpha, self.alpha_q, self.beta = scene, alpha, alpha_q, beta
        self.d_safe, self.h, self.g = d_safe, h, np.asarray(gravity, np.float64)
        self.max_iter, self.tol = max_iter, tol
        self.evals = 0
        self.stalls = 0   # solves ended at a feasible iterate with no feasible step left

    # constraint c(x) = D - d_safe and its gradient in x = (p, theta), theta a
    # rotation vector applied on the left of the step's start orientation R0
    def constraint(self, body, x, R0, grad=True):
        R = rotvec_to_matrix(x[3:]) @ R0
        Rt = torch.as_tensor(R.astype(np.float32), device="cuda").reshape(1, 3, 3)
        tt = torch.as_tensor(x[:3].astype(np.float32), device="cuda").reshape(1, 3)
        self.evals += 1
        if not grad:
            Q = api.sd_rigid_transform(body.Xd, Rt, tt)
            d, _ = api.sd_eval_grad(self.scene, Q, self.alpha, self.beta)
            D, _, _ = api.sd_query_mesh_lse(d.reshape(1, -1), None, self.alpha_q, want_w=False, want_vgrad=False)
            return float(D.item()) - self.d_safe, None
        Rt.requires_grad_(True)
        tt.requires_grad_(True)
        D = api.rigid_query_mesh_distance(body.Xd, Rt, tt, self.scene, self.alpha, self.alpha_q, beta=self.beta)
        D.sum().backward()
        gt = tt.grad.double().cpu().numpy().reshape(3)
        GR = Rt.grad.double().cpu().numpy().reshape(3, 3)
        # d/dtheta at theta: for R = exp([theta]) R0 and a small left rotation
        # dR = [dtheta] R, dD = sum_ab GR_ab ([dtheta] R)_ab = dtheta . (axial of GR R^T)
        M = GR @ R.T
        g_left = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
        # chain through exp: d exp([theta]) = [J_l(theta) dtheta] exp([theta])
        return float(D.item()) - self.d_safe, np.concatenate([gt, left_jacobian(x[3:]).T @ g_left])

    def step(self, body):
        """Advance the body by one time step; returns (iterations, final c)."""
        h, m = self.h, body.mass
        R0 = body.R.copy()
        I_w = R0 @ body.I_body @ R0.T
        # unconstrained minimiser: implicit Euler in position, exponential Euler in orientation
        p_hat = body.p + h * body.v + h * h * self.g
        th_hat = h * body.omega
        Hm = np.zeros((6, 6))
        Hm[:3, :3] = m / h ** 2 * np.eye(3)
        Hm[3:, 3:] = I_w / h ** 2 + 1e-12 * np.eye(3)
        x_hat = np.concatenate([p_hat, th_hat])
        grad_E = lambda x: Hm @ (x - x_hat)
        x = np.concatenate([body.p, np.zeros(3)])
        c, gc = self.constraint(body, x, R0)
        if not c > 0:
            raise RuntimeError(f"infeasible start: constraint {c:.3e}")
        lam, mu = 1.0, 1.0
        s = c
        it = 0
        for it in range(1, self.max_iter + 1):
            # primal-dual system (Nocedal & Wright 19.12) with the Hessian block
            # of the Lagrangian replaced by the potential's Hessian
            mu = max(0.1 * s * lam, 1e-16)
            rd = grad_E(x) - lam * gc              # dual residual
            rp = c - s                              # primal residual (s = c at feasible iterates)
            # eliminating ds = gc.dx + rp and dlam = (mu - s lam - lam ds) / s:
            # (H + (lam / s) gc gc^T) dx = -rd + gc (mu - s lam - lam rp) / s
            A = Hm + (lam / s) * np.outer(gc, gc)
            rhs = -rd + gc * ((mu - s * lam) - lam * rp) / s
            dx = np.linalg.solve(A, rhs)
            ds = gc @ dx + rp
            dl = (mu - s * lam - lam * ds) / s
            # fraction to the boundary, then backtrack until the new point is feasible
            tau = 0.995
            a_s = 1.0 if ds >= 0 else min(1.0, -tau * s / ds)
            a_l = 1.0 if dl >= 0 else min(1.0, -tau * lam / dl)
            a = min(a_s, 1.0)
            while True:
                xn = x + a * dx
                cn, gn = self.constraint(body, xn, R0)
                if cn > 0 or a < 1e-12:
                    break
                a *= 0.5
            if not cn > 0:
                # no feasible step along dx: next to the boundary the
                # Barnes-Hut constraint is only piecewise smooth (the near/far
                # switch moves it by rounding-sized jumps), so a Newton step
                # that would bring c closer to 0 can leave the feasible side
                # however short it is.  The current iterate is feasible and
                # as close to the optimum as the constraint resolves: end here.
                self.stalls += 1
                break
            x, c, gc = xn, cn, gn
            s = c
            lam = max(lam + a_l * dl, 1e-16)
            kkt = max(np.linalg.norm(grad_E(x) - lam * gc) / max(1.0, np.linalg.norm(Hm @ x_hat)), s * lam)
            if kkt < self.tol and np.linalg.norm(a * dx) < 1e-10 * max(1.0, np.linalg.norm(x)):
                break
            if np.linalg.norm(a * dx) < 1e-13 * max(1.0, np.linalg.norm(x)):
                break
        # update state: velocities from the step (implicit Euler)
        p_new = x[:3]
        R_new = rotvec_to_matrix(x[3:]) @ R0
        body.v = (p_new - body.p) / h
        body.omega = x[3:] / h
        body.p, body.R = p_new, R_new
        return it, c
