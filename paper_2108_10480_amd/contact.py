"""Frictionless rigid-body contact with one smooth-distance constraint (Sec. 4.5).

Each time step minimises an incremental potential whose unconstrained
minimiser is an implicit Euler step in position and an exponential Euler step
in orientation, subject to the single constraint

    D(M_d, M_q(p, theta)) - d_safe >= 0                       (Eq. 9)

where D is the smooth distance between the data mesh and the body's query
mesh (its vertices, outer log-sum-exp of Sec. 3.6).  Where the unconstrained
minimiser (the implicit Euler step) is feasible it is the step; otherwise the
constrained minimiser is found by sequential quadratic programming (a
quasi-Newton model of the Lagrangian, in variables scaled so that the
potential's Hessian is the identity) with the target c >= c_res > 0.  The
paper solves this with a primal-dual interior-point method whose Hessian
block it replaces by an identity; built that way (also with the mass matrix,
with damped BFGS, and on a log barrier) the solve crept along the curved
constraint near an impact and often ended millimetres from the minimiser,
because the constraint's curvature lambda grad^2 c is there as large as the
mass matrix; the quasi-Newton model of the Lagrangian in SQP carries it.
Every returned step is strictly feasible.

The constraint value and gradient come from the library: the body vertices
are moved rigidly on the GPU, their smooth distances and gradients are
evaluated by Barnes-Hut, combined by the query-mesh log-sum-exp, and pulled
back to (p, theta) through the rigid adjoint.  Only the 6 x 6 solve runs on
the host.

Next to the boundary the Barnes-Hut constraint is only piecewise smooth: as
the body moves, nodes switch between the far field and their children, and
each switch moves the value by a small jump (Sec. 4.3), which no smooth model
of the constraint can follow.  So where the Barnes-Hut value lies below
`exact_band` the constraint is evaluated exactly (beta = 0: every primitive,
Eq. 3), which is smooth; far from contact Barnes-Hut is used.  For point
clouds and closed triangle meshes the exact value is at least the Barnes-Hut
one (App. A with the far field's n_B A^S >= each weight), so the switch never
makes a feasible point infeasible.
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
        self.radius = float(np.linalg.norm(self.X.astype(np.float64), axis=1).max())
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
                 max_iter=50, exact_band=None, c_res=None, kkt_tol=1e-7):
        self.scene, self.alpha, self.alpha_q, self.beta = scene, alpha, alpha_q, beta
        self.d_safe, self.h, self.g = d_safe, h, np.asarray(gravity, np.float64)
        self.max_iter, self.kkt_tol = max_iter, kkt_tol
        # constraint values below this are re-evaluated exactly (default: the
        # safety distance, at least 1e-3)
        self.exact_band = max(d_safe, 1e-3) if exact_band is None else exact_band
        # the solve targets c >= c_res > 0 and accepts the constraint met to
        # within c_res / 2, so every returned step keeps c >= c_res / 2 > 0.
        # The computed constraint carries FP32 vertex positions and distances,
        # rounded at about 2^-24 of the body's world coordinates (`rounding`);
        # a target below that would be chased without end.  By default c_res
        # is 64 times that rounding, set per step.
        self.c_res_fixed = c_res
        self.c_res = c_res
        self.evals = 0
        self.exact_evals = 0
        self.stalls = 0       # solves that did not converge
        self.infeasible = 0   # of those, solves that ended infeasible (the step returned its start)

    # constraint c(x) = D - d_safe and its gradient in x = (p, theta), theta a
    # rotation vector applied on the left of the step's start orientation R0
    def constraint(self, body, x, R0, grad=True):
        c, gc = self._constraint(body, x, R0, grad, self.beta)
        if self.beta > 0 and c < self.exact_band:
            self.exact_evals += 1
            c, gc = self._constraint(body, x, R0, grad, 0.0)
        return c, gc

    def _constraint(self, body, x, R0, grad, beta):
        R = rotvec_to_matrix(x[3:]) @ R0
        Rt = torch.as_tensor(R.astype(np.float32), device="cuda").reshape(1, 3, 3)
        tt = torch.as_tensor(x[:3].astype(np.float32), device="cuda").reshape(1, 3)
        self.evals += 1
        if not grad:
            Q = api.sd_rigid_transform(body.Xd, Rt, tt)
            d, _ = api.sd_eval_grad(self.scene, Q, self.alpha, beta)
            D, _, _ = api.sd_query_mesh_lse(d.reshape(1, -1), None, self.alpha_q, want_w=False, want_vgrad=False)
            return float(D.item()) - self.d_safe, None
        Rt.requires_grad_(True)
        tt.requires_grad_(True)
        D = api.rigid_query_mesh_distance(body.Xd, Rt, tt, self.scene, self.alpha, self.alpha_q, beta=beta)
        D.sum().backward()
        gt = tt.grad.double().cpu().numpy().reshape(3)
        GR = Rt.grad.double().cpu().numpy().reshape(3, 3)
        # d/dtheta at theta: for R = exp([theta]) R0 and a small left rotation
        # dR = [dtheta] R, dD = sum_ab GR_ab ([dtheta] R)_ab = dtheta . (axial of GR R^T)
        M = GR @ R.T
        g_left = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
        # chain through exp: d exp([theta]) = [J_l(theta) dtheta] exp([theta])
        return float(D.item()) - self.d_safe, np.concatenate([gt, left_jacobian(x[3:]).T @ g_left])

    @staticmethod
    def rounding(body):
        """Rounding level of the computed constraint near the body: half an
        FP32 unit in the last place of its largest world coordinate."""
        return 2.0 ** -24 * (float(np.abs(body.p).max()) + body.radius)

    def step(self, body):
        """Advance the body by one time step; returns (iterations, final c)."""
        h, m = self.h, body.mass
        self.noise = self.rounding(body)
        self.c_res = 64.0 * self.noise if self.c_res_fixed is None else self.c_res_fixed
        R0 = body.R.copy()
        I_w = R0 @ body.I_body @ R0.T
        # unconstrained minimiser: implicit Euler in position, exponential Euler in orientation
        p_hat = body.p + h * body.v + h * h * self.g
        th_hat = h * body.omega
        Hm = np.zeros((6, 6))
        Hm[:3, :3] = m / h ** 2 * np.eye(3)
        Hm[3:, 3:] = I_w / h ** 2 + 1e-12 * np.eye(3)
        x_hat = np.concatenate([p_hat, th_hat])
        x = np.concatenate([body.p, np.zeros(3)])
        it = 0
        # the unconstrained minimiser, where it is feasible, is the step
        c, gc = self.constraint(body, x_hat, R0)
        if c > 0:
            x = x_hat
        else:
            x, c, it = self._solve(body, R0, Hm, x_hat, x)
        # update state: velocities from the step (implicit Euler)
        p_new = x[:3]
        R_new = rotvec_to_matrix(x[3:]) @ R0
        body.v = (p_new - body.p) / h
        body.omega = x[3:] / h
        body.p, body.R = p_new, R_new
        return it, c

    def _solve(self, body, R0, Hm, x_hat, x):
        """min E(x) s.t. c(x) >= c_res by sequential quadratic programming in
        variables y scaled so that E = |y|^2 / 2 (x = x_hat + Linv^T y).

        Each iteration solves the QP  min 1/2 d^T B d + y^T d  s.t.
        g + a^T d >= 0  (g = c - c_res, a its gradient in y) in closed form,
        B being a BFGS model of the Lagrangian's Hessian I - mu grad^2 g with
        Powell's damping (the constraint's curvature, as large here as the
        energy's, is what B learns), and steps along d with a backtracking
        line search on the l1 merit function E + rho max(0, -g) that accepts
        an increase up to what the constraint's rounding can cause
        (rho times twice the rounding): near a flat contact the constraint
        barely changes along some directions, and its rounding would
        otherwise reject every step there.  The solve
        has converged once the constraint is met to within c_res / 2 and the
        Lagrangian's gradient y - mu a is below kkt_tol (mu >= 0 the least
        squares multiplier), a test first order in the distance to the
        minimiser along the constraint.  A solve that ends infeasible returns
        its start (a feasible point); one that ends without converging is
        counted as a stall."""
        L = np.linalg.cholesky(Hm)
        Linv_t = np.linalg.inv(L).T

        def cons(y):
            c, gc = self.constraint(body, x_hat + Linv_t @ y, R0)
            return c - self.c_res, gc @ Linv_t

        y = L.T @ (x - x_hat)
        g, a = cons(y)
        B = np.eye(6)
        rho, mu = 0.0, 0.0
        it, converged = 0, False
        while it < self.max_iter:
            aa = float(a @ a)
            if aa == 0.0 and g < 0.0:
                break                      # violated and no gradient to follow
            mu_ls = max(0.0, float(y @ a) / aa) if aa > 0.0 else 0.0
            if g >= -0.5 * self.c_res and (mu_ls == 0.0 or g <= 0.5 * self.c_res) \
                    and np.linalg.norm(y - mu_ls * a) <= self.kkt_tol * max(1.0, np.linalg.norm(y)):
                converged = True
                break
            it += 1
            Bi_y, Bi_a = np.linalg.solve(B, y), np.linalg.solve(B, a)
            d, mu = -Bi_y, 0.0
            if g + a @ d < 0.0:
                mu = -(g + a @ d) / (a @ Bi_a)
                d = d + mu * Bi_a
            rho = max(rho, 2.0 * mu)
            merit = lambda yy, gg: 0.5 * yy @ yy + rho * max(0.0, -gg)
            m0 = merit(y, g)
            slope = y @ d - rho * max(0.0, -g)
            t = 1.0
            while True:
                y1 = y + t * d
                g1, a1 = cons(y1)
                if merit(y1, g1) <= m0 + 1e-4 * t * slope + 2.0 * rho * self.noise or t < 2.0 ** -12:
                    break
                t *= 0.5
            s = y1 - y
            r = s - mu * (a1 - a)          # change of the Lagrangian's gradient
            Bs = B @ s
            sBs, sr = float(s @ Bs), float(s @ r)
            if sBs > 0.0:
                th = 1.0 if sr >= 0.2 * sBs else 0.8 * sBs / (sBs - sr)
                r = th * r + (1.0 - th) * Bs
                B = B + np.outer(r, r) / float(s @ r) - np.outer(Bs, Bs) / sBs
            y, g, a = y1, g1, a1
        c = g + self.c_res
        xs = x_hat + Linv_t @ y
        if not converged:
            self.stalls += 1
        if not (c > 0):
            self.infeasible += 1
            xs, (c, _) = x, self.constraint(body, x, R0, grad=False)
        return xs, c, it
