"""Forward-mode derivatives of the V-cycle iteration (oracle, test infrastructure only).

The map u_{i+1} = MG_L(u_i, b) (Alg. gmg with the additive smoother of
eq. additiveschwarz) depends on the right-hand side b, the per-level damping
omega_l and the per-level penalty factor gamma_hat_l.  Every matrix of a level
is affine in gamma_hat (the penalty term of eq. bfsipg is linear in gamma_e,
eq. penalty), so dA_l/dgamma_hat_l = A1_l, the penalty term assembled with
gamma_hat = 1, and the exact local solvers change by
d(A_j^-1) = -A_j^-1 (R_j A1_l R_j^T) A_j^-1.  This module propagates a tangent
(db, domega, dgamma) through the plain recursion step by step (no adjoint, no
tensor structure), giving directional derivatives of any output; the gradient
of a loss along a direction is then an inner product.

Pinned in tests/test_oracle_tangent.py against central finite differences of
the oracle's own forward map.
"""
import numpy as np
import scipy.linalg as sla

from .sipg import assemble


class TangentHierarchy:
    """Wraps an oracle multigrid.Hierarchy with the penalty derivatives."""

    def __init__(self, h):
        self.h = h
        self.A1 = []
        for m in h.meshes:
            self.A1.append(assemble(m, penalty_only=True) / m.gamma_hat)

    def vcycle(self, x, dx, b, db, domega, dgamma, l=None):
        h = self.h
        l = h.L if l is None else l
        if l == 0:
            x0 = sla.lu_solve(h.coarse_lu, b)
            dx0 = sla.lu_solve(h.coarse_lu, db - dgamma[0] * (self.A1[0] @ x0))
            return x0, dx0
        A, A1, om = h.A[l], self.A1[l], h.omegas[l]
        sol = h.solvers[l]

        def step(x, dx):
            r = b - A @ x
            dr = db - dgamma[l] * (A1 @ x) - A @ dx
            y = np.zeros_like(x)
            dy = np.zeros_like(x)
            for j, idx in enumerate(sol.subs):
                yj = sol.local_solve(j, r[idx])
                dAj = A1[idx][:, idx] @ yj
                y[idx] += yj
                dy[idx] += sol.local_solve(j, dr[idx] - dgamma[l] * dAj)
            return x + om * y, dx + domega[l] * y + om * dy

        for _ in range(h.m_pre):
            x, dx = step(x, dx)
        r = b - A @ x
        dr = db - dgamma[l] * (A1 @ x) - A @ dx
        P = h.P[l]
        n0 = h.meshes[l - 1].ndofs
        e, de = self.vcycle(np.zeros(n0), np.zeros(n0), P.T @ r, P.T @ dr, domega, dgamma, l - 1)
        x, dx = x + P @ e, dx + P @ de
        for _ in range(h.m_post):
            x, dx = step(x, dx)
        return x, dx

    def iterate(self, b, db, domega, dgamma, ncycles):
        """u_k and du_k after ncycles V-cycles from u_0 = 0."""
        u = np.zeros_like(b)
        du = np.zeros_like(b)
        for _ in range(ncycles):
            u, du = self.vcycle(u, du, b, db, domega, dgamma)
        return u, du
