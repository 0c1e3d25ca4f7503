"""Geometric multigrid V-cycle (oracle, test infrastructure only).

Sec. 2.2, Alg. (gmg): on level 0 the coarse problem is solved exactly (here by
dense LU of A_0, the coarse solver of the benchmark workloads); on level l > 0:
m_pre smoothing steps, restriction of the residual, recursion with zero
initial guess, prolongation and correction, m_post smoothing steps.  The
printed algorithm has no return after the coarse solve; the oracle returns
there (the only meaningful reading).

A_l is the SIPG matrix re-discretised on each level.  The prolongation is the
embedding of the nested spaces V_{l-1} in V_l: the fine coefficients of a
coarse function are its values at the fine Gauss-Lobatto nodes.  The
restriction is its transpose (adjoint in the Euclidean coefficient inner
product).

Pins: polynomial reproduction of the prolongation, restriction = transpose,
one level = LU solve, symmetry of the V-cycle preconditioner for
m_pre = m_post, and contraction of the error in the energy norm.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import gll_nodes, lagrange_values
from .mesh import coarsen
from .sipg import assemble, tensor
from .schwarz import (ExactLocalSolvers, cell_subdomains, vertex_patch_subdomains, additive_smooth,
                      multiplicative_smooth, cell_red_black, vertex_patch_mult_colors)


def prolongation(mesh_c, mesh_f):
    """Sparse P: V_{l-1} -> V_l, P[(Kf, i), (Kc, j)] = phi_{Kc, j}(x_{Kf, i})."""
    d, n1 = mesh_f.dim, mesh_f.n1
    nodes = gll_nodes(mesh_f.k)
    rows, cols, vals = [], [], []
    for cf in mesh_f.cells():
        cc = tuple(c // 2 for c in cf)
        factors = []
        for a in range(d):
            xf = mesh_f.offsets(a)[cf[a]] + mesh_f.widths[a][cf[a]] * nodes
            xi = (xf - mesh_c.offsets(a)[cc[a]]) / mesh_c.widths[a][cc[a]]
            factors.append(lagrange_values(nodes, xi))
        B = tensor(factors)
        r = mesh_f.cell_dofs(cf)
        c = mesh_c.cell_dofs(cc)
        rows.append(np.repeat(r, len(c)))
        cols.append(np.tile(c, len(r)))
        vals.append(B.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh_f.ndofs, mesh_c.ndofs)).tocsr()


class Hierarchy:
    """Levels 0..L built by coarsening ``fine`` nlevels-1 times.

    omegas[l] and gamma_hats[l] (l = 0..L) are per-level relaxation and
    penalty factors (omegas[0] unused).  smoother: "additive" (Alg. addsmoother)
    or "multiplicative" (Alg. multsmoother with red-black cells or the 2^(d+1)
    vertex-patch colors, pre- and post-smoothing in the same color order), or
    "multiplicative_symmetric" (post-smoothing in the reverse color order, the
    symmetrisation Sec. 4 applies so that the V-cycle preconditions CG)."""

    def __init__(self, fine, nlevels, kind="vertex", omegas=0.5, m_pre=1, m_post=1,
                 gamma_hats=None, cache=True, smoother="additive"):
        meshes = [fine]
        for _ in range(nlevels - 1):
            meshes.insert(0, coarsen(meshes[0]))
        L = nlevels - 1
        self.omegas = [omegas] * (L + 1) if np.isscalar(omegas) else list(omegas)
        if gamma_hats is not None:
            gh = [gamma_hats] * (L + 1) if np.isscalar(gamma_hats) else list(gamma_hats)
            for l, m in enumerate(meshes):
                m.gamma_hat = gh[l]
        self.meshes, self.L, self.kind = meshes, L, kind
        self.m_pre, self.m_post = m_pre, m_post
        self.A = [assemble(m) for m in meshes]
        self.P = [None] + [prolongation(meshes[l - 1], meshes[l]) for l in range(1, L + 1)]
        subs = cell_subdomains if kind == "cell" else vertex_patch_subdomains
        self.solvers = [None] + [ExactLocalSolvers(self.A[l], subs(meshes[l]), cache)
                                 for l in range(1, L + 1)]
        self.coarse_lu = sla.lu_factor(self.A[0].toarray())
        self.smoother = smoother
        col = cell_red_black if kind == "cell" else vertex_patch_mult_colors
        self.colors = [None] + [col(meshes[l]) for l in range(1, L + 1)]

    def smooth(self, l, x, b, post=False):
        if self.smoother in ("multiplicative", "multiplicative_symmetric"):
            colors = self.colors[l]
            if post and self.smoother == "multiplicative_symmetric":
                top = max(colors)
                colors = [top - c for c in colors]  # the same colors, visited in reverse order
            return multiplicative_smooth(self.A[l], self.solvers[l], x, b, self.omegas[l], colors)
        return additive_smooth(self.A[l], self.solvers[l], x, b, self.omegas[l])

    def vcycle(self, x, b, l=None):
        l = self.L if l is None else l
        if l == 0:
            return sla.lu_solve(self.coarse_lu, b)
        for _ in range(self.m_pre):
            x = self.smooth(l, x, b)
        bc = self.P[l].T @ (b - self.A[l] @ x)
        e = self.vcycle(np.zeros(self.meshes[l - 1].ndofs), bc, l - 1)
        x = x + self.P[l] @ e
        for _ in range(self.m_post):
            x = self.smooth(l, x, b, post=True)
        return x
