"""SIPG on meshes of mapped cells and the Cartesian surrogate local solvers of
Sec. 4 (oracle, test infrastructure only).

Mesh.  A logically Cartesian mesh whose cells are the images of the
reference cell [0, 1]^d under the multilinear map through their 2^d vertices
(vertices shared by neighbouring cells, so the mesh is conforming; faces of
3-D cells are bilinear surfaces).  Cells and DoFs are numbered as on
Cartesian meshes (Sec. 2.1, eq. multiindex: cells lexicographic with x
fastest, Lagrange DoFs in the Gauss-Lobatto points of the reference cell).

Operator.  The interior penalty form eq. (bfsipg) with the averages of
eq. (jumpavgscalar) integrated on the mapped cells: gradients
grad phi = J^-T grad_xi phi, volume element det J, on a face the outward unit
normal n = J^-T e_t / |J^-T e_t| (times the side's sign) and the area element
det J |J^-T e_t| (Nanson's formula), all evaluated by a tensor Gauss rule of
k+1 points per axis (the integrands are no longer polynomial: the rule is part
of the discrete operator).  The penalty eq. (penalty) needs h+- orthogonal to
the face; on a mapped cell it is read as h = |K| / |F| (cell volume over face
area, the width of a box cell), gamma_e = gamma_hat k(k+1)(1/h+ + 1/h-), with
h+ = h- on the boundary.

Surrogates.  Sec. 4 replaces a cell by a rectangle (box) whose width along
axis t is the mean length of the cell's edges along t (eq. avglength, edge
lengths taken as vertex distances), and solves the local problem of the
Cartesian SIPG form on that box (eq. schwarzproj).  Reading: the box's faces
see the surrogate widths of the neighbouring cells along the same axis (its
penalties and, as on Cartesian meshes, nothing else of the neighbours), and a
boundary face stays a boundary face.  The surrogate local matrix is then the
Cartesian cell block of a rectilinear patch of 3 (or 2 at the boundary) boxes
per axis, taken from ``sipg.assemble``.

Smoother (Sec. 4, eq. schwarzproj with the additive cell smoother):
x <- x + omega sum_K R_K^T Atilde_K^-1 R_K (b - A x) with the mapped A; the
multiplicative variant (Alg. multsmoother) takes the red-black colors of the
cells one after the other with the residual recomputed before each.

Pins (tests/test_oracle_mapped.py): on rectilinear vertex grids the mapped
matrix equals ``sipg.assemble`` and the surrogate solver equals the exact local
solver; on distorted meshes A is symmetric positive definite (gamma_hat = 4)
and reproduces linear functions with their boundary data exactly (A u_I = b,
which fixes volume, face normal, area element and consistency terms) and,
with the volume load, quadratics with their Laplacian (k >= 2, where every
integrand is a polynomial the rule integrates exactly); the right-hand side
equals ``sipg.rhs`` on rectilinear grids; the surrogate widths of affine cells
are their edge lengths; the multiplicative surrogate step equals the
sequential formula with explicit inverses, and the multiplicative V-cycle is
symmetric with reversed post-smoothing (and not without it).
"""
import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import gll_nodes, gauss_rule, lagrange_values, lagrange_derivatives
from .mesh import Mesh
from . import sipg


class MappedMesh:
    """Logically Cartesian mesh: ``ncells`` per axis and the vertex coordinates
    ``verts`` of shape (nverts, d), vertex (v_0, .., v_{d-1}) at index
    v_0 + (m_0 + 1) (v_1 + (m_1 + 1) v_2), x fastest."""

    def __init__(self, dim, k, ncells, verts, gamma_hat=1.0):
        self.dim, self.k, self.gamma_hat = dim, k, float(gamma_hat)
        self.ncells = tuple(int(m) for m in ncells)
        self.verts = np.asarray(verts, dtype=np.float64)
        nv = int(np.prod([m + 1 for m in self.ncells]))
        if self.verts.shape != (nv, dim):
            raise ValueError("vertex array must be (prod(m+1), dim)")

    n1 = property(lambda self: self.k + 1)
    dofs_per_cell = property(lambda self: self.n1 ** self.dim)
    ncells_total = property(lambda self: int(np.prod(self.ncells)))
    ndofs = property(lambda self: self.ncells_total * self.dofs_per_cell)

    def cells(self):
        for lin in range(self.ncells_total):
            yield self.cell_multi(lin)

    def cell_lin(self, c):
        lin, stride = 0, 1
        for a in range(self.dim):
            lin += c[a] * stride
            stride *= self.ncells[a]
        return lin

    def cell_multi(self, lin):
        c = []
        for a in range(self.dim):
            c.append(lin % self.ncells[a])
            lin //= self.ncells[a]
        return tuple(c)

    def cell_dofs(self, c):
        base = self.cell_lin(c) * self.dofs_per_cell
        return np.arange(base, base + self.dofs_per_cell)

    def vertex(self, v):
        idx, stride = 0, 1
        for a in range(self.dim):
            idx += v[a] * stride
            stride *= self.ncells[a] + 1
        return self.verts[idx]

    def corners(self, c):
        """Vertex coordinates of cell c, corner o (o_a in {0, 1}) at index
        sum_a o_a 2^a: array (2^d, d)."""
        out = np.zeros((2 ** self.dim, self.dim))
        for idx in range(2 ** self.dim):
            o = [(idx >> a) & 1 for a in range(self.dim)]
            out[idx] = self.vertex([c[a] + o[a] for a in range(self.dim)])
        return out


def multilinear_map(X, xi):
    """Points x(xi) and Jacobians J[p, b, a] = d x_b / d xi_a of the multilinear
    map through the corners X (2^d, d) at reference points xi (npts, d)."""
    xi = np.atleast_2d(xi)
    npts, d = xi.shape
    x = np.zeros((npts, d))
    J = np.zeros((npts, d, d))
    for idx in range(2 ** d):
        o = [(idx >> a) & 1 for a in range(d)]
        fac = [xi[:, a] if o[a] else 1.0 - xi[:, a] for a in range(d)]
        dfac = [np.ones(npts) if o[a] else -np.ones(npts) for a in range(d)]
        N = np.prod(fac, axis=0)
        x += N[:, None] * X[idx][None, :]
        for a in range(d):
            dN = dfac[a] * np.prod([fac[b] for b in range(d) if b != a], axis=0) if d > 1 else dfac[a]
            J[:, :, a] += dN[:, None] * X[idx][None, :]
    return x, J


class _Tab:
    def __init__(self, k):
        self.nodes = gll_nodes(k)
        self.xq, self.wq = gauss_rule(k + 1)
        self.V = lagrange_values(self.nodes, self.xq)
        self.D = lagrange_derivatives(self.nodes, self.xq)
        self.ev = [lagrange_values(self.nodes, [s]) for s in (0.0, 1.0)]
        self.ed = [lagrange_derivatives(self.nodes, [s]) for s in (0.0, 1.0)]


def _ref_basis(tab, d, fixed=None):
    """Reference points (x fastest), weights, basis values (npts, ndof) and
    reference gradients [a] (npts, ndof).  fixed = (t, side) puts axis t on
    the endpoint `side` (a face rule of the other axes)."""
    coords, wts, vals, ders = [], [], [], []
    for a in range(d):
        if fixed is not None and a == fixed[0]:
            coords.append(np.array([float(fixed[1])]))
            wts.append(np.ones(1))
            vals.append(tab.ev[fixed[1]])
            ders.append(tab.ed[fixed[1]])
        else:
            coords.append(tab.xq)
            wts.append(tab.wq)
            vals.append(tab.V)
            ders.append(tab.D)
    pts = sipg.tensor_points(coords)
    W = sipg.tensor(wts)
    Phi = sipg.tensor(vals)
    G = [sipg.tensor([ders[a] if a == t else vals[a] for a in range(d)]) for t in range(d)]
    return pts, W, Phi, G


def _phys_grad(J, G):
    """grad phi = J^-T grad_xi phi at every point: list over physical axes."""
    npts, d, _ = J.shape
    Jinv = np.linalg.inv(J)  # Jinv[p, a, b] = d xi_a / d x_b
    return [sum(Jinv[:, a, b][:, None] * G[a] for a in range(d)) for b in range(d)]


def cell_volume(mesh, c, tab):
    pts, W, _, _ = _ref_basis(tab, mesh.dim)
    _, J = multilinear_map(mesh.corners(c), pts)
    return float(np.sum(W * np.linalg.det(J)))


def _face_geometry(mesh, c, t, side, tab):
    """On the face xi_t = side of cell c: basis values, physical gradients,
    outward unit normal n (npts, d) and area weights dS (npts)."""
    d = mesh.dim
    pts, W, Phi, G = _ref_basis(tab, d, fixed=(t, side))
    _, J = multilinear_map(mesh.corners(c), pts)
    Jinv = np.linalg.inv(J)
    m = Jinv[:, t, :]                      # row t of J^-1 = J^-T e_t
    norm = np.linalg.norm(m, axis=1)
    sign = 1.0 if side == 1 else -1.0
    n = sign * m / norm[:, None]
    dS = W * np.abs(np.linalg.det(J)) * norm
    grad = _phys_grad(J, G)
    return Phi, grad, n, dS


def face_area(mesh, c, t, side, tab):
    return float(np.sum(_face_geometry(mesh, c, t, side, tab)[3]))


def cell_matrix(mesh, c, tab):
    """int_K grad phi_i . grad phi_iota on the mapped cell."""
    pts, W, _, G = _ref_basis(tab, mesh.dim)
    _, J = multilinear_map(mesh.corners(c), pts)
    grad = _phys_grad(J, G)
    w = W * np.linalg.det(J)
    return sum(g.T @ (w[:, None] * g) for g in grad)


def _dn(grad, n):
    return sum(n[:, b][:, None] * grad[b] for b in range(len(grad)))


def interior_face_matrix(mesh, ca, cb, t, tab, vol):
    """Face terms between ca (lower along t) and cb (upper): rows/cols
    [dofs of ca, dofs of cb]; n points from ca to cb."""
    Pa, ga, n, dS = _face_geometry(mesh, ca, t, 1, tab)
    Pb, gb, _, _ = _face_geometry(mesh, cb, t, 0, tab)
    area = float(np.sum(dS))
    ha, hb = vol[ca] / area, vol[cb] / area
    gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (1.0 / ha + 1.0 / hb)
    Jmp = np.hstack([Pa, -Pb])
    Dsum = np.hstack([_dn(ga, n), _dn(gb, n)])
    WJ = dS[:, None] * Jmp
    return 0.5 * gamma * (Jmp.T @ WJ) - 0.5 * (WJ.T @ Dsum) - 0.5 * (Dsum.T @ WJ)


def boundary_face_matrix(mesh, c, t, side, tab, vol):
    P, g, n, dS = _face_geometry(mesh, c, t, side, tab)
    h = vol[c] / float(np.sum(dS))
    gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (2.0 / h)
    dn = _dn(g, n)
    WP = dS[:, None] * P
    return gamma * (P.T @ WP) - WP.T @ dn - dn.T @ WP


def assemble(mesh):
    """Global SIPG matrix of the mapped mesh (CSR)."""
    d, tab = mesh.dim, _Tab(mesh.k)
    vol = {c: cell_volume(mesh, c, tab) for c in mesh.cells()}
    rows, cols, vals = [], [], []

    def add(dofs, M):
        idx = np.concatenate(dofs)
        rows.append(np.repeat(idx, len(idx)))
        cols.append(np.tile(idx, len(idx)))
        vals.append(M.ravel())

    for c in mesh.cells():
        add([mesh.cell_dofs(c)], cell_matrix(mesh, c, tab))
        for t in range(d):
            if c[t] + 1 < mesh.ncells[t]:
                cb = list(c)
                cb[t] += 1
                cb = tuple(cb)
                add([mesh.cell_dofs(c), mesh.cell_dofs(cb)], interior_face_matrix(mesh, c, cb, t, tab, vol))
            for side in (0, 1):
                if (side == 0 and c[t] == 0) or (side == 1 and c[t] == mesh.ncells[t] - 1):
                    add([mesh.cell_dofs(c)], boundary_face_matrix(mesh, c, t, side, tab, vol))
    N = mesh.ndofs
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def rhs_boundary(mesh, g):
    """Boundary part of the right-hand side of eq. (sipg) for Dirichlet data g:
    int_bdry (gamma_e g v - g d_n v), same quadrature and penalty as A."""
    d, tab = mesh.dim, _Tab(mesh.k)
    b = np.zeros(mesh.ndofs)
    for c in mesh.cells():
        for t in range(d):
            for side in (0, 1):
                if not ((side == 0 and c[t] == 0) or (side == 1 and c[t] == mesh.ncells[t] - 1)):
                    continue
                P, gr, n, dS = _face_geometry(mesh, c, t, side, tab)
                pts, _, _, _ = _ref_basis(tab, d, fixed=(t, side))
                xp, _ = multilinear_map(mesh.corners(c), pts)
                gp = g(xp)
                h = cell_volume(mesh, c, tab) / float(np.sum(dS))
                gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (2.0 / h)
                b[mesh.cell_dofs(c)] += gamma * (P.T @ (dS * gp)) - _dn(gr, n).T @ (dS * gp)
    return b


def rhs(mesh, f, g=None):
    """Right-hand side of eq. (sipg) on the mapped cells: int_Omega f v plus,
    for Dirichlet data g, the boundary terms of ``rhs_boundary``; the volume
    integral uses the operator's rule (k+1 Gauss points per axis, weights
    times det J).  f, g: callables on an (npts, d) array of physical points."""
    d, tab = mesh.dim, _Tab(mesh.k)
    pts, W, Phi, _ = _ref_basis(tab, d)
    b = np.zeros(mesh.ndofs)
    for c in mesh.cells():
        x, J = multilinear_map(mesh.corners(c), pts)
        b[mesh.cell_dofs(c)] += Phi.T @ (W * np.linalg.det(J) * f(x))
    if g is not None:
        b += rhs_boundary(mesh, g)
    return b


def interpolate(mesh, u):
    """Nodal interpolant: u at the images of the reference Gauss-Lobatto nodes."""
    d, nodes = mesh.dim, gll_nodes(mesh.k)
    ref = sipg.tensor_points([nodes] * d)
    out = np.zeros(mesh.ndofs)
    for c in mesh.cells():
        x, _ = multilinear_map(mesh.corners(c), ref)
        out[mesh.cell_dofs(c)] = u(x)
    return out


def surrogate_widths(mesh):
    """hbar[c] (d,): mean length of the cell's 2^(d-1) edges along each axis
    (eq. avglength, vertex distances)."""
    d = mesh.dim
    out = {}
    for c in mesh.cells():
        X = mesh.corners(c)
        hb = np.zeros(d)
        for t in range(d):
            lens = [np.linalg.norm(X[idx | (1 << t)] - X[idx]) for idx in range(2 ** d) if not (idx >> t) & 1]
            hb[t] = np.mean(lens)
        out[c] = hb
    return out


def surrogate_local_matrix(mesh, c, hbar):
    """Cartesian SIPG cell matrix of the surrogate box of cell c: the centre
    block of a rectilinear patch whose cells along axis t have the surrogate
    widths (along t) of c's neighbours and of c."""
    d = mesh.dim
    widths, centre = [], []
    for t in range(d):
        w = [hbar[c][t]]
        pos = 0
        if c[t] > 0:
            lo = list(c)
            lo[t] -= 1
            w.insert(0, hbar[tuple(lo)][t])
            pos = 1
        if c[t] < mesh.ncells[t] - 1:
            hi = list(c)
            hi[t] += 1
            w.append(hbar[tuple(hi)][t])
        widths.append(np.array(w))
        centre.append(pos)
    mini = Mesh(d, mesh.k, tuple(widths), mesh.gamma_hat)
    A = sipg.assemble(mini, rows_cells=[tuple(centre)])
    dofs = mini.cell_dofs(tuple(centre))
    return A[dofs][:, dofs].toarray()


class SurrogateCellSolvers:
    """LU factors of the surrogate local matrices of every cell."""

    def __init__(self, mesh):
        hbar = surrogate_widths(mesh)
        self.mesh = mesh
        self.lu = {c: sla.lu_factor(surrogate_local_matrix(mesh, c, hbar)) for c in mesh.cells()}

    def apply(self, r, color=None):
        """sum_K R_K^T Atilde_K^-1 R_K r over all cells, or over the cells of
        one red-black color (sum of the cell indices modulo 2)."""
        out = np.zeros_like(r)
        for c, f in self.lu.items():
            if color is not None and sum(c) % 2 != color:
                continue
            dofs = self.mesh.cell_dofs(c)
            out[dofs] = sla.lu_solve(f, r[dofs])
        return out


class ExactCellSolvers:
    """LU factors of the exact cell blocks R_K A R_K^T of the mapped matrix
    (the sACS smoother of Tab. cubedist25acp), with the interface of
    ``SurrogateCellSolvers``."""

    def __init__(self, mesh, A):
        A = A.tocsr()
        self.mesh = mesh
        self.lu = {}
        for c in mesh.cells():
            dofs = mesh.cell_dofs(c)
            self.lu[c] = sla.lu_factor(A[dofs][:, dofs].toarray())

    apply = SurrogateCellSolvers.apply


def surrogate_smooth(A, solvers, x, b, omega):
    """One additive step with the surrogate cell solvers (eq. schwarzproj)."""
    return x + omega * solvers.apply(b - A @ x)


def surrogate_mult_smooth(A, solvers, x, b, omega, reverse=False):
    """One multiplicative step (Alg. multsmoother, eq. coloredschwarz) with the
    surrogate cell solvers and the red-black coloring of the cells: the
    residual is recomputed before each color.  reverse runs black before red,
    which is how Sec. 4 symmetrises the V-cycle (post-smoothing in the reverse
    order of pre-smoothing)."""
    for color in ((1, 0) if reverse else (0, 1)):
        x = x + omega * solvers.apply(b - A @ x, color)
    return x


class MappedHierarchy:
    """Alg. (gmg) on mapped meshes (Sec. 4): ``meshes`` coarsest first, each the
    uniform refinement of the previous one on its cell maps (the fine cells are
    the images of the children of the coarse reference cell), so the spaces
    are nested.  The prolongation evaluates a coarse function at the fine
    Gauss-Lobatto nodes; in reference coordinates that is the embedding of the
    children, the same matrix as on a uniform Cartesian mesh of the same cell
    counts (``multigrid.prolongation`` of two such meshes).  Smoother on
    levels l >= 1: the additive cell smoother with the surrogate solvers
    (``surrogate_smooth``, omegas[l]); on level 0 dense LU of A_0.  Restriction
    is the transpose of the prolongation; the V-cycle is the one of
    ``multigrid.Hierarchy``.  smoother="multiplicative" replaces the additive
    step by ``surrogate_mult_smooth``, red before black in pre-smoothing and
    black before red in post-smoothing (Sec. 4: the reversed order makes the
    V-cycle symmetric, so that it can precondition CG).  local="exact" uses
    ``ExactCellSolvers`` instead of the surrogates."""

    def __init__(self, meshes, omegas, m_pre=1, m_post=1, smoother="additive", local="surrogate"):
        from .multigrid import prolongation
        self.meshes, self.L = meshes, len(meshes) - 1
        self.omegas, self.m_pre, self.m_post = list(omegas), m_pre, m_post
        self.smoother = smoother
        self.A = [assemble(m) for m in meshes]
        shapes = [Mesh(m.dim, m.k, tuple(np.full(n, 1.0 / n) for n in m.ncells), 1.0) for m in meshes]
        self.P = [None] + [prolongation(shapes[l - 1], shapes[l]) for l in range(1, self.L + 1)]
        if local == "exact":
            self.solvers = [None] + [ExactCellSolvers(m, self.A[l]) for l, m in enumerate(meshes) if l > 0]
        else:
            self.solvers = [None] + [SurrogateCellSolvers(m) for m in meshes[1:]]
        self.coarse_lu = sla.lu_factor(self.A[0].toarray())

    def vcycle(self, x, b, l=None):
        l = self.L if l is None else l
        if l == 0:
            return sla.lu_solve(self.coarse_lu, b)
        for _ in range(self.m_pre):
            x = self.smooth(l, x, b, False)
        bc = self.P[l].T @ (b - self.A[l] @ x)
        e = self.vcycle(np.zeros(self.meshes[l - 1].ndofs), bc, l - 1)
        x = x + self.P[l] @ e
        for _ in range(self.m_post):
            x = self.smooth(l, x, b, True)
        return x

    def smooth(self, l, x, b, post):
        if self.smoother == "multiplicative":
            return surrogate_mult_smooth(self.A[l], self.solvers[l], x, b, self.omegas[l], reverse=post)
        return surrogate_smooth(self.A[l], self.solvers[l], x, b, self.omegas[l])
