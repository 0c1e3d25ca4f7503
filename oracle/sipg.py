"""Global SIPG matrix by d-dimensional quadrature (oracle, test infrastructure only).

Written directly from the interior penalty form eq. (bfsipg) of Sec. 2.1:

    a(u, v) = sum_K int_K grad u . grad v
            + sum_e int_e ( gamma_e {u n}.{v n} - {grad u}.{v n} - {u n}.{grad v} )

with the averaging operator {v} = (v+ + v-)/sqrt(2) on interior faces
(eq. jumpavgscalar) and {v} = v on boundary faces (eq. avgbdry), and the penalty
gamma_e = gamma_hat k (k+1) (1/h+ + 1/h-) of eq. (penalty), h+- being the cell
lengths orthogonal to the face and h+ = h- = h on the boundary.

Written out for the two cells a (lower coordinate) and b (upper coordinate) of
an interior face with n = +e_t, the 1/sqrt(2) average gives
    {u n}.{v n}     = (u_a - u_b)(v_a - v_b) / 2
    {grad u}.{v n}  = (d_n u_a + d_n u_b)(v_a - v_b) / 2
and on a boundary face with outward normal n
    {u n}.{v n} = u v,   {grad u}.{v n} = d_n u v.

No 1-D factorisation is used: the cell and face matrices are integrated with a
tensor Gauss rule of k+1 points per axis (exact for these polynomial
integrands) over the d-dimensional cell or (d-1)-dimensional face.

Pins: symmetry and positive definiteness, consistency on polynomials
(A u_I = F(f, g) for u in Q_k, which fixes bulk, consistency and boundary
terms), the closed-form energy of a cell indicator (which fixes the penalty
weight gamma_e/2 on interior and gamma_e on boundary faces), optimal L2
convergence h^(k+1) of the discrete solution, and the separability identity
against the independent 1-D formulas (tests/test_oracle_sipg.py).
"""
import numpy as np
import scipy.sparse as sp

from .basis import gll_nodes, gauss_rule, lagrange_values, lagrange_derivatives


def tensor(factors):
    """kron(F_{d-1}, ..., F_1, F_0): axis 0 (x) is the fastest index."""
    out = np.ones((1, 1)) if np.ndim(factors[0]) == 2 else np.ones(1)
    for F in reversed(factors):
        out = np.kron(out, F)
    return out


def tensor_points(coords):
    """Tensor grid of per-axis coordinates, x fastest: array (npts, d)."""
    grids = np.meshgrid(*reversed(coords), indexing="ij")
    return np.stack([g.ravel() for g in reversed(grids)], axis=1)


class _Tables:
    def __init__(self, k, nq):
        self.nodes = gll_nodes(k)
        self.xq, self.wq = gauss_rule(nq)
        self.V = lagrange_values(self.nodes, self.xq)
        self.D = lagrange_derivatives(self.nodes, self.xq)
        self.end_val = [lagrange_values(self.nodes, [s]) for s in (0.0, 1.0)]
        self.end_der = [lagrange_derivatives(self.nodes, [s]) for s in (0.0, 1.0)]


def cell_bulk_matrix(mesh, c, tab):
    """int_K grad phi_i . grad phi_iota over cell c, d-dimensional quadrature."""
    d = mesh.dim
    h = [mesh.widths[a][c[a]] for a in range(d)]
    W = tensor([tab.wq * h[a] for a in range(d)])
    K = 0.0
    for t in range(d):
        G = tensor([tab.D / h[a] if a == t else tab.V for a in range(d)])
        K = K + G.T @ (W[:, None] * G)
    return K


def _face_traces(mesh, c, t, side, tab):
    """Traces on the face xi_t = side of cell c: values, d/dx_t, face weights."""
    d = mesh.dim
    h = [mesh.widths[a][c[a]] for a in range(d)]
    val = tensor([tab.end_val[side] if a == t else tab.V for a in range(d)])
    der = tensor([tab.end_der[side] / h[t] if a == t else tab.V for a in range(d)])
    W = tensor([np.ones(1) if a == t else tab.wq * h[a] for a in range(d)])
    return val, der, W


def interior_face_matrix(mesh, ca, cb, t, tab):
    """Face matrix [test, trial] on the face between ca (lower) and cb (upper)
    along axis t, rows/cols ordered [dofs of ca, dofs of cb]."""
    va, da, W = _face_traces(mesh, ca, t, 1, tab)
    vb, db, _ = _face_traces(mesh, cb, t, 0, tab)
    ha, hb = mesh.widths[t][ca[t]], mesh.widths[t][cb[t]]
    gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (1.0 / ha + 1.0 / hb)
    J = np.hstack([va, -vb])          # jump u_a - u_b
    Dsum = np.hstack([da, db])        # d_n u_a + d_n u_b with n = +e_t
    WJ = W[:, None] * J
    return 0.5 * gamma * (J.T @ WJ) - 0.5 * (WJ.T @ Dsum) - 0.5 * (Dsum.T @ WJ)


def boundary_face_matrix(mesh, c, t, side, tab):
    """Face matrix on the boundary face xi_t = side of cell c."""
    v, dx, W = _face_traces(mesh, c, t, side, tab)
    dn = dx if side == 1 else -dx      # outward normal derivative
    h = mesh.widths[t][c[t]]
    gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (2.0 / h)
    Wv = W[:, None] * v
    return gamma * (v.T @ Wv) - Wv.T @ dn - dn.T @ Wv


def assemble(mesh, rows_cells=None, penalty_only=False):
    """Global SIPG matrix as scipy CSR (N x N).

    rows_cells: optional iterable of cell multi-indices; only the rows of
    those cells are assembled (all columns kept), for local computations on
    large meshes.  penalty_only: assemble only the penalty term (the
    derivative of A with respect to gamma_hat, times gamma_hat).
    """
    d, tab = mesh.dim, _Tables(mesh.k, mesh.k + 1)
    keep = None if rows_cells is None else {tuple(c) for c in rows_cells}
    rows, cols, vals = [], [], []

    def add(blocks_dofs, mat, owners):
        if keep is not None and not any(o in keep for o in owners):
            return
        idx = np.concatenate(blocks_dofs)
        if keep is not None:
            mask = np.concatenate([np.full(len(b), o in keep) for b, o in zip(blocks_dofs, owners)])
        else:
            mask = np.ones(len(idx), dtype=bool)
        r = np.repeat(idx[mask], len(idx))
        cidx = np.tile(idx, int(mask.sum()))
        rows.append(r)
        cols.append(cidx)
        vals.append(mat[mask].ravel())

    if keep is None:
        touched = list(mesh.cells())
    else:
        touched = set()
        for c in keep:
            touched.add(c)
            for t in range(d):
                for s in (-1, 1):
                    nb = list(c)
                    nb[t] += s
                    if 0 <= nb[t] < mesh.ncells[t]:
                        touched.add(tuple(nb))
        touched = sorted(touched, key=mesh.cell_lin)

    for c in touched:
        if not penalty_only and (keep is None or c in keep):
            add([mesh.cell_dofs(c)], cell_bulk_matrix(mesh, c, tab), [c])
        for t in range(d):
            if c[t] + 1 < mesh.ncells[t]:
                cb = list(c)
                cb[t] += 1
                cb = tuple(cb)
                F = (_penalty_part(mesh, c, cb, t, tab) if penalty_only
                     else interior_face_matrix(mesh, c, cb, t, tab))
                add([mesh.cell_dofs(c), mesh.cell_dofs(cb)], F, [c, cb])
            for side in (0, 1):
                on_bdry = (side == 0 and c[t] == 0) or (side == 1 and c[t] == mesh.ncells[t] - 1)
                if on_bdry and (keep is None or c in keep):
                    F = (_penalty_part_bdry(mesh, c, t, side, tab) if penalty_only
                         else boundary_face_matrix(mesh, c, t, side, tab))
                    add([mesh.cell_dofs(c)], F, [c])
    N = mesh.ndofs
    if not rows:
        return sp.csr_matrix((N, N))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsr()


def _penalty_part(mesh, ca, cb, t, tab):
    va, _, W = _face_traces(mesh, ca, t, 1, tab)
    vb, _, _ = _face_traces(mesh, cb, t, 0, tab)
    ha, hb = mesh.widths[t][ca[t]], mesh.widths[t][cb[t]]
    gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (1.0 / ha + 1.0 / hb)
    J = np.hstack([va, -vb])
    return 0.5 * gamma * (J.T @ (W[:, None] * J))


def _penalty_part_bdry(mesh, c, t, side, tab):
    v, _, W = _face_traces(mesh, c, t, side, tab)
    h = mesh.widths[t][c[t]]
    gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (2.0 / h)
    return gamma * (v.T @ (W[:, None] * v))


def rhs(mesh, f, g=None, nq=None):
    """Right-hand side of eq. (sipg): int f v + int_bdry (gamma_e g v - g d_n v).
    f, g: callables on an (npts, d) array of physical points."""
    d = mesh.dim
    nq = nq or mesh.k + 3
    tab = _Tables(mesh.k, nq)
    b = np.zeros(mesh.ndofs)
    for c in mesh.cells():
        h = [mesh.widths[a][c[a]] for a in range(d)]
        x0 = [mesh.offsets(a)[c[a]] for a in range(d)]
        pts = tensor_points([x0[a] + h[a] * tab.xq for a in range(d)])
        Phi = tensor([tab.V] * d)
        W = tensor([tab.wq * h[a] for a in range(d)])
        dofs = mesh.cell_dofs(c)
        b[dofs] += Phi.T @ (W * f(pts))
        if g is None:
            continue
        for t in range(d):
            for side in (0, 1):
                if not ((side == 0 and c[t] == 0) or (side == 1 and c[t] == mesh.ncells[t] - 1)):
                    continue
                v, dx, Wf = _face_traces(mesh, c, t, side, tab)
                dn = dx if side == 1 else -dx
                coords = [np.array([x0[a] + side * h[a]]) if a == t else x0[a] + h[a] * tab.xq
                          for a in range(d)]
                gp = g(tensor_points(coords))
                gamma = mesh.gamma_hat * mesh.k * (mesh.k + 1) * (2.0 / h[t])
                b[dofs] += gamma * (v.T @ (Wf * gp)) - dn.T @ (Wf * gp)
    return b


def interpolate(mesh, u):
    """Nodal interpolant: coefficient = u at the cell's GLL nodes (Lagrange basis)."""
    d = mesh.dim
    nodes = gll_nodes(mesh.k)
    out = np.zeros(mesh.ndofs)
    for c in mesh.cells():
        h = [mesh.widths[a][c[a]] for a in range(d)]
        x0 = [mesh.offsets(a)[c[a]] for a in range(d)]
        out[mesh.cell_dofs(c)] = u(tensor_points([x0[a] + h[a] * nodes for a in range(d)]))
    return out


def l2_error(mesh, coeffs, u, nq=None):
    """|| u_h - u ||_L2 with a (k+3)-point tensor Gauss rule per cell."""
    d = mesh.dim
    nq = nq or mesh.k + 3
    tab = _Tables(mesh.k, nq)
    Phi = tensor([tab.V] * d)
    err2 = 0.0
    for c in mesh.cells():
        h = [mesh.widths[a][c[a]] for a in range(d)]
        x0 = [mesh.offsets(a)[c[a]] for a in range(d)]
        pts = tensor_points([x0[a] + h[a] * tab.xq for a in range(d)])
        W = tensor([tab.wq * h[a] for a in range(d)])
        diff = Phi @ coeffs[mesh.cell_dofs(c)] - u(pts)
        err2 += float(np.sum(W * diff * diff))
    return np.sqrt(err2)
