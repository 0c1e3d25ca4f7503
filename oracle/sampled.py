"""The oracle's definitions evaluated on a few cells of a large mesh (test infrastructure only).

The residual of a cell depends on the cell and its face neighbours, and one
additive Schwarz step on a cell depends on the residual of the subdomains that
contain it (Sec. 2.3, eq. additiveschwarz).  So both can be computed exactly
for a sample of cells of a full-size mesh by assembling only the rows of the
SIPG matrix (``sipg.assemble(rows_cells=...)``) that these need and by
extracting and LU-factoring only the local matrices of the subdomains that
touch the sampled cells.  Same arithmetic as ``sipg`` and ``schwarz``.
"""
import itertools
import numpy as np
import scipy.linalg as sla

from .sipg import assemble
from .schwarz import patch_dofs


def residual_cells(mesh, x, b, cells):
    """r = b - A x on the given cells; returns {cell: r_K}."""
    A = assemble(mesh, rows_cells=cells)
    out = {}
    for c in cells:
        dofs = mesh.cell_dofs(c)
        out[tuple(c)] = b[dofs] - A[dofs] @ x
    return out


def _patches_touching(mesh, c, kind):
    if kind == "cell":
        return [("cell", tuple(c))]
    out = []
    for off in itertools.product((0, 1), repeat=mesh.dim):
        v = tuple(c[t] + off[t] for t in range(mesh.dim))
        if all(1 <= v[t] <= mesh.ncells[t] - 1 for t in range(mesh.dim)):
            out.append(("vertex", v))
    return out


def _sub_dofs(mesh, sub):
    kind, key = sub
    return mesh.cell_dofs(key) if kind == "cell" else patch_dofs(mesh, key)


def _sub_cells(mesh, sub):
    kind, key = sub
    if kind == "cell":
        return [key]
    return [tuple(key[t] - 1 + o[t] for t in range(mesh.dim))
            for o in itertools.product((0, 1), repeat=mesh.dim)]


def smooth_cells(mesh, x, b, omega, kind, cells):
    """One additive Schwarz step x + omega sum_j R_j^T A_j^-1 R_j (b - A x),
    evaluated on the given cells only; returns {cell: x_new_K}."""
    out = {}
    for c in cells:
        c = tuple(c)
        subs = _patches_touching(mesh, c, kind)
        region = sorted({cc for s in subs for cc in _sub_cells(mesh, s)}, key=mesh.cell_lin)
        A = assemble(mesh, rows_cells=region)
        r = np.zeros_like(x)
        for cc in region:
            dofs = mesh.cell_dofs(cc)
            r[dofs] = b[dofs] - A[dofs] @ x
        dofs_c = mesh.cell_dofs(c)
        corr = np.zeros(len(dofs_c))
        for s in subs:
            idx = _sub_dofs(mesh, s)
            Aj = A[idx][:, idx].toarray()
            sol = sla.lu_solve(sla.lu_factor(Aj), r[idx])
            pos = {g: i for i, g in enumerate(idx)}
            corr += sol[[pos[g] for g in dofs_c]]
        out[c] = x[dofs_c] + omega * corr
    return out
