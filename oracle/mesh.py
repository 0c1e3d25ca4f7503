"""Rectilinear Cartesian meshes and the DoF numbering (oracle, test infrastructure only).

Sec. 2.1: cells are axis-aligned boxes; V_l is the direct sum of the cell
spaces (eq. discFEspace), so DoFs are numbered cell by cell.  Cells are
numbered lexicographically with x fastest and the DoFs of a cell by the
lexicographic multi-index i = sum_t i_t (k+1)^(t-1) of eq. (multiindex), again
x fastest.  Axis 0 is x.

A mesh is given by its per-axis cell widths (a rectilinear grid); the domain is
[0, sum h_x] x [0, sum h_y] (x [0, sum h_z]).  Coarser levels merge pairs of
neighbouring cells (the midpoint split of Sec. 2.1 read backwards).
"""
from dataclasses import dataclass
import itertools
import numpy as np


@dataclass
class Mesh:
    dim: int
    k: int
    widths: tuple          # per-axis 1-D arrays of cell widths
    gamma_hat: float = 1.0  # penalty factor of eq. (penalty)

    def __post_init__(self):
        self.widths = tuple(np.asarray(w, dtype=np.float64) for w in self.widths)
        if len(self.widths) != self.dim:
            raise ValueError("need one width array per axis")

    @property
    def n1(self):
        return self.k + 1

    @property
    def ncells(self):
        return tuple(len(w) for w in self.widths)

    @property
    def ncells_total(self):
        return int(np.prod(self.ncells))

    @property
    def dofs_per_cell(self):
        return self.n1 ** self.dim

    @property
    def ndofs(self):
        return self.ncells_total * self.dofs_per_cell

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

    def cells(self):
        """All cell multi-indices in lexicographic order (x fastest)."""
        rng = [range(m) for m in self.ncells]
        for c in itertools.product(*reversed(rng)):
            yield tuple(reversed(c))

    def cell_dofs(self, c):
        base = self.cell_lin(c) * self.dofs_per_cell
        return np.arange(base, base + self.dofs_per_cell)

    def local_multi(self, i):
        """Local multi-index of local DoF i (x fastest)."""
        out = []
        for _ in range(self.dim):
            out.append(i % self.n1)
            i //= self.n1
        return tuple(out)

    def offsets(self, axis):
        """Coordinates of the cell boundaries along ``axis``."""
        return np.concatenate(([0.0], np.cumsum(self.widths[axis])))


def uniform_mesh(dim, k, m, gamma_hat=1.0, length=1.0):
    """m cells per axis (int or per-axis tuple) of equal width on [0, length]^d."""
    ms = (m,) * dim if np.isscalar(m) else tuple(m)
    return Mesh(dim, k, tuple(np.full(mm, length / mm) for mm in ms), gamma_hat)


def coarsen(mesh):
    """Parent mesh: each coarse cell is the union of 2^d children (Sec. 2.1).
    Requires an even number of cells per axis with equal halves."""
    ws = []
    for w in mesh.widths:
        if len(w) % 2:
            raise ValueError("cannot coarsen an odd number of cells")
        a, b = w[0::2], w[1::2]
        if not np.allclose(a, b, rtol=1e-14, atol=0):
            raise ValueError("children of a coarse cell must be equal halves")
        ws.append(a + b)
    return Mesh(mesh.dim, mesh.k, tuple(ws), mesh.gamma_hat)


def refine(mesh):
    """Child mesh: split every cell at its midpoint (Sec. 2.1)."""
    ws = [np.repeat(w / 2.0, 2) for w in mesh.widths]
    return Mesh(mesh.dim, mesh.k, tuple(ws), mesh.gamma_hat)
