"""Pins of the oracle's sampled evaluation (``oracle/sampled.py``).

The residual of a cell and one additive Schwarz step restricted to a cell are
fixed by the global definitions (eq. bfsipg, eq. additiveschwarz): on meshes
small enough to assemble whole, the sampled values must equal the rows of the
full residual b - A x and of the full smoother output, for corner, edge, face
and interior cells, cell and vertex-patch subdomains, random rectilinear
widths.  The full definitions are pinned independently in test_oracle_sipg.py
and test_oracle_schwarz.py.
"""
import itertools

import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle import sipg, schwarz, sampled
from synthetic import loguniform_widths, random_vector


def _mesh(d, k, ms, seed):
    rng = np.random.default_rng(seed)
    return Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0), 1.1)


def _sample_cells(mesh):
    """Every corner, and one edge, face and interior cell where they exist."""
    ms = mesh.ncells
    cells = set(itertools.product(*[(0, m - 1) for m in ms]))
    mid = tuple(m // 2 for m in ms)
    cells.add(mid)
    for t in range(mesh.dim):
        c = list(mid)
        c[t] = 0
        cells.add(tuple(c))
        c = list(mid)
        c[t] = ms[t] - 1
        c[(t + 1) % mesh.dim] = 0
        cells.add(tuple(c))
    return sorted(cells)


@pytest.mark.parametrize("d,k,ms", [(2, 3, (5, 4)), (3, 2, (4, 3, 5)), (3, 3, (3, 4, 3))])
def test_residual_cells_equal_full_residual(d, k, ms):
    m = _mesh(d, k, ms, 31)
    A = sipg.assemble(m)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    full = b - A @ x
    cells = _sample_cells(m)
    got = sampled.residual_cells(m, x, b, cells)
    assert set(got) == set(cells)
    for c in cells:
        ref = full[m.cell_dofs(c)]
        assert np.abs(got[c] - ref).max() <= 1e-13 * np.abs(full).max(), c


@pytest.mark.parametrize("kind", ["cell", "vertex"])
@pytest.mark.parametrize("d,k,ms", [(2, 3, (5, 4)), (3, 2, (4, 3, 5))])
def test_smooth_cells_equal_full_smoother(kind, d, k, ms):
    m = _mesh(d, k, ms, 32)
    A = sipg.assemble(m)
    subs = schwarz.cell_subdomains(m) if kind == "cell" else schwarz.vertex_patch_subdomains(m)
    sol = schwarz.ExactLocalSolvers(A, subs, cache=False)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    omega = 0.7 if kind == "cell" else 0.3
    full = schwarz.additive_smooth(A, sol, x, b, omega)
    cells = _sample_cells(m)
    got = sampled.smooth_cells(m, x, b, omega, kind, cells)
    assert set(got) == set(cells)
    for c in cells:
        ref = full[m.cell_dofs(c)]
        assert np.abs(got[c] - ref).max() <= 1e-13 * np.abs(full).max(), c
