"""Sec. 4 on the GPU: the matrix-free SIPG operator on mapped cells and the
additive cell smoother with Cartesian surrogate local solvers, against the
oracle (mapped-cell quadrature assembly, surrogate matrices by the Cartesian
assembly of the surrogate boxes, dense LU) on distorted meshes of the unit
square and cube and on rectilinear vertex grids (the Cartesian limit)."""
import numpy as np
import pytest

from oracle import mapped
from synthetic import distorted_vertices, grid_vertices, loguniform_widths, random_vector
from gpu_util import dev, host, rel, announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1910_11239_amd as fts  # noqa: E402

TOL = 1e-12

CASES = [("distorted", 2, 1, 3, 1), ("distorted", 2, 3, 3, 1), ("distorted", 2, 5, 2, 1), ("distorted", 2, 7, 2, 1),
         ("distorted", 2, 11, 2, 1), ("distorted", 2, 15, 2, 1),
         ("distorted", 3, 1, 2, 1), ("distorted", 3, 2, 2, 1), ("distorted", 3, 3, 2, 1), ("distorted", 3, 5, 1, 1),
         ("distorted", 2, 3, 8, 2), ("distorted", 3, 3, 4, 1),
         ("rect", 2, 4, (5, 3), 0), ("rect", 3, 3, (3, 4, 2), 0)]


def _mesh(kind, d, k, m, levels, seed=5):
    if kind == "distorted":
        ms, V = distorted_vertices(d, m, levels, 0.25, seed)
        return mapped.MappedMesh(d, k, ms, V, 4.0)
    rng = np.random.default_rng(seed)
    ws = loguniform_widths(rng, d, m, 0.25, 4.0)
    return mapped.MappedMesh(d, k, m, grid_vertices(ws), 1.3)


def _glevel(mm):
    return fts.MappedLevel(mm.dim, mm.k, mm.ncells, mm.verts, mm.gamma_hat)


@pytest.mark.parametrize("kind,d,k,m,levels", CASES)
def test_mapped_operator_and_residual(kind, d, k, m, levels):
    announce("mapped operator", kind, d, k, m, levels)
    mm = _mesh(kind, d, k, m, levels)
    A = mapped.assemble(mm)
    x, b = random_vector(mm.ndofs, 1), random_vector(mm.ndofs, 0)
    lv = _glevel(mm)
    y = dev(np.zeros(mm.ndofs))
    lv.apply(dev(x), y)
    assert rel(host(y), A @ x) < TOL
    r = dev(np.zeros(mm.ndofs))
    lv.residual(dev(b), dev(x), r)
    assert rel(host(r), b - A @ x) < TOL


@pytest.mark.parametrize("kind,d,k,m,levels", CASES)
def test_surrogate_cell_smoother(kind, d, k, m, levels):
    """Two sweeps x <- x + omega sum_K R_K^T Atilde_K^-1 R_K (b - A x) and the
    local-solver part alone; surrogate widths equal the oracle's."""
    announce("mapped smoother", kind, d, k, m, levels)
    mm = _mesh(kind, d, k, m, levels)
    A = mapped.assemble(mm)
    sol = mapped.SurrogateCellSolvers(mm)
    x, b = random_vector(mm.ndofs, 1), random_vector(mm.ndofs, 0)
    omega = 0.5
    x1 = mapped.surrogate_smooth(A, sol, x, b, omega)
    x2 = mapped.surrogate_smooth(A, sol, x1, b, omega)
    lv = _glevel(mm)
    hb = lv.surrogate_widths()
    hbo = mapped.surrogate_widths(mm)
    for c in mm.cells():
        assert np.allclose(hb[mm.cell_lin(c)], hbo[c], rtol=1e-14, atol=0)
    xg = dev(x)
    lv.schwarz_smooth(omega, dev(b), xg, nsweeps=1)
    assert rel(host(xg), x1) < TOL
    lv.schwarz_smooth(omega, dev(b), xg, nsweeps=1)
    assert rel(host(xg), x2) < TOL
    r = b - A @ x
    xa = dev(np.zeros(mm.ndofs))
    lv.schwarz_apply(1.0, dev(r), xa)
    assert rel(host(xa), sol.apply(r)) < TOL


def test_inverted_cell_is_refused():
    V = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])[[1, 0, 2, 3]]
    with pytest.raises(fts.FtsError, match="orientation"):
        fts.MappedLevel(2, 2, (1, 1), V, 4.0)
