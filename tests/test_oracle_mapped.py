"""Pins of the mapped-cell SIPG oracle and the Cartesian surrogate solvers
(Sec. 4; oracle/mapped.py)."""
import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle import sipg, schwarz, mapped
from synthetic import distorted_vertices, grid_vertices, loguniform_widths, random_vector


def _rect(d, k, ms, seed, gamma_hat=1.3):
    rng = np.random.default_rng(seed)
    ws = loguniform_widths(rng, d, ms, 0.25, 4.0)
    return Mesh(d, k, ws, gamma_hat), mapped.MappedMesh(d, k, ms, grid_vertices(ws), gamma_hat)


def _distorted(d, k, m, levels, seed, gamma_hat=4.0, distortion=0.25):
    ms, V = distorted_vertices(d, m, levels, distortion, seed)
    return mapped.MappedMesh(d, k, ms, V, gamma_hat)


@pytest.mark.parametrize("d,k,ms", [(2, 1, (3, 4)), (2, 3, (4, 3)), (3, 2, (3, 2, 3))])
def test_rectilinear_vertices_give_the_cartesian_matrix(d, k, ms):
    """Cartesian limit: on a rectilinear vertex grid every map is a scaling,
    |K| / |F| is the width orthogonal to the face, and the mapped matrix is
    the Cartesian SIPG matrix (itself pinned in test_oracle_sipg.py)."""
    cart, mm = _rect(d, k, ms, 3)
    A0 = sipg.assemble(cart).toarray()
    A1 = mapped.assemble(mm).toarray()
    assert np.abs(A1 - A0).max() <= 1e-12 * np.abs(A0).max()


@pytest.mark.parametrize("d,k,m,levels", [(2, 1, 3, 1), (2, 3, 3, 1), (3, 1, 2, 1), (3, 2, 2, 1)])
def test_distorted_matrix_is_spd(d, k, m, levels):
    mm = _distorted(d, k, m, levels, 5)
    A = mapped.assemble(mm).toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


@pytest.mark.parametrize("d,k,m,levels", [(2, 1, 3, 1), (2, 3, 3, 1), (2, 4, 2, 1), (3, 1, 2, 1), (3, 3, 2, 1)])
def test_linear_functions_are_reproduced_on_distorted_meshes(d, k, m, levels):
    """A linear u* lies in the mapped space (a multilinear function of the
    reference coordinates), and SIPG is consistent: A u*_I equals the boundary
    right-hand side for g = u*, f = 0.  A wrong normal, area element, Jacobian
    transpose or consistency sign breaks the identity."""
    mm = _distorted(d, k, m, levels, 7)
    A = mapped.assemble(mm)
    coef = np.array([0.7, -1.3, 0.4][:d])
    u = lambda X: X @ coef + 0.25
    uI = mapped.interpolate(mm, u)
    b = mapped.rhs_boundary(mm, u)
    assert np.linalg.norm(A @ uI - b) <= 1e-11 * np.linalg.norm(b)


def test_undistorted_surrogate_is_the_exact_local_solver():
    """On a rectilinear mesh the surrogate box is the cell itself: the
    surrogate local matrix equals R_K A R_K^T for every cell."""
    cart, mm = _rect(3, 2, (3, 3, 2), 9)
    A = sipg.assemble(cart)
    hbar = mapped.surrogate_widths(mm)
    for c in mm.cells():
        assert np.allclose(hbar[c], [cart.widths[a][c[a]] for a in range(3)], rtol=1e-14, atol=0)
        dofs = cart.cell_dofs(c)
        ref = A[dofs][:, dofs].toarray()
        got = mapped.surrogate_local_matrix(mm, c, hbar)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_surrogate_widths_of_affine_and_trapezoid_cells():
    """eq. (avglength): a parallelogram's surrogate widths are its side lengths;
    a trapezoid with parallel sides 1 and 2 (height 1) has width 1.5 along the
    parallel sides and the mean of its two legs across."""
    V = np.array([[0.0, 0.0], [1.0, 0.0], [0.3, 1.0], [1.3, 1.0]])
    mm = mapped.MappedMesh(2, 1, (1, 1), V)
    hb = mapped.surrogate_widths(mm)[(0, 0)]
    assert np.allclose(hb, [1.0, np.hypot(0.3, 1.0)], rtol=1e-15)
    V = np.array([[0.0, 0.0], [2.0, 0.0], [0.5, 1.0], [1.5, 1.0]])
    mm = mapped.MappedMesh(2, 1, (1, 1), V)
    hb = mapped.surrogate_widths(mm)[(0, 0)]
    assert np.allclose(hb, [1.5, np.hypot(0.5, 1.0)], rtol=1e-15)


def test_surrogate_smoother_step_and_local_stability():
    """One surrogate ACS step equals x + omega sum_K R_K^T Atilde_K^-1 R_K r
    built from explicit inverses; the local stability constant of
    eq. (localstab), max over cells of lambda_max(Atilde_K^-1 A_K), is finite
    and, for a 25 % distortion, moderate (the surrogate is spectrally close)."""
    mm = _distorted(2, 3, 3, 1, 11)
    A = mapped.assemble(mm)
    sol = mapped.SurrogateCellSolvers(mm)
    hbar = mapped.surrogate_widths(mm)
    b, x = random_vector(mm.ndofs, 0), random_vector(mm.ndofs, 1)
    out = mapped.surrogate_smooth(A, sol, x, b, 0.5)
    r = b - A @ x
    ref = x.copy()
    eta = 0.0
    Ad = A.toarray()
    for c in mm.cells():
        dofs = mm.cell_dofs(c)
        At = mapped.surrogate_local_matrix(mm, c, hbar)
        ref[dofs] += 0.5 * np.linalg.solve(At, r[dofs])
        eta = max(eta, np.max(np.real(np.linalg.eigvals(np.linalg.solve(At, Ad[np.ix_(dofs, dofs)])))))
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    assert 1.0 < eta < 3.0
