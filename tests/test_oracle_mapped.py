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


@pytest.mark.parametrize("d,k,m,levels", [(2, 2, 3, 1), (2, 3, 2, 1), (3, 2, 2, 1), (3, 3, 2, 0)])
def test_quadratics_are_reproduced_with_their_load(d, k, m, levels):
    """A quadratic u* composed with a multilinear map has degree <= 2 in every
    reference coordinate, so it lies in the mapped Q_k space for k >= 2, and
    every integrand of a(u*, v) and of the load (f v det J, grad u* . cof(J)
    grad_xi v, the Nanson face terms) is a polynomial of degree <= 2k + 1
    per axis, which k+1 Gauss points integrate exactly.  Consistency of SIPG
    then gives A u*_I = rhs(-Laplace u*, u*) to rounding.  A dropped det J in
    the load, a wrong sign of f or of a boundary term breaks it."""
    mm = _distorted(d, k, m, levels, 11)
    A = mapped.assemble(mm)
    if d == 2:
        u = lambda X: X[:, 0] ** 2 - 0.5 * X[:, 1] ** 2 + 0.3 * X[:, 0] * X[:, 1] + 0.7 * X[:, 0] - 0.2
        lap = 1.0
    else:
        u = lambda X: X[:, 0] ** 2 + 0.5 * X[:, 1] ** 2 - 2.5 * X[:, 2] ** 2 + 0.3 * X[:, 1] * X[:, 2] + 0.1
        lap = -2.0
    f = lambda X: np.full(len(X), -lap)
    b = mapped.rhs(mm, f, u)
    uI = mapped.interpolate(mm, u)
    res = np.linalg.norm(A @ uI - b)
    assert res <= 1e-11 * np.linalg.norm(b)
    # the load is small next to the boundary penalty terms, but not zero:
    # dropping it leaves a residual far above rounding
    assert np.linalg.norm(A @ uI - mapped.rhs_boundary(mm, u)) > 1e6 * max(res, 1e-300)


@pytest.mark.parametrize("d,k,ms", [(2, 2, (3, 4)), (3, 1, (2, 3, 2))])
def test_rectilinear_rhs_is_the_cartesian_rhs(d, k, ms):
    """On a rectilinear grid the mapped load and boundary terms equal the
    Cartesian ones of ``sipg.rhs`` (polynomial data, so both quadrature rules
    are exact and agree)."""
    cart, mm = _rect(d, k, ms, 13)
    f = lambda X: 1.0 + X[:, 0] - 0.5 * X[:, -1] ** 2
    g = lambda X: 0.3 - X[:, 0] * X[:, -1]
    b0 = sipg.rhs(cart, f, g)
    b1 = mapped.rhs(mm, f, g)
    assert np.linalg.norm(b1 - b0) <= 1e-12 * np.linalg.norm(b0)


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


def test_mapped_prolongation_is_nested():
    """The refined distorted mesh is the uniform refinement of the coarse one on
    its cell maps, and the prolongation is the embedding: the interpolant of a
    linear function (which lies in both mapped spaces) on the coarse mesh is
    carried to its interpolant on the fine mesh."""
    for d, k, m in ((2, 2, 3), (2, 3, 2), (3, 2, 2)):
        meshes = [_distorted(d, k, m, lev, 13) for lev in (0, 1)]
        hier = mapped.MappedHierarchy(meshes, [0.0, 0.5])
        coef = np.array([0.3, -1.1, 0.8][:d])
        u = lambda X: X @ coef - 0.4
        uc, uf = mapped.interpolate(meshes[0], u), mapped.interpolate(meshes[1], u)
        assert np.abs(hier.P[1] @ uc - uf).max() <= 1e-13 * np.abs(uf).max()


def test_mapped_hierarchy_on_rectilinear_grids_is_the_cartesian_vcycle():
    """On rectilinear vertex grids the surrogate solvers are the exact cell
    solvers and the mapped matrices the Cartesian ones, so the mapped V-cycle
    is the Cartesian V-cycle with the additive cell smoother (the oracle's
    multigrid.Hierarchy, pinned in test_oracle_mg.py)."""
    from oracle import multigrid
    from synthetic import random_vector
    for d, k, m in ((2, 2, 2), (3, 1, 2)):
        fine = Mesh(d, k, tuple(np.full(2 * m, 0.5 / m) for _ in range(d)), 4.0)
        cart = multigrid.Hierarchy(fine, 2, "cell", [0.0, 0.45], m_pre=2, m_post=1)
        meshes = [mapped.MappedMesh(d, k, (n,) * d, grid_vertices([np.full(n, 1.0 / n)] * d), 4.0)
                  for n in (m, 2 * m)]
        hier = mapped.MappedHierarchy(meshes, [0.0, 0.45], m_pre=2, m_post=1)
        b, x = random_vector(fine.ndofs, 0), random_vector(fine.ndofs, 1)
        ref = cart.vcycle(x.copy(), b)
        got = hier.vcycle(x.copy(), b)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_multiplicative_surrogate_step_against_explicit_inverses():
    """Alg. multsmoother with red-black cells: x1 = x + omega sum_red
    Atilde_K^-1 R_K (b - A x), x2 = x1 + omega sum_black Atilde_K^-1 R_K
    (b - A x1), built from explicit inverses of the surrogate local matrices;
    reversed, black goes first."""
    mm = _distorted(2, 2, 3, 1, 17)
    A = mapped.assemble(mm)
    sol = mapped.SurrogateCellSolvers(mm)
    hbar = mapped.surrogate_widths(mm)
    b, x = random_vector(mm.ndofs, 2), random_vector(mm.ndofs, 3)
    inv = {c: np.linalg.inv(mapped.surrogate_local_matrix(mm, c, hbar)) for c in mm.cells()}
    for reverse in (False, True):
        ref = x.copy()
        for color in ((1, 0) if reverse else (0, 1)):
            r = b - A @ ref
            dx = np.zeros_like(ref)
            for c in mm.cells():
                if sum(c) % 2 == color:
                    dofs = mm.cell_dofs(c)
                    dx[dofs] = inv[c] @ r[dofs]
            ref = ref + 0.7 * dx
        out = mapped.surrogate_mult_smooth(A, sol, x, b, 0.7, reverse=reverse)
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    # one color holding every cell reduces the multiplicative step to the additive one
    assert np.allclose(sol.apply(b), sol.apply(b, 0) + sol.apply(b, 1), rtol=0, atol=1e-14 * np.abs(sol.apply(b)).max())


def test_reversed_post_smoothing_makes_the_mapped_vcycle_symmetric():
    """Sec. 4: with the colors of post-smoothing in the reverse order of
    pre-smoothing the multiplicative V-cycle, as a linear map b -> MG(0, b),
    is symmetric (it can precondition CG); with the same order it is not."""
    meshes = [_distorted(2, 2, 2, lev, 19) for lev in (0, 1)]
    N = meshes[-1].ndofs
    for smoother in ("multiplicative", "additive"):
        h = mapped.MappedHierarchy(meshes, [0.0, 0.6], m_pre=2, m_post=2, smoother=smoother)
        B = np.column_stack([h.vcycle(np.zeros(N), e) for e in np.eye(N)])
        assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max(), smoother
    h = mapped.MappedHierarchy(meshes, [0.0, 0.6], m_pre=1, m_post=1, smoother="multiplicative")
    h.smooth = lambda l, x, b, post: mapped.surrogate_mult_smooth(h.A[l], h.solvers[l], x, b, 0.6, reverse=False)
    B = np.column_stack([h.vcycle(np.zeros(N), e) for e in np.eye(N)])
    assert np.abs(B - B.T).max() > 1e-4 * np.abs(B).max()


def test_exact_cell_solvers_equal_the_surrogates_on_rectilinear_grids():
    """The exact cell blocks of the mapped matrix and the surrogate boxes are
    built by separate routes (the mapped quadrature against a Cartesian
    mini-mesh); on a rectilinear grid both are the Cartesian cell block, and
    on a distorted mesh they differ."""
    _, mm = _rect(2, 3, (3, 4), 23)
    r = random_vector(mm.ndofs, 4)
    ex = mapped.ExactCellSolvers(mm, mapped.assemble(mm)).apply(r)
    su = mapped.SurrogateCellSolvers(mm).apply(r)
    assert np.abs(ex - su).max() <= 1e-11 * np.abs(su).max()
    md = _distorted(2, 3, 3, 1, 23)
    r = random_vector(md.ndofs, 4)
    ex = mapped.ExactCellSolvers(md, mapped.assemble(md)).apply(r)
    su = mapped.SurrogateCellSolvers(md).apply(r)
    assert np.abs(ex - su).max() > 1e-3 * np.abs(su).max()
