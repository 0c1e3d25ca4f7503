"""Pins of the oracle's SIPG matrix (eq. bfsipg, penalty, jumpavgscalar).

Each pin comes from outside the oracle: symmetry/positivity of the form,
consistency of SIPG on polynomials, a hand-derived closed form for the energy
of cell indicators (the only term that survives for piecewise constants is the
penalty, weighted 1/2 inside by the 1/sqrt(2) average and 1 on the boundary),
the optimal L2 convergence order k+1, and the separability identity between
the quadrature matrix and the independent 1-D formulas of Sec. 3.2.
"""
import numpy as np
import pytest

from oracle.mesh import Mesh, uniform_mesh
from oracle import sipg, onedim
from oracle.schwarz import patch_dofs, interior_vertices
from synthetic import loguniform_widths


def _mesh(d, k, ms, seed, gamma_hat=1.3):
    rng = np.random.default_rng(seed)
    return Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0), gamma_hat)


CASES = [(1, 3, (5,)), (2, 1, (3, 4)), (2, 3, (4, 3)), (3, 2, (3, 2, 3)), (3, 1, (2, 3, 2))]


@pytest.mark.parametrize("d,k,ms", CASES)
def test_symmetric_positive_definite(d, k, ms):
    A = sipg.assemble(_mesh(d, k, ms, 1)).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("d,k,ms", CASES)
def test_consistency_on_polynomials(d, k, ms):
    """SIPG is consistent: for u in Q_k (so u_I = u) with boundary data g = u,
    A u_I equals the right-hand side of eq. (sipg) with f = -Lap u."""
    mesh = _mesh(d, k, ms, 2)
    rng = np.random.default_rng(5)
    # random polynomial of degree <= k per variable, product form + sum form
    cs = rng.uniform(-1, 1, (d, k + 1))

    def u(X):
        out = np.ones(len(X))
        for a in range(d):
            out *= np.polynomial.polynomial.polyval(X[:, a] / 3.0, cs[a])
        return out + X[:, 0] ** k

    def f(X):
        tot = np.zeros(len(X))
        for t in range(d):
            dd = np.polynomial.polynomial.polyder(cs[t], 2) / 9.0
            term = np.polynomial.polynomial.polyval(X[:, t] / 3.0, dd)
            for a in range(d):
                if a != t:
                    term = term * np.polynomial.polynomial.polyval(X[:, a] / 3.0, cs[a])
            tot += term
        tot += k * (k - 1) * X[:, 0] ** (k - 2) if k >= 2 else 0.0
        return -tot

    A = sipg.assemble(mesh)
    b = sipg.rhs(mesh, f, u)
    uI = sipg.interpolate(mesh, u)
    assert np.abs(A @ uI - b).max() <= 1e-11 * max(1.0, np.abs(b).max())


@pytest.mark.parametrize("d,k,ms", CASES)
def test_indicator_energy_closed_form(d, k, ms):
    """For u = 1 on cell K (0 elsewhere) only the penalty term survives:
    a(1_K, 1_K) = sum_{interior faces} gamma_e/2 |e| + sum_{boundary faces} gamma_e |e|
    and for face neighbours a(1_K, 1_K') = -gamma_e/2 |e|."""
    mesh = _mesh(d, k, ms, 3)
    A = sipg.assemble(mesh)
    kk = mesh.gamma_hat * k * (k + 1)
    for c in mesh.cells():
        e = np.zeros(mesh.ndofs)
        e[mesh.cell_dofs(c)] = 1.0
        h = [mesh.widths[a][c[a]] for a in range(d)]
        expect = 0.0
        for t in range(d):
            area = np.prod([h[a] for a in range(d) if a != t])
            for s in (-1, 1):
                nb = c[t] + s
                if 0 <= nb < mesh.ncells[t]:
                    g = kk * (1 / h[t] + 1 / mesh.widths[t][nb])
                    expect += g / 2 * area
                    cn = list(c)
                    cn[t] = nb
                    en = np.zeros(mesh.ndofs)
                    en[mesh.cell_dofs(tuple(cn))] = 1.0
                    assert abs(en @ (A @ e) + g / 2 * area) < 1e-10 * g * area
                else:
                    expect += kk * (2 / h[t]) * area
        assert abs(e @ (A @ e) - expect) < 1e-10 * expect


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2])
def test_l2_convergence_order(k):
    """Discrete solution of -Lap u = f, u = 0 on the boundary of [0,1]^2, with
    u = sin(pi x) sin(pi y): L2 error decays like h^(k+1) (SIPG theory)."""
    u = lambda X: np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
    f = lambda X: 2 * np.pi ** 2 * u(X)
    errs = []
    for m in (4, 8, 16):
        mesh = uniform_mesh(2, k, m, gamma_hat=1.0)
        A = sipg.assemble(mesh).tocsc()
        import scipy.sparse.linalg as spla
        uh = spla.spsolve(A, sipg.rhs(mesh, f))
        errs.append(sipg.l2_error(mesh, uh, u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 1 - 0.2, rates


def _kron_local(mesh, chains):
    ref = onedim.Ref1D(mesh.k)
    As, Ms = [], []
    for a, (ws, lo, hi) in enumerate(chains):
        A1, M1 = onedim.chain_operator(ref, ws, lo, hi, mesh.gamma_hat)
        As.append(A1)
        Ms.append(M1)
    return onedim.kron_sum(As, Ms)


@pytest.mark.parametrize("d,k,ms", [(2, 3, (4, 3)), (3, 2, (3, 3, 4)), (2, 5, (3, 3))])
def test_separability_cells_and_patches(d, k, ms):
    """R_j A R_j^T of the quadrature matrix equals the Kronecker sum of the
    1-D cell/patch factors (eq. KDseparable with eq. 1Dsipg / 1DsipgVP),
    interior and boundary subdomains, random rectilinear widths."""
    mesh = _mesh(d, k, ms, 4)
    A = sipg.assemble(mesh).tocsr()
    for c in mesh.cells():
        idx = mesh.cell_dofs(c)
        G = _kron_local(mesh, [onedim.axis_chain(mesh, a, c[a], 1) for a in range(d)])
        assert np.abs(A[idx][:, idx].toarray() - G).max() < 1e-12 * np.abs(G).max()
    for v in interior_vertices(mesh):
        idx = patch_dofs(mesh, v)
        G = _kron_local(mesh, [onedim.axis_chain(mesh, a, v[a] - 1, 2) for a in range(d)])
        assert np.abs(A[idx][:, idx].toarray() - G).max() < 1e-12 * np.abs(G).max()


@pytest.mark.parametrize("d,k,ms", CASES)
def test_separability_global(d, k, ms):
    """On a rectilinear mesh the whole matrix is the Kronecker sum of the global
    block-tridiagonal 1-D matrices, up to the cell-major permutation."""
    mesh = _mesh(d, k, ms, 6)
    A = sipg.assemble(mesh).toarray()
    G = _kron_local(mesh, [(mesh.widths[a], None, None) for a in range(d)])
    perm = onedim.to_axis_tensor(mesh, np.arange(mesh.ndofs, dtype=float)).ravel().astype(int)
    assert np.abs(A[np.ix_(perm, perm)] - G).max() < 1e-12 * np.abs(G).max()


@pytest.mark.parametrize("d,k,ms", CASES)
def test_global_fastdiag_solve(d, k, ms):
    mesh = _mesh(d, k, ms, 7)
    A = sipg.assemble(mesh)
    b = np.random.default_rng(0).uniform(-1, 1, mesh.ndofs)
    u = onedim.global_fastdiag_solve(mesh, b)
    assert np.linalg.norm(A @ u - b) < 1e-12 * np.linalg.norm(b) * np.linalg.cond(A.toarray())


def test_rows_subset_matches_full():
    mesh = _mesh(3, 2, (3, 4, 3), 8)
    A = sipg.assemble(mesh).tocsr()
    cells = [(1, 2, 1), (0, 0, 0), (2, 3, 2)]
    As = sipg.assemble(mesh, rows_cells=cells).tocsr()
    for c in cells:
        idx = mesh.cell_dofs(c)
        assert np.abs((A[idx] - As[idx]).toarray()).max() < 1e-13


def test_penalty_part_is_gamma_derivative():
    mesh = _mesh(2, 2, (3, 3), 9, gamma_hat=1.7)
    A1 = sipg.assemble(mesh).toarray()
    P = sipg.assemble(mesh, penalty_only=True).toarray()
    mesh.gamma_hat = 2.2
    A2 = sipg.assemble(mesh).toarray()
    # A is affine in gamma_hat: A(g) = A0 + g * P/g0
    assert np.abs((A2 - A1) - (2.2 - 1.7) * P / 1.7).max() < 1e-11 * np.abs(A1).max()
