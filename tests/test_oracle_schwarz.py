"""Pins of the oracle's Schwarz smoothers (Sec. 2.3, Sec. 3.2)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.mesh import Mesh, uniform_mesh
from oracle import sipg, onedim, schwarz
from synthetic import loguniform_widths, random_vector


def _mesh(d, k, ms, seed, gamma_hat=1.0):
    rng = np.random.default_rng(seed)
    return Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0), gamma_hat)


@pytest.mark.parametrize("d,k", [(1, 3), (2, 2), (3, 2), (2, 5)])
def test_one_cell_mesh_cell_smoother_is_exact(d, k):
    """A single cell is the whole space: one ACS step with omega = 1 solves."""
    mesh = _mesh(d, k, (1,) * d, 1)
    A = sipg.assemble(mesh)
    sol = schwarz.ExactLocalSolvers(A, schwarz.cell_subdomains(mesh), cache=False)
    rng = np.random.default_rng(0)
    b, x = rng.uniform(-1, 1, mesh.ndofs), rng.uniform(-1, 1, mesh.ndofs)
    x1 = schwarz.additive_smooth(A, sol, x, b, 1.0)
    assert np.linalg.norm(A @ x1 - b) < 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("d,k", [(1, 4), (2, 3), (3, 2)])
def test_one_patch_mesh_vertex_smoother_is_exact(d, k):
    """The 2^d-cell mesh is one vertex patch (coarse mesh of Sec. 2.4):
    one AVS step with omega = 1 solves."""
    mesh = _mesh(d, k, (2,) * d, 2)
    A = sipg.assemble(mesh)
    subs = schwarz.vertex_patch_subdomains(mesh)
    assert len(subs) == 1 and sorted(subs[0]) == list(range(mesh.ndofs))
    sol = schwarz.ExactLocalSolvers(A, subs, cache=False)
    rng = np.random.default_rng(1)
    b, x = rng.uniform(-1, 1, mesh.ndofs), rng.uniform(-1, 1, mesh.ndofs)
    x1 = schwarz.additive_smooth(A, sol, x, b, 1.0)
    assert np.linalg.norm(A @ x1 - b) < 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("kind", ["cell", "vertex"])
def test_ritz_projection_properties(kind):
    """P_j = R_j^T A_j^-1 R_j A is an A-orthogonal projection onto V_j (eq. ritzproj)."""
    mesh = _mesh(2, 2, (3, 3), 3)
    A = sipg.assemble(mesh).toarray()
    subs = schwarz.cell_subdomains(mesh) if kind == "cell" else schwarz.vertex_patch_subdomains(mesh)
    for idx in subs[:3]:
        R = np.zeros((len(idx), mesh.ndofs))
        R[np.arange(len(idx)), idx] = 1
        P = R.T @ np.linalg.solve(R @ A @ R.T, R @ A)
        assert np.abs(P @ P - P).max() < 1e-11
        assert np.abs(A @ P - (A @ P).T).max() < 1e-10 * np.abs(A).max()
        # a(P u, v) = a(u, v) for v in V_j
        u = np.random.default_rng(4).uniform(-1, 1, mesh.ndofs)
        assert np.abs(R @ A @ (P @ u) - R @ A @ u).max() < 1e-10 * np.abs(A).max()


@pytest.mark.parametrize("d,k,ms", [(2, 3, (4, 3)), (3, 2, (3, 3, 2))])
def test_fast_diagonalisation_equals_exact_local_solve(d, k, ms):
    """Independent path (Sec. 3.2): 1-D generalized eigenproblems (DSYGV semantics)
    give S^T M S = I, S^T A S = Lambda > 0, and (S x S) Lambda^-1 (S x S)^T r
    equals the dense-LU local solve for every cell and vertex patch."""
    mesh = _mesh(d, k, ms, 5, gamma_hat=1.25)
    A = sipg.assemble(mesh)
    ref = onedim.Ref1D(k)
    rng = np.random.default_rng(2)
    for kind in ("cell", "vertex"):
        if kind == "cell":
            keys = list(mesh.cells())
            subs = schwarz.cell_subdomains(mesh)
            chains = lambda key: [onedim.axis_chain(mesh, a, key[a], 1) for a in range(d)]
        else:
            keys = list(schwarz.interior_vertices(mesh))
            subs = schwarz.vertex_patch_subdomains(mesh)
            chains = lambda key: [onedim.axis_chain(mesh, a, key[a] - 1, 2) for a in range(d)]
        sol = schwarz.ExactLocalSolvers(A, subs, cache=False)
        for j, key in enumerate(keys):
            Ss, lams = [], []
            for ws, lo, hi in chains(key):
                A1, M1 = onedim.chain_operator(ref, ws, lo, hi, mesh.gamma_hat)
                lam, S = sla.eigh(A1, M1)
                assert np.abs(S.T @ M1 @ S - np.eye(len(lam))).max() < 1e-12
                assert np.abs(S.T @ A1 @ S - np.diag(lam)).max() < 1e-10 * lam.max()
                assert lam.min() > 0
                Ss.append(S)
                lams.append(lam)
            r = rng.uniform(-1, 1, len(subs[j]))
            Zk = np.ones((1, 1))
            for a in reversed(range(d)):
                Zk = np.kron(Zk, Ss[a])
            Lam = onedim.kron_sum([np.diag(l) for l in lams], [np.eye(len(l)) for l in lams]).diagonal()
            fd = Zk @ ((Zk.T @ r) / Lam)
            lu = sol.local_solve(j, r)
            assert np.linalg.norm(fd - lu) < 1e-12 * np.linalg.norm(lu) * 10


def test_colored_equals_uncolored():
    """Colored additive Schwarz is the same operator (Sec. 2.3); 2^d parquet
    colors give patches of one color no common cell."""
    mesh = _mesh(2, 2, (5, 4), 6)
    A = sipg.assemble(mesh)
    subs = schwarz.vertex_patch_subdomains(mesh)
    colors = schwarz.vertex_patch_colors(mesh)
    for c in set(colors):
        cells = [set(idx // mesh.dofs_per_cell) for idx, cc in zip(subs, colors) if cc == c]
        for i in range(len(cells)):
            for j in range(i):
                assert not (cells[i] & cells[j])
    sol = schwarz.ExactLocalSolvers(A, subs)
    rng = np.random.default_rng(3)
    b, x = rng.uniform(-1, 1, mesh.ndofs), rng.uniform(-1, 1, mesh.ndofs)
    x1 = schwarz.additive_smooth(A, sol, x, b, 0.5)
    x2 = schwarz.additive_smooth(A, sol, x, b, 0.5, order=schwarz.colored_order(colors))
    assert np.abs(x1 - x2).max() < 1e-13 * np.abs(x1).max()


def test_brute_force_dense_operator():
    """The smoother equals x + omega B (b - A x) with B = sum_j R_j^T (R_j A R_j^T)^-1 R_j
    built by explicit inversion of every local matrix."""
    mesh = _mesh(2, 2, (3, 4), 7)
    A = sipg.assemble(mesh).toarray()
    subs = schwarz.vertex_patch_subdomains(mesh)
    B = np.zeros_like(A)
    for idx in subs:
        B[np.ix_(idx, idx)] += np.linalg.inv(A[np.ix_(idx, idx)])
    rng = np.random.default_rng(4)
    b, x = rng.uniform(-1, 1, mesh.ndofs), rng.uniform(-1, 1, mesh.ndofs)
    ref = x + 0.3 * B @ (b - A @ x)
    sol = schwarz.ExactLocalSolvers(sipg.assemble(mesh), subs, cache=False)
    out = schwarz.additive_smooth(sipg.assemble(mesh), sol, x, b, 0.3)
    assert np.abs(out - ref).max() < 1e-11 * np.abs(ref).max()


def test_additive_overlap_bound():
    """Coloring bound: if the subspaces split into C colors that are mutually
    A-orthogonal within each color, lambda_max(sum_j P_j) <= C.  Red-black cells
    give C = 2 and the multi red-black vertex-patch coloring C = 2^(d+1) (Sec. 2.3)."""
    mesh = uniform_mesh(2, 2, 4)
    A = sipg.assemble(mesh).toarray()
    for subs, bound in ((schwarz.vertex_patch_subdomains(mesh), 8.0), (schwarz.cell_subdomains(mesh), 2.0)):
        B = np.zeros_like(A)
        for idx in subs:
            B[np.ix_(idx, idx)] += np.linalg.inv(A[np.ix_(idx, idx)])
        lam = np.max(np.real(np.linalg.eigvals(B @ A)))
        assert 1.0 < lam <= bound + 1e-10


def test_multiplicative_one_color_per_cell_is_sequential_gauss_seidel():
    """With one color per subdomain Alg. (multsmoother) is the product form
    eq. (multschwarz1); checked against the explicit product of (I - P_j)."""
    mesh = _mesh(1, 2, (4,), 8)
    A = sipg.assemble(mesh)
    Ad = A.toarray()
    subs = schwarz.cell_subdomains(mesh)
    sol = schwarz.ExactLocalSolvers(A, subs)
    rng = np.random.default_rng(5)
    b, x = rng.uniform(-1, 1, mesh.ndofs), rng.uniform(-1, 1, mesh.ndofs)
    out = schwarz.multiplicative_smooth(A, sol, x, b, 1.0, colors=list(range(len(subs))))
    xs = np.linalg.solve(Ad, b)
    E = np.eye(mesh.ndofs)
    for idx in subs:
        R = np.zeros((len(idx), mesh.ndofs))
        R[np.arange(len(idx)), idx] = 1
        E = (np.eye(mesh.ndofs) - R.T @ np.linalg.solve(R @ Ad @ R.T, R @ Ad)) @ E
    assert np.abs((out - xs) - E @ (x - xs)).max() < 1e-11


@pytest.mark.parametrize("d,k,ms", [(2, 2, (5, 4)), (3, 1, (4, 5, 3))])
def test_mult_vertex_colors_decouple(d, k, ms):
    """2^(d+1) colors: two patches of one color share no DoF and A couples none
    of their DoFs (brute force on the assembled matrix)."""
    rng = np.random.default_rng(5)
    m = Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0))
    A = sipg.assemble(m).tocsr()
    subs = schwarz.vertex_patch_subdomains(m)
    cols = schwarz.vertex_patch_mult_colors(m)
    assert set(cols) == set(range(2 ** (d + 1)))
    for c in range(2 ** (d + 1)):
        js = [j for j, cc in enumerate(cols) if cc == c]
        for a in js:
            for b in js:
                if a < b:
                    assert not set(subs[a]) & set(subs[b])
                    assert abs(A[subs[a]][:, subs[b]]).max() == 0.0


@pytest.mark.parametrize("kind,d,k,ms", [("cell", 2, 3, (4, 3)), ("vertex", 2, 2, (4, 5)), ("vertex", 3, 1, (3, 4, 3))])
def test_colored_multiplicative_equals_sequential(kind, d, k, ms):
    """Within a color the local problems do not couple (eq. coloredschwarz), so
    Alg. multsmoother with one residual per color equals the fully sequential
    product over single subdomains in the same order."""
    rng = np.random.default_rng(6)
    m = Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0))
    A = sipg.assemble(m).tocsr()
    if kind == "cell":
        subs, cols = schwarz.cell_subdomains(m), schwarz.cell_red_black(m)
    else:
        subs, cols = schwarz.vertex_patch_subdomains(m), schwarz.vertex_patch_mult_colors(m)
    sol = schwarz.ExactLocalSolvers(A, subs)
    b = random_vector(m.ndofs, 0)
    x0 = random_vector(m.ndofs, 1)
    omega = 0.8
    xm = schwarz.multiplicative_smooth(A, sol, x0, b, omega, cols)
    xs = x0.copy()
    for j in schwarz.colored_order(cols):
        r = b - A @ xs
        xs[subs[j]] += omega * sol.local_solve(j, r[subs[j]])
    assert np.linalg.norm(xm - xs) <= 1e-12 * np.linalg.norm(xs)
