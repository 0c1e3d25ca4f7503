"""Pins of the oracle's transfers, V-cycle and PCG (Sec. 2.2, Alg. gmg, Sec. 2.4)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.mesh import Mesh, uniform_mesh, coarsen, refine
from oracle import sipg, onedim, multigrid, krylov
from synthetic import loguniform_widths, random_vector


@pytest.mark.parametrize("d,k", [(1, 3), (2, 2), (3, 2), (2, 4)])
def test_prolongation_reproduces_polynomials(d, k):
    """Nested spaces (Sec. 2.2): the embedding maps the coarse interpolant of
    a Q_k polynomial onto its fine interpolant exactly."""
    rng = np.random.default_rng(1)
    fine = Mesh(d, k, loguniform_widths(rng, d, (4,) * d, 0.25, 4.0, paired=True))
    coarse = coarsen(fine)
    P = multigrid.prolongation(coarse, fine)
    cs = rng.uniform(-1, 1, (d, k + 1))

    def u(X):
        out = np.ones(len(X))
        for a in range(d):
            out *= np.polynomial.polynomial.polyval(X[:, a] / 4.0, cs[a])
        return out

    uc, uf = sipg.interpolate(coarse, u), sipg.interpolate(fine, u)
    assert np.abs(P @ uc - uf).max() < 1e-12 * np.abs(uf).max()


def test_refine_coarsen_roundtrip():
    m = Mesh(2, 2, (np.array([0.3, 0.5]), np.array([1.0, 0.25, 0.75])))
    assert all(np.allclose(a, b) for a, b in zip(coarsen(refine(m)).widths, m.widths))


def test_single_level_vcycle_is_lu():
    mesh = uniform_mesh(2, 2, 2)
    h = multigrid.Hierarchy(mesh, 1, "vertex", 0.5)
    b = np.random.default_rng(0).uniform(-1, 1, mesh.ndofs)
    x = h.vcycle(np.zeros_like(b), b)
    assert np.linalg.norm(h.A[0] @ x - b) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("kind,omega,msm", [("cell", 0.7, 1), ("vertex", 0.25, 2)])
def test_vcycle_symmetric_positive(kind, omega, msm):
    """For m_pre = m_post and symmetric additive smoothers the V-cycle
    preconditioner x = MG(0, b) is a symmetric linear map B.  With the
    damping of Sec. 2.4 (0.7 for cells, 2^-d for overlapping vertex patches)
    B A has a positive spectrum with a small condition number, as CG needs."""
    fine = uniform_mesh(2, 2, 8)
    h = multigrid.Hierarchy(fine, 3, kind, omega, m_pre=msm, m_post=msm)
    N = fine.ndofs
    B = np.column_stack([h.vcycle(np.zeros(N), e) for e in np.eye(N)])
    assert np.abs(B - B.T).max() < 1e-10 * np.abs(B).max()
    A = h.A[-1].toarray()
    ev = np.linalg.eigvals(B @ A)
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() > 0.1 and ev.real.max() / ev.real.min() < 10


def test_vcycle_linear_in_x_and_b():
    fine = uniform_mesh(2, 2, 4)
    h = multigrid.Hierarchy(fine, 2, "vertex", 0.3, m_pre=2, m_post=2)
    rng = np.random.default_rng(2)
    x, b = rng.uniform(-1, 1, fine.ndofs), rng.uniform(-1, 1, fine.ndofs)
    A = h.A[-1]
    # MG(x, b) = x + B (b - A x) with B = MG(0, .)
    lhs = h.vcycle(x, b)
    rhs = x + h.vcycle(np.zeros_like(b), b - A @ x)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()


def test_pcg_with_vcycle_converges():
    """CG preconditioned by one V-cycle with the additive cell smoother,
    omega = 0.7 (Sec. 2.4) reaches 1e-10 in a bounded number of steps and
    matches the exact discrete solution (global fast diagonalisation)."""
    fine = uniform_mesh(2, 3, 8)
    h = multigrid.Hierarchy(fine, 3, "cell", 0.7, m_pre=1, m_post=1)
    b = np.random.default_rng(3).uniform(-1, 1, fine.ndofs)
    x, it, hist = krylov.pcg(h.A[-1], b, lambda r: h.vcycle(np.zeros_like(r), r), rtol=1e-10)
    assert it < 40 and hist[-1] <= 1e-10
    xs = onedim.global_fastdiag_solve(fine, b)
    assert np.linalg.norm(x - xs) < 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("kind,d,k,ms", [("vertex", 2, 2, (4, 4)), ("cell", 2, 3, (4, 4))])
def test_gmres_with_multiplicative_vcycle_converges(kind, d, k, ms):
    """GMRES with the multiplicative V-cycle (Alg. multsmoother on every level)
    reaches the exact discrete solution (global fast diagonalisation)."""
    from oracle import krylov, onedim
    fine = refine(uniform_mesh(d, k, ms))
    oh = multigrid.Hierarchy(fine, 2, kind, [0.0, 1.0], m_pre=1, m_post=1, smoother="multiplicative")
    b = random_vector(fine.ndofs, 0)
    x, it, hist = krylov.gmres(oh.A[-1], b, lambda v: oh.vcycle(np.zeros_like(v), v), restart=20, rtol=1e-10)
    assert hist[-1] <= 1e-10 and it < 40
    xs = onedim.global_fastdiag_solve(fine, b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("kind,d,k,ms", [("cell", 2, 2, (4, 4)), ("vertex", 2, 1, (4, 4)), ("cell", 3, 1, (2, 2, 4))])
def test_reversed_post_smoothing_symmetrises_the_multiplicative_vcycle(kind, d, k, ms):
    """With the colors of post-smoothing in the reverse order of
    pre-smoothing, the multiplicative V-cycle as a linear map b -> MG(0, b) is
    symmetric (and positive: CG can use it); with the same order it is not."""
    mesh = Mesh(d, k, [np.full(m, 1.0 / m) for m in ms], 1.0)
    N = mesh.ndofs
    for smoother, sym in (("multiplicative_symmetric", True), ("multiplicative", False)):
        h = multigrid.Hierarchy(mesh, 2, kind, [0.0, 0.8], m_pre=1, m_post=1, smoother=smoother)
        B = np.column_stack([h.vcycle(np.zeros(N), e) for e in np.eye(N)])
        asym = np.abs(B - B.T).max() / np.abs(B).max()
        if sym:
            assert asym <= 1e-10, (smoother, asym)
            assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
        else:
            assert asym > 1e-4, (smoother, asym)
