"""Pins of the oracle's Krylov solvers against what the mathematics fixes.

GMRES: the k-th iterate minimises ||b - A x|| over x0 + M K_k(A M, r0) (checked
against a brute-force least-squares solve over an explicitly built Krylov
basis), terminates with the exact solution after at most n steps, and its
restarted form decreases the residual monotonically.  CG is pinned through
the multigrid tests (convergence to the exact solution)."""
import numpy as np

from oracle import krylov


def _system(n, seed, sym=False):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (n, n)) + n * np.eye(n)
    if sym:
        A = A @ A.T
    M = np.eye(n) + 0.1 * rng.uniform(-1, 1, (n, n))
    b = rng.uniform(-1, 1, n)
    return A, M, b


def test_gmres_minimal_residual_over_krylov_space():
    n = 14
    A, M, b = _system(n, 0)
    for k in range(1, 9):
        x, it, hist = krylov.gmres(A, b, lambda v: M @ v, restart=n, rtol=0.0, maxit=k)
        assert it == k
        # brute force: orthonormal basis of K_k(A M, b), directions M K
        K = [b]
        for _ in range(k - 1):
            K.append(A @ (M @ K[-1]))
        Q, _ = np.linalg.qr(np.column_stack(K))
        X = M @ Q
        c = np.linalg.lstsq(A @ X, b, rcond=None)[0]
        best = np.linalg.norm(b - A @ X @ c)
        got = np.linalg.norm(b - A @ x)
        assert abs(got - best) <= 1e-10 * np.linalg.norm(b), (k, got, best)
        assert abs(hist[-1] * np.linalg.norm(b) - got) <= 1e-10 * np.linalg.norm(b)


def test_gmres_exact_after_n_steps():
    n = 12
    A, M, b = _system(n, 1)
    x, it, hist = krylov.gmres(A, b, lambda v: M @ v, restart=n, rtol=1e-13, maxit=n)
    assert it <= n
    assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)


def test_restarted_gmres_monotone_and_converges():
    n = 40
    A, M, b = _system(n, 2, sym=True)
    x, it, hist = krylov.gmres(A, b, lambda v: M @ v, restart=5, rtol=1e-10, maxit=500)
    assert hist[-1] <= 1e-10
    assert all(h1 <= h0 * (1 + 1e-12) for h0, h1 in zip(hist, hist[1:]))
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_gmres_with_identity_preconditioner_on_spd_matches_cg_solution():
    A, _, b = _system(20, 3, sym=True)
    xg, _, _ = krylov.gmres(A, b, lambda v: v, restart=20, rtol=1e-12, maxit=40)
    xc, _, _ = krylov.pcg(A, b, lambda v: v, rtol=1e-12, maxit=200)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(xg - xs) <= 1e-9 * np.linalg.norm(xs)
    assert np.linalg.norm(xc - xs) <= 1e-9 * np.linalg.norm(xs)


def test_flexible_pcg_equals_standard_pcg_for_fixed_spd_preconditioner():
    """For a fixed symmetric positive definite preconditioner the Polak-Ribiere
    beta r_new.(z_new - z_old) / (r_old.z_old) equals the Fletcher-Reeves beta,
    since r_new.z_old = r_new.M r_old = 0 (residuals are M-orthogonal in PCG):
    the flexible branch must give the standard residual history."""
    n = 60
    rng = np.random.default_rng(7)
    Q = rng.uniform(-1, 1, (n, n))
    A = Q @ Q.T / n + 0.2 * np.eye(n)
    R = rng.uniform(-1, 1, (n, n))
    M = R @ R.T / n + np.eye(n)
    b = rng.uniform(-1, 1, n)
    xs, its, hs = krylov.pcg(A, b, lambda v: M @ v, rtol=1e-11, maxit=200)
    xf, itf, hf = krylov.pcg(A, b, lambda v: M @ v, rtol=1e-11, maxit=200, flexible=True)
    assert abs(its - itf) <= 1 and its > 10
    # the two betas differ by r_new.z_old, zero in exact arithmetic and a
    # rounding residue that grows once the residual is small: compare the
    # history down to 1e-6
    nh = sum(1 for h in hs if h > 1e-6)
    assert nh > 10
    assert np.allclose(hf[:nh], hs[:nh], rtol=1e-11, atol=0)
    assert np.linalg.norm(xf - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(np.linalg.solve(A, b))


def test_flexible_pcg_first_step_and_a_conjugacy():
    """Plain consequences of CG that a wrong sign or index would break: the
    first step is the exact line search along p_0 = M r_0, and with a fixed SPD
    preconditioner successive search directions are A-conjugate, so the
    iterate after n steps is the exact solution."""
    n = 12
    rng = np.random.default_rng(8)
    Q = rng.uniform(-1, 1, (n, n))
    A = Q @ Q.T + np.eye(n)
    M = np.diag(rng.uniform(0.5, 2.0, n))
    b = rng.uniform(-1, 1, n)
    x1, it1, h1 = krylov.pcg(A, b, lambda v: M @ v, rtol=0.0, maxit=1, flexible=True)
    p = M @ b
    alpha = (b @ p) / (p @ A @ p)
    assert np.allclose(x1, alpha * p, rtol=1e-13, atol=0)
    assert abs(h1[1] - np.linalg.norm(b - alpha * A @ p) / np.linalg.norm(b)) < 1e-13
    xn, itn, hn = krylov.pcg(A, b, lambda v: M @ v, rtol=0.0, maxit=n, flexible=True)
    assert np.linalg.norm(A @ xn - b) <= 1e-8 * np.linalg.norm(b)


def test_flexible_pcg_with_symmetric_vcycle_matches_standard():
    """The case the library's CG is compared in: one symmetric V-cycle
    (additive vertex patches, 2 + 2 sweeps) as a fixed SPD preconditioner of the
    3-D SIPG matrix.  Flexible and standard beta give the same residual history
    (to 1e-12 while the residual is above 1e-6) and the same solution."""
    from oracle.mesh import refine, uniform_mesh
    from oracle import multigrid
    from synthetic import random_vector
    fine = refine(refine(uniform_mesh(3, 2, 1)))
    oh = multigrid.Hierarchy(fine, 3, "vertex", [0.0, 0.125, 0.125], m_pre=2, m_post=2)
    b = random_vector(fine.ndofs, 0)
    pre = lambda r: oh.vcycle(np.zeros_like(r), r)
    xs, its, hs = krylov.pcg(oh.A[-1], b, pre, rtol=1e-10)
    xf, itf, hf = krylov.pcg(oh.A[-1], b, pre, rtol=1e-10, flexible=True)
    nh = sum(1 for h in hs if h > 1e-6)
    assert nh >= 5 and abs(its - itf) <= 1
    assert np.allclose(hf[:nh], hs[:nh], rtol=1e-12, atol=0)
    assert np.linalg.norm(xf - xs) <= 1e-9 * np.linalg.norm(xs)
