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
