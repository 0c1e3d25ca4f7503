"""Textbook Krylov solvers (oracle, test infrastructure only).

Sec. 2.4 uses CG preconditioned by one V-cycle for the additive smoothers and
GMRES for the multiplicative ones, stopping at a relative residual reduction.
Plain algorithms, FP64, zero start.
"""
import numpy as np


def pcg(A, b, precond, rtol=1e-10, maxit=1000, flexible=False):
    """Returns (x, iterations, list of ||r_i|| / ||b||).  flexible=True uses the
    Polak-Ribiere beta r_new.(z_new - z_old) / (r_old.z_old), which equals the
    standard beta for a fixed symmetric preconditioner in exact arithmetic."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    z = precond(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while hist[-1] > rtol and it < maxit:
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        it += 1
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
        z_old = z
        z = precond(r)
        rz_new = r @ z
        beta = (rz_new - r @ z_old) / rz if flexible else rz_new / rz
        p = z + beta * p
        rz = rz_new
    return x, it, hist


def gmres(A, b, precond, restart=30, rtol=1e-10, maxit=1000):
    """Right-preconditioned restarted GMRES in its flexible form (the
    preconditioned directions z_j = M v_j are kept, so a preconditioner that
    is not a fixed linear map is allowed; for a fixed one this is plain right-
    preconditioned GMRES).  Each cycle: Arnoldi with modified Gram-Schmidt on
    v_1 = r / |r|, z_j = M v_j, w = A z_j; the iterate x0 + Z y minimises
    |b - A x| over the cycle's directions, with y from the (j+1) x j
    Hessenberg least-squares problem.  Returns (x, iterations, list of
    ||r_i|| / ||b||) with the residual norm of every inner step."""
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    r = b - A @ x
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while hist[-1] > rtol and it < maxit:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            Z.append(precond(V[j]))
            w = A @ Z[j]
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            it += 1
            hist.append(res / nb)
            if hist[-1] <= rtol or it >= maxit or H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        x = x + np.column_stack(Z[:len(y)]) @ y
        r = b - A @ x
        hist[-1] = np.linalg.norm(r) / nb
    return x, it, hist
