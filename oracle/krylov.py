"""Textbook preconditioned conjugate gradients (oracle, test infrastructure only).

Sec. 2.4 uses CG preconditioned by one V-cycle for the additive smoothers,
stopping at a relative residual reduction.  Plain algorithm, FP64, zero start.
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
