"""Algorithmic work and traffic of the hot path (host logic, no device code).

Counts follow the structure of the method, not the kernels' implementation:

* a local solve by fast diagonalisation on an n^d subdomain is d forward and
  d backward 1-D contractions of n^(d+1) multiply-adds each plus the
  eigenvalue scaling and the accumulation: 4 d n^(d+1) + 2 n^d flops
  (Sec. 3.2, eq. eigenvectormatvec; reproduces Table tab:flop-additive);
* one sweep of the additive smoother must read x and b, and read/write x once
  more for the update; the residual r is written and read once:
  5 words per DoF (Sec. 2.3, Alg. addsmoother);
* the residual apply r = b - A x reads x and b and writes r: 3 words per DoF.
"""


def local_solver_flops(dim, n):
    return 4 * dim * n ** (dim + 1) + 2 * n ** dim


def n_subdomains(ncells, kind):
    out = 1
    for m in ncells:
        out *= m if kind == "cell" else (m - 1)
    return out


def smoother_flops(dim, k, ncells, kind):
    n = (k + 1) if kind == "cell" else 2 * (k + 1)
    return n_subdomains(ncells, kind) * local_solver_flops(dim, n)


def ndofs(dim, k, ncells):
    out = (k + 1) ** dim
    for m in ncells:
        out *= m
    return out


def residual_bytes(dim, k, ncells, word=8):
    return 3 * word * ndofs(dim, k, ncells)


def patch_apply_bytes(dim, k, ncells, word=8):
    """Local-solve pass given r: read r, read and write x: 3 words per DoF."""
    return 3 * word * ndofs(dim, k, ncells)


def smoother_sweep_bytes(dim, k, ncells, word=8):
    return 5 * word * ndofs(dim, k, ncells)
