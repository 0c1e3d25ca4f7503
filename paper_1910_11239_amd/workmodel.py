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


def coarse_solve_bytes(dim, k, ncells, word=8):
    """Factor bytes read by one slab-blocked coarse solve on a mesh of
    ``ncells`` cells (slabs along the last axis): every diagonal block in
    full (B^2 for its lower and upper halves), and for each pair of
    neighbouring slabs the nonzero parts of W_i (row of cell c from column
    c nc on) and V_i (row of cell c up to column (c + 1) rc) plus the per-cell
    factors P_i and R_i, with nc = (k+1)^d unknowns and rc = 2 (k+1)^(d-1)
    face numbers per cell."""
    n1 = k + 1
    nc, rc = n1 ** dim, 2 * n1 ** (dim - 1)
    nb = ncells[-1]
    ncs = 1
    for m in ncells[:-1]:
        ncs *= int(m)
    B = ncs * nc
    w = rc * (ncs * B - nc * ncs * (ncs - 1) // 2)
    v = nc * rc * ncs * (ncs + 1) // 2
    return word * (nb * B * B + (nb - 1) * (w + v + 2 * ncs * rc * nc))
