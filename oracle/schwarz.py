"""Schwarz subspaces and smoothers with exact local solvers (oracle, test infrastructure only).

Sec. 2.3: the subspaces V_j are either single cells or vertex patches (all
2^d cells sharing an interior vertex).  The local solver is the Ritz
projection eq. (ritzproj), i.e. the exact inverse of A_j = R_j A R_j^T, taken
here by extracting A_j from the assembled matrix and factoring it by dense LU
(the plain "sACS"-style algorithm; no tensor structure is used).  The additive
smoother is eq. (additiveschwarz) / Alg. (addsmoother) with the relaxation
parameter multiplying the sum of local corrections:

    x <- x + omega * sum_j R_j^T A_j^-1 R_j (b - A x).

Patch-local ordering: the local 1-D index along axis t is
a_t = (c_t - first cell_t) * (k+1) + i_t, lexicographic with x fastest.

Pins: exact solve on a one-cell mesh (cell smoother, omega = 1) and on a
2^d-cell mesh (one vertex patch, omega = 1); the local solve equals the
independent fast-diagonalisation of the 1-D factors; the Ritz projection is
an A-orthogonal projection; colored and uncolored sums agree (Sec. 2.3).
"""
import hashlib
import itertools
import numpy as np
import scipy.linalg as sla


def cell_subdomains(mesh):
    return [mesh.cell_dofs(c) for c in mesh.cells()]


def interior_vertices(mesh):
    """Interior vertices v (1 <= v_t <= m_t - 1), lexicographic, x fastest."""
    rng = [range(1, m) for m in mesh.ncells]
    for v in itertools.product(*reversed(rng)):
        yield tuple(reversed(v))


def patch_dofs(mesh, v):
    """Global DoFs of the vertex patch around interior vertex v, patch-local order."""
    d, n1 = mesh.dim, mesh.n1
    n = 2 * n1
    out = np.empty(n ** d, dtype=np.int64)
    for p in range(n ** d):
        a, q = [], p
        for _ in range(d):
            a.append(q % n)
            q //= n
        cell = tuple(v[t] - 1 + a[t] // n1 for t in range(d))
        loc = sum((a[t] % n1) * n1 ** t for t in range(d))
        out[p] = mesh.cell_lin(cell) * mesh.dofs_per_cell + loc
    return out


def vertex_patch_subdomains(mesh):
    return [patch_dofs(mesh, v) for v in interior_vertices(mesh)]


def vertex_patch_colors(mesh):
    """2^d parquet colors (Sec. 2.3): color bits (v_t - 1) mod 2; two patches of
    one color share no cell."""
    return [sum(((v[t] - 1) % 2) << t for t in range(mesh.dim)) for v in interior_vertices(mesh)]


def cell_red_black(mesh):
    """Red-black coloring of cells (Sec. 2.3, multiplicative cell smoother)."""
    return [sum(c) % 2 for c in mesh.cells()]


def vertex_patch_mult_colors(mesh):
    """2^(d+1) colors of the multiplicative vertex-patch smoother (Sec. 2.3:
    parqueting combined with red-black).  Reading: the parquet color of
    eq. (vertex_patch_colors) in the low d bits, and in bit d the red-black
    parity of the patch inside its parquet sub-lattice,
    sum_t floor((v_t - 1) / 2) mod 2.  Two patches of one color then share no
    cell and no face, so their local problems do not couple through A."""
    d = mesh.dim
    return [sum(((v[t] - 1) % 2) << t for t in range(d)) + ((sum((v[t] - 1) // 2 for t in range(d)) % 2) << d)
            for v in interior_vertices(mesh)]


class ExactLocalSolvers:
    """Dense LU of every A_j = R_j A R_j^T.  Factors are shared between
    subdomains whose local matrices are bit-identical (switch off with cache=False)."""

    def __init__(self, A, subdomains, cache=True):
        self.subs = [np.asarray(s) for s in subdomains]
        self.lus = []
        seen = {}
        A = A.tocsr()
        for idx in self.subs:
            Aj = A[idx][:, idx].toarray()
            key = hashlib.sha1(Aj.tobytes()).hexdigest() if cache else None
            if key is not None and key in seen:
                self.lus.append(seen[key])
                continue
            lu = sla.lu_factor(Aj)
            if key is not None:
                seen[key] = lu
            self.lus.append(lu)

    def local_solve(self, j, rj):
        return sla.lu_solve(self.lus[j], rj)

    def apply(self, r, order=None):
        """sum_j R_j^T A_j^-1 R_j r, summed in the given subdomain order."""
        out = np.zeros_like(r)
        for j in (range(len(self.subs)) if order is None else order):
            idx = self.subs[j]
            out[idx] += self.local_solve(j, r[idx])
        return out


def additive_smooth(A, solvers, x, b, omega, order=None):
    """One step of Alg. (addsmoother): r = b - A x once, then the local solves."""
    r = b - A @ x
    return x + omega * solvers.apply(r, order)


def colored_order(colors):
    """Subdomain order 'color by color' (eq. coloredschwarz)."""
    colors = np.asarray(colors)
    return [int(j) for c in sorted(set(colors.tolist())) for j in np.nonzero(colors == c)[0]]


def multiplicative_smooth(A, solvers, x, b, omega, colors):
    """Alg. (multsmoother): residual updated before each color."""
    colors = np.asarray(colors)
    x = x.copy()
    for c in sorted(set(colors.tolist())):
        r = b - A @ x
        dx = np.zeros_like(x)
        for j in np.nonzero(colors == c)[0]:
            idx = solvers.subs[j]
            dx[idx] += solvers.local_solve(j, r[idx])
        x = x + omega * dx
    return x
