"""Separate 1-D path (oracle, test infrastructure only; never used by the smoother).

Sec. 3.2 states that on Cartesian meshes the SIPG matrix restricted to a cell
or vertex patch is a Kronecker sum (eq. KDseparable) of 1-D matrices: mass
matrices M = h Mhat and interior stiffness L = Lhat / h (eq. 1Dstiffnessmass),
plus 1-D Nitsche terms for the two faces (eq. 1Dconsistencypenalty, 1Dnitsche,
1Dsipg) and, for a vertex patch, 2 x 2 block matrices whose off-diagonal
blocks couple the two cells through their common face (eq. 1DsipgVP).

Readings taken where the printed formulas are garbled (derived from
eq. bfsipg with the 1/sqrt(2) average, and checked by the separability
identity against the quadrature matrix of ``sipg``):

* the penalty of one cell's face term carries the same weight eta as the
  consistency term: N_p = eta gamma M_p - G_p - G_p^T, eta = 1/2 inside and 1
  on the boundary;
* the interface block between the left cell (width hl) and the right cell
  (width hr) of a patch, rows = test functions of the left cell, columns =
  trial functions of the right cell, is
      A_lr = -(gamma/2) v1 v0^T - 1/(2 hr) v1 d0^T + 1/(2 hl) d1 v0^T,
  with A_rl = A_lr^T and gamma = gamma_hat k (k+1) (1/hl + 1/hr).

Here v0 = (phi_i(0))_i, v1 = (phi_i(1))_i, d0 = (phi_i'(0))_i, d1 = (phi_i'(1))_i.
These formulas are pinned by tests/test_oracle_sipg.py (separability identity
for cells, vertex patches and the whole mesh, random rectilinear widths).
"""
import numpy as np
import scipy.linalg as sla

from .basis import gll_nodes, lagrange_values, lagrange_derivatives, reference_mass_stiffness


class Ref1D:
    def __init__(self, k):
        self.k = k
        self.Mhat, self.Lhat = reference_mass_stiffness(k)
        nodes = gll_nodes(k)
        self.v = [lagrange_values(nodes, [s])[0] for s in (0.0, 1.0)]
        self.dv = [lagrange_derivatives(nodes, [s])[0] for s in (0.0, 1.0)]

    def penalty(self, gamma_hat, ha, hb):
        return gamma_hat * self.k * (self.k + 1) * (1.0 / ha + 1.0 / hb)

    def nitsche(self, p, h, gamma, eta):
        """One face of a cell of width h; p = 0 left face, p = 1 right face."""
        s = -1.0 if p == 0 else 1.0
        v, dv = self.v[p], self.dv[p]
        G = s * (eta / h) * np.outer(v, dv)
        return eta * gamma * np.outer(v, v) - G - G.T

    def cell_operator(self, h, h_left, h_right, gamma_hat):
        """A = L + N_0 + N_1 of eq. (1Dsipg); h_left/h_right = None on the boundary."""
        A = self.Lhat / h
        for p, hn in ((0, h_left), (1, h_right)):
            if hn is None:
                A = A + self.nitsche(p, h, self.penalty(gamma_hat, h, h), 1.0)
            else:
                A = A + self.nitsche(p, h, self.penalty(gamma_hat, h, hn), 0.5)
        return A

    def interface(self, hl, hr, gamma_hat):
        """Block coupling test functions of the left cell to trial functions of the right cell."""
        g = self.penalty(gamma_hat, hl, hr)
        v0, v1, d0, d1 = self.v[0], self.v[1], self.dv[0], self.dv[1]
        return -(g / 2) * np.outer(v1, v0) - np.outer(v1, d0) / (2 * hr) + np.outer(d1, v0) / (2 * hl)

    def mass(self, h):
        return h * self.Mhat


def chain_operator(ref, widths, lo_nb, hi_nb, gamma_hat):
    """1-D SIPG matrix and mass of a chain of consecutive cells ``widths``.
    lo_nb / hi_nb: width of the outside neighbour beyond the chain ends, or
    None where the chain touches the boundary.  One cell gives eq. (1Dsipg),
    two cells a vertex-patch factor eq. (1DsipgVP), all cells of an axis the
    global 1-D matrix (block tridiagonal)."""
    m, n1 = len(widths), ref.k + 1
    A = np.zeros((m * n1, m * n1))
    M = np.zeros_like(A)
    for j in range(m):
        hl = widths[j - 1] if j > 0 else lo_nb
        hr = widths[j + 1] if j + 1 < m else hi_nb
        sl = slice(j * n1, (j + 1) * n1)
        A[sl, sl] = ref.cell_operator(widths[j], hl, hr, gamma_hat)
        M[sl, sl] = ref.mass(widths[j])
        if j + 1 < m:
            sr = slice((j + 1) * n1, (j + 2) * n1)
            B = ref.interface(widths[j], widths[j + 1], gamma_hat)
            A[sl, sr] = B
            A[sr, sl] = B.T
    return A, M


def kron_sum(As, Ms):
    """sum_t M_{d-1} x ... x A_t x ... x M_0 (x fastest), eq. (KDseparable)."""
    d = len(As)
    out = 0.0
    for t in range(d):
        F = np.ones((1, 1))
        for a in reversed(range(d)):
            F = np.kron(F, As[a] if a == t else Ms[a])
        out = out + F
    return out


def axis_chain(mesh, axis, first, count):
    """Widths of cells first..first+count-1 along axis and their outside neighbours."""
    w = mesh.widths[axis]
    lo = w[first - 1] if first > 0 else None
    hi = w[first + count] if first + count < len(w) else None
    return w[first:first + count], lo, hi


def global_fastdiag_solve(mesh, b):
    """Exact solution of A u = b on a rectilinear mesh by global fast
    diagonalisation (Lynch et al.): per axis the generalized eigenproblem of the
    global 1-D pair (A_t, M_t) (eq. generalizedEVP), then
    u = Z Lambda^-1 Z^T b with Z the Kronecker product (eq. fastinverse).
    Cost O(N * sum_t m_t n1), usable at full problem size."""
    d, n1 = mesh.dim, mesh.n1
    ref = Ref1D(mesh.k)
    Zs, lams = [], []
    for a in range(d):
        A1, M1 = chain_operator(ref, mesh.widths[a], None, None, mesh.gamma_hat)
        lam, Z = sla.eigh(A1, M1)
        Zs.append(Z)
        lams.append(lam)
    T = to_axis_tensor(mesh, b)
    for a in range(d):
        T = _apply_axis(T, Zs[a].T, a, d)
    L = np.zeros(T.shape)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = len(lams[a])
        L = L + lams[a].reshape(shape)
    T = T / L
    for a in range(d):
        T = _apply_axis(T, Zs[a], a, d)
    return from_axis_tensor(mesh, T)


def _apply_axis(T, Mat, a, d):
    """Contract Mat (out x in) with tensor axis ``a`` (numpy axis d-1-a)."""
    ax = d - 1 - a
    T = np.tensordot(T, Mat, axes=([ax], [1]))  # contracted axis moved last
    return np.moveaxis(T, -1, ax)


def to_axis_tensor(mesh, vec):
    """Cell-major vector -> d-way tensor indexed [I_{d-1}, ..., I_0] with the
    global 1-D index I_a = c_a * n1 + i_a."""
    d, n1, m = mesh.dim, mesh.n1, mesh.ncells
    shape = []
    for a in reversed(range(d)):
        shape += [m[a]]
    shape += [n1] * d
    T = vec.reshape(shape)          # [c_{d-1}..c_0, i_{d-1}..i_0]
    perm = []
    for j in range(d):
        perm += [j, d + j]
    T = T.transpose(perm)           # [c_{d-1}, i_{d-1}, ..., c_0, i_0]
    return T.reshape([m[a] * n1 for a in reversed(range(d))])


def from_axis_tensor(mesh, T):
    d, n1, m = mesh.dim, mesh.n1, mesh.ncells
    shape = []
    for a in reversed(range(d)):
        shape += [m[a], n1]
    T = T.reshape(shape)
    perm = [2 * j for j in range(d)] + [2 * j + 1 for j in range(d)]
    return T.transpose(perm).reshape(-1).copy()
