"""1-D reference basis and quadrature on [0, 1] (oracle, test infrastructure only).

Sec. 2.1 and Sec. 3 intro: the shape functions are tensor products of degree-k
Lagrange polynomials in the Gauss-Lobatto points of the reference interval;
integrals use a tensor product of a 1-D quadrature rule.  The oracle integrates
exactly with the (k+1)-point Gauss-Legendre rule (degree 2k+1 exact), which is
the reading of "quadrature almost identical with k" (Sec. 3.1) that makes the
1-D mass and stiffness matrices of eq. (1Dstiffnessmass) exact.

Pins (tests/test_oracle_basis.py): textbook GLL nodes for k = 1..4, the GLL
weights recovered as row sums of the exact mass matrix, closed forms for k = 1,
partition of unity, and exactness of the Gauss rule on monomials.
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gll_nodes(k):
    """Gauss-Lobatto nodes of degree k on [0, 1]: the endpoints and the roots
    of the derivative of the Legendre polynomial P_k, mapped from [-1, 1]."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if k == 1:
        inner = np.array([])
    else:
        coef = np.zeros(k + 1)
        coef[k] = 1.0
        inner = np.sort(np.real(_leg.legroots(_leg.legder(coef))))
    x = np.concatenate(([-1.0], inner, [1.0]))
    return 0.5 * (x + 1.0)


def gauss_rule(nq):
    """nq-point Gauss-Legendre rule on [0, 1]: (points, weights)."""
    x, w = _leg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """V[q, i] = phi_i(x_q) for the Lagrange polynomials of ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[q, i] = phi_i'(x_q) by the product rule applied to the Lagrange form."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D


def reference_mass_stiffness(k):
    """Exact reference matrices on [0, 1]: Mhat[iota, i] = int phi_i phi_iota,
    Lhat[iota, i] = int phi_i' phi_iota' (eq. 1Dstiffnessmass with h = 1)."""
    nodes = gll_nodes(k)
    xq, wq = gauss_rule(k + 1)
    V = lagrange_values(nodes, xq)
    D = lagrange_derivatives(nodes, xq)
    Mhat = V.T @ (wq[:, None] * V)
    Lhat = D.T @ (wq[:, None] * D)
    return Mhat, Lhat
