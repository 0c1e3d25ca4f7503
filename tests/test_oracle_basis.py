"""Pins of the oracle's 1-D reference basis against textbook closed forms."""
import numpy as np
import pytest

from oracle.basis import (gll_nodes, gauss_rule, lagrange_values, lagrange_derivatives,
                          reference_mass_stiffness)

# Gauss-Lobatto points and weights on [0, 1] (textbook values on [-1, 1] mapped
# by x -> (x + 1)/2, weights halved).
GLL = {
    1: ([0.0, 1.0], [0.5, 0.5]),
    2: ([0.0, 0.5, 1.0], [1 / 6, 2 / 3, 1 / 6]),
    3: ([0.0, (1 - 1 / np.sqrt(5)) / 2, (1 + 1 / np.sqrt(5)) / 2, 1.0], [1 / 12, 5 / 12, 5 / 12, 1 / 12]),
    4: ([0.0, (1 - np.sqrt(3 / 7)) / 2, 0.5, (1 + np.sqrt(3 / 7)) / 2, 1.0],
        [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20]),
}


@pytest.mark.parametrize("k", sorted(GLL))
def test_gll_nodes_textbook(k):
    assert np.allclose(gll_nodes(k), GLL[k][0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", sorted(GLL))
def test_mass_row_sums_are_gll_weights(k):
    # sum_i Mhat[iota, i] = int phi_iota = GLL weight (GLL rule exact to degree 2k-1 >= k)
    Mhat, _ = reference_mass_stiffness(k)
    assert np.allclose(Mhat.sum(axis=1), GLL[k][1], rtol=0, atol=1e-15)


def test_k1_closed_forms():
    Mhat, Lhat = reference_mass_stiffness(1)
    assert np.allclose(Mhat, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    assert np.allclose(Lhat, [[1, -1], [-1, 1]], atol=1e-15)
    nodes = gll_nodes(1)
    assert np.allclose(lagrange_derivatives(nodes, [0.0])[0], [-1, 1])
    assert np.allclose(lagrange_derivatives(nodes, [1.0])[0], [-1, 1])


@pytest.mark.parametrize("k", range(1, 11))
def test_partition_of_unity_and_invariants(k):
    nodes = gll_nodes(k)
    x = np.linspace(0, 1, 13)
    assert np.allclose(lagrange_values(nodes, x).sum(axis=1), 1.0, atol=1e-12)
    assert np.allclose(lagrange_derivatives(nodes, x).sum(axis=1), 0.0, atol=1e-9)
    Mhat, Lhat = reference_mass_stiffness(k)
    assert abs(Mhat.sum() - 1.0) < 1e-13
    assert np.allclose(Lhat @ np.ones(k + 1), 0.0, atol=1e-10)
    assert np.allclose(Mhat, Mhat.T) and np.allclose(Lhat, Lhat.T)
    # Lagrange property
    assert np.allclose(lagrange_values(nodes, nodes), np.eye(k + 1), atol=1e-13)


@pytest.mark.parametrize("k", range(1, 10))
def test_derivative_reproduces_monomials(k):
    nodes = gll_nodes(k)
    x = np.linspace(0, 1, 7)
    D = lagrange_derivatives(nodes, x)
    for p in range(1, k + 1):
        assert np.allclose(D @ nodes ** p, p * x ** (p - 1), atol=1e-9)


@pytest.mark.parametrize("nq", range(1, 12))
def test_gauss_rule_exactness(nq):
    x, w = gauss_rule(nq)
    for p in range(2 * nq):
        assert abs(w @ x ** p - 1.0 / (p + 1)) < 1e-14


@pytest.mark.parametrize("k", [2, 3, 5])
def test_mass_stiffness_exact_integrals(k):
    # Mhat, Lhat integrate products of the interpolants of monomials exactly
    nodes = gll_nodes(k)
    Mhat, Lhat = reference_mass_stiffness(k)
    for p in range(k + 1):
        for q in range(k + 1):
            up, uq = nodes ** p, nodes ** q
            assert abs(up @ Mhat @ uq - 1.0 / (p + q + 1)) < 1e-13
            if p and q:
                assert abs(up @ Lhat @ uq - p * q / (p + q - 1)) < 1e-11
