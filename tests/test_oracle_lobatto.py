"""Pins of the oracle's Gauss-Lobatto nodes and integration matrix.

Paper section 3.3.2 (equation sdc) integrates with the trapezoidal rule on
t^n, t^{n+1}: the M = 2 case.  Higher M are pinned to closed forms and to
exactness on polynomials of degree <= M-1.
"""
import numpy as np
import pytest

from oracle.lobatto import integration_matrix, nodes


def test_nodes_closed_forms():
    s5, s21 = np.sqrt(5.0), np.sqrt(21.0)
    np.testing.assert_allclose(nodes(2), [0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(nodes(3), [0.0, 0.5, 1.0], atol=1e-15)
    np.testing.assert_allclose(nodes(4), [0.0, (5 - s5) / 10, (5 + s5) / 10, 1.0], atol=1e-15)
    np.testing.assert_allclose(nodes(5), [0.0, (7 - s21) / 14, 0.5, (7 + s21) / 14, 1.0], atol=1e-15)


def test_trapezoid_is_the_two_node_case():
    np.testing.assert_allclose(integration_matrix(2), [[0.5, 0.5]], atol=1e-15)


def test_three_node_closed_form():
    # integral of the quadratic interpolant over [0, 1/2] and [1/2, 1]
    S = integration_matrix(3)
    np.testing.assert_allclose(S, [[5 / 24, 1 / 3, -1 / 24], [-1 / 24, 1 / 3, 5 / 24]], atol=1e-15)


@pytest.mark.parametrize("M", [2, 3, 4, 5])
def test_row_sums_and_polynomial_exactness(M):
    c = nodes(M)
    S = integration_matrix(M)
    np.testing.assert_allclose(S.sum(axis=1), np.diff(c), atol=1e-15)
    for deg in range(M):
        f = c ** deg
        exact = (c[1:] ** (deg + 1) - c[:-1] ** (deg + 1)) / (deg + 1)
        np.testing.assert_allclose(S @ f, exact, atol=1e-15)
    # and not exact one degree higher (so the test above is not vacuous)
    f = c ** (2 * M - 1)
    exact = (c[1:] ** (2 * M) - c[:-1] ** (2 * M)) / (2 * M)
    assert np.max(np.abs(S @ f - exact)) > 1e-6
