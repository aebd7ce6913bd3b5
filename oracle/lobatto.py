"""Gauss-Lobatto collocation nodes and the spectral integration matrix
(oracle; test infrastructure).

The paper's correction (section 3.3.2, equation sdc) integrates F with the
trapezoidal rule on the two nodes t^n, t^{n+1}; that is the M = 2 member of the
Gauss-Lobatto family used by multi-node SDC (the paper's SDC references,
cited in the introduction).  For M nodes on [0, 1] the interior abscissae are
the roots of P'_{M-1}, the derivative of the Legendre polynomial of degree
M-1, mapped from [-1, 1]; the integration matrix entry

    S[m, j] = integral from c_m to c_{m+1} of l_j(s) ds,   m = 0..M-2,

with l_j the Lagrange basis polynomial of node j, integrates the degree-(M-1)
interpolant of F node to node.  Multiplying S by dt gives the quadrature
weights of one time step.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L
from numpy.polynomial import polynomial as P


def nodes(M: int) -> np.ndarray:
    if M < 2:
        raise ValueError("Gauss-Lobatto needs at least 2 nodes")
    if M == 2:
        x = np.array([-1.0, 1.0])
    else:
        inner = np.sort(L.Legendre.basis(M - 1).deriv().roots().real)
        x = np.concatenate(([-1.0], inner, [1.0]))
    return 0.5 * (x + 1.0)


def lagrange_basis(c: np.ndarray, j: int) -> P.Polynomial:
    others = np.delete(c, j)
    num = P.Polynomial.fromroots(others)
    return num / np.prod(c[j] - others)


def integration_matrix(M: int) -> np.ndarray:
    """S of shape (M-1, M), for the unit interval."""
    c = nodes(M)
    S = np.empty((M - 1, M))
    for j in range(M):
        Lj = lagrange_basis(c, j).integ()
        for m in range(M - 1):
            S[m, j] = Lj(c[m + 1]) - Lj(c[m])
    return S
