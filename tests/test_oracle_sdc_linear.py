"""Pins of the oracle's SDC machinery on problems with known answers.

* K = 0 (predictor only): backward Euler on every Gauss-Lobatto sub-interval,
  amplification prod_m 1 / (1 - dtau_m lam).
* K -> infinity: the sweeps converge to the Lobatto IIIA collocation solution,
  whose amplification is the (M-1, M-1) Pade approximant of exp(z).
* M = 2, K = 1: the paper's equation sdc (section 3.3.2) written out directly,
  on a nonlinear problem, with the backward-Euler predictor.
"""
import math

import numpy as np
import pytest

from oracle.lobatto import nodes
from oracle.models import TEST_LINEAR, TEST_LOGISTIC
from oracle.sdc import advance

PADE = {
    2: ([1, 1 / 2], [1, -1 / 2]),
    3: ([1, 1 / 2, 1 / 12], [1, -1 / 2, 1 / 12]),
    4: ([1, 1 / 2, 1 / 10, 1 / 120], [1, -1 / 2, 1 / 10, -1 / 120]),
    5: ([1, 1 / 2, 3 / 28, 1 / 84, 1 / 1680], [1, -1 / 2, 3 / 28, -1 / 84, 1 / 1680]),
}


def pade(M, z):
    num, den = PADE[M]
    return sum(a * z ** k for k, a in enumerate(num)) / sum(b * z ** k for k, b in enumerate(den))


def one_step(lam, dt, M, K, y0=1.0):
    mdl = TEST_LINEAR.with_params(lam=lam, b=0.0)
    X, _ = advance(mdl, np.array([[y0]]), dt=dt, n_steps=1, n_nodes=M, n_sweeps=K, tol=1e-15)
    return X[0, 0] / y0


@pytest.mark.parametrize("M", [2, 3, 4, 5])
@pytest.mark.parametrize("z", [-0.1, -0.7, -2.0])
def test_predictor_only_is_backward_euler_product(M, z):
    dt = 0.5
    lam = z / dt
    dtau = np.diff(nodes(M)) * dt
    expect = np.prod(1.0 / (1.0 - dtau * lam))
    assert one_step(lam, dt, M, 0) == pytest.approx(expect, rel=1e-14)


@pytest.mark.parametrize("M", [2, 3, 4, 5])
@pytest.mark.parametrize("z", [-0.5, -1.5, -3.0, 0.5])
def test_many_sweeps_reach_lobatto_collocation(M, z):
    dt = 0.25
    got = one_step(z / dt, dt, M, 60)
    assert got == pytest.approx(pade(M, z), rel=1e-12)
    # and the Pade value is distinguishable from exp(z) at this z
    assert abs(pade(M, z) - math.exp(z)) > 10 * 1e-12 * abs(pade(M, z))


def test_two_nodes_one_sweep_is_the_papers_correction():
    """Equation sdc with M~ = I on y' = y (1 - y): predictor by backward Euler,
    then (1 - tau J(Xt)) eps = X^n - Xt + tau/2 (F(X^n) + F(Xt))."""
    tau, y0 = 0.3, 0.2
    F = lambda y: y * (1.0 - y)
    J = lambda y: 1.0 - 2.0 * y
    # backward Euler by a scalar quadratic: y - y0 - tau y (1 - y) = 0
    a, b, c = tau, 1.0 - tau, -y0
    yt = (-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)
    eps = (y0 - yt + 0.5 * tau * (F(y0) + F(yt))) / (1.0 - tau * J(yt))
    X, _ = advance(TEST_LOGISTIC, np.array([[y0]]), dt=tau, n_steps=1, n_nodes=2, n_sweeps=1, tol=1e-15)
    assert X[0, 0] == pytest.approx(yt + eps, rel=1e-14)


def test_forcing_enters_through_i_diff():
    # y' = lam y + i_diff has the steady state -i_diff/lam, a fixed point of every scheme
    mdl = TEST_LINEAR.with_params(lam=-2.0, b=0.0)
    y_ss = 0.75
    X, _ = advance(mdl, np.array([[y_ss]]), dt=0.1, n_steps=20, n_nodes=3, n_sweeps=2,
                   i_diff=np.array([1.5]))
    assert X[0, 0] == pytest.approx(y_ss, rel=1e-14)
