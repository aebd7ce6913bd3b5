"""Pins of the oracle's ROS2 predictor (paper section 3.3.1, equations
rb_system and second_sol) and of the SDC scheme built on it (section 3.3.2,
equation sdc).

The paper states the properties of ROS2 (two stages, second order, L-stable,
embedded second solution for step control) but prints no coefficients, so the
pins are those properties, measured on problems with closed forms:
* local error O(tau^3) of the main and O(tau^2) of the embedded solution, on
  y' = lam y (stability function against exp) and on the logistic equation
  (nonlinear order conditions, exact Jacobian);
* L-stability: the amplification tends to 0 as lam tau -> -infinity and
  stays below 1 in magnitude on the whole negative axis;
* M = 2, K = 1 with the ROS2 predictor is the paper's equation sdc applied to
  the ROS2 value, written out directly;
* the sweeps still converge to Lobatto collocation and gain one order each,
  from the predictor's order 2.
"""
import math

import numpy as np
import pytest

from oracle.models import TEST_LINEAR, TEST_LOGISTIC, TT06
from oracle import tt06
from oracle.ros2 import ros2_step
from oracle.sdc import advance
from oracle.testmodels import Logistic

from test_oracle_sdc_linear import pade


def amplification(z, embedded=False):
    mdl = TEST_LINEAR.with_params(lam=z, b=0.0)
    X, Xh, _ = ros2_step(mdl, np.array([[1.0]]), 1.0, 0.0, 0.0)
    return (Xh if embedded else X)[0, 0]


def local_orders(errs):
    errs = np.abs(np.asarray(errs))
    return np.log2(errs[:-1] / errs[1:])


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_linear_local_error_orders(sign):
    zs = sign * np.array([0.04, 0.02, 0.01, 0.005])
    main = [amplification(z) - math.exp(z) for z in zs]
    emb = [amplification(z, True) - math.exp(z) for z in zs]
    assert np.all(np.abs(local_orders(main)[-2:] - 3.0) < 0.1)   # second-order method
    assert np.all(np.abs(local_orders(emb)[-2:] - 2.0) < 0.1)    # first-order embedding


def test_l_stable():
    for z in (-1e3, -1e6, -1e9):
        assert abs(amplification(z)) < 10.0 / abs(z)
    for z in (-0.1, -1.0, -10.0, -1e3):
        assert abs(amplification(z)) < 1.0


def test_nonlinear_local_error_orders():
    rate, y0 = 3.0, 0.2
    mdl = TEST_LOGISTIC.with_params(rate=rate)
    main, emb = [], []
    for tau in (0.02, 0.01, 0.005, 0.0025):
        X, Xh, F0 = ros2_step(mdl, np.array([[y0]]), tau, 0.0, 0.0)
        ex = Logistic.exact(y0, tau, dict(rate=rate))
        main.append(X[0, 0] - ex)
        emb.append(Xh[0, 0] - ex)
        assert F0[0, 0] == pytest.approx(rate * y0 * (1 - y0), rel=1e-15)
    assert np.all(np.abs(local_orders(main)[-2:] - 3.0) < 0.15)
    assert np.all(np.abs(local_orders(emb)[-2:] - 2.0) < 0.15)


def test_two_nodes_one_sweep_on_ros2_is_the_papers_correction():
    """Equation sdc with M~ = I, predictor = one ROS2 step:
    (1 - tau J(Xt)) eps = X^n - Xt + tau/2 (F(X^n) + F(Xt))."""
    tau, y0, rate = 0.3, 0.2, 1.0
    mdl = TEST_LOGISTIC.with_params(rate=rate)
    F = lambda y: rate * y * (1.0 - y)
    J = lambda y: rate * (1.0 - 2.0 * y)
    Xt, _, _ = ros2_step(mdl, np.array([[y0]]), tau, 0.0, 0.0)
    yt = Xt[0, 0]
    eps = (y0 - yt + 0.5 * tau * (F(y0) + F(yt))) / (1.0 - tau * J(yt))
    X, st = advance(mdl, np.array([[y0]]), dt=tau, n_steps=1, n_nodes=2, n_sweeps=1,
                    predictor="ros2")
    assert X[0, 0] == pytest.approx(yt + eps, rel=1e-14)
    assert st.newton_iters_total == 0 and len(st.embedded_error) == 1


@pytest.mark.parametrize("M", [2, 3, 4])
def test_many_sweeps_reach_lobatto_collocation(M):
    z, dt = -1.5, 0.25
    mdl = TEST_LINEAR.with_params(lam=z / dt, b=0.0)
    X, _ = advance(mdl, np.array([[1.0]]), dt=dt, n_steps=1, n_nodes=M, n_sweeps=60,
                   predictor="ros2")
    assert X[0, 0] == pytest.approx(pade(M, z), rel=1e-12)


def observed_orders(M, K, dts, rate=3.0, y0=0.05, T=2.0):
    mdl = TEST_LOGISTIC.with_params(rate=rate)
    exact = Logistic.exact(y0, T, dict(rate=rate))
    errs = []
    for dt in dts:
        X, _ = advance(mdl, np.array([[y0]]), dt=dt, n_steps=int(round(T / dt)), n_nodes=M,
                       n_sweeps=K, predictor="ros2")
        errs.append(X[0, 0] - exact)
    return local_orders(errs)


@pytest.mark.parametrize("M,K,p", [(2, 0, 2), (2, 1, 2), (3, 0, 2), (3, 1, 3), (3, 2, 4), (4, 2, 4)])
def test_global_order_with_sweeps(M, K, p):
    o = observed_orders(M, K, (0.1, 0.05, 0.025))
    assert o[-1] > p - 0.25


@pytest.mark.parametrize("M,K", [(2, 1), (2, 2), (3, 2)])
def test_collocation_order_caps_the_gain(M, K):
    # asymptotic regime, above the rounding floor
    o = observed_orders(M, K, (0.025, 0.0125, 0.00625) if M == 2 else (0.1, 0.05, 0.025))
    assert abs(o[-1] - (2 * M - 2)) < 0.2


@pytest.mark.slow
def test_second_order_on_tt06():
    """A 19-state nonlinear system (catches transposed or misplaced Jacobian
    use that a scalar problem cannot): ROS2 alone, self-convergence on a
    smooth window against a far more accurate oracle run."""
    x = tt06.published_initial()
    x[0] = -75.0
    X0 = x[:, None]
    T = 1.0
    ref, _ = advance(TT06, X0, dt=0.025 / 4, n_steps=160, n_nodes=5, n_sweeps=8, tol=1e-14)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        X, _ = advance(TT06, X0, dt=dt, n_steps=int(round(T / dt)), n_nodes=2, n_sweeps=0,
                       predictor="ros2")
        errs.append(np.max(np.abs(X - ref) / np.maximum(np.abs(ref), TT06.newton_scale[:, None])))
    o = local_orders(errs)
    assert o[-1] > 1.8
