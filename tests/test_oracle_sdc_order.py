"""Convergence-order pins of the oracle SDC (paper section 4.2, table
partitioned_order: the first-order scheme gains one order with one
correction).  On the logistic problem, which has a closed form, the observed
order under dt-halving must be at least min(K+1, 2M-2) (one order per sweep,
capped by the Lobatto collocation order), equal to 2M-2 once the cap binds,
and 1 without sweeps."""
import numpy as np
import pytest

from oracle.models import TEST_LOGISTIC
from oracle.sdc import advance
from oracle.testmodels import Logistic

RATE, Y0, T = 3.0, 0.05, 2.0


def observed_orders(M, K, dts):
    mdl = TEST_LOGISTIC.with_params(rate=RATE)
    exact = Logistic.exact(Y0, T, dict(rate=RATE))
    errs = []
    for dt in dts:
        X, _ = advance(mdl, np.array([[Y0]]), dt=dt, n_steps=int(round(T / dt)),
                       n_nodes=M, n_sweeps=K, tol=1e-15)
        errs.append(abs(X[0, 0] - exact))
    errs = np.array(errs)
    return np.log2(errs[:-1] / errs[1:])


def test_predictor_alone_is_first_order():
    p = observed_orders(3, 0, (0.02, 0.01, 0.005))
    assert 0.85 < p[-1] < 1.15


@pytest.mark.parametrize("M,K", [(2, 1), (3, 1), (3, 2), (4, 2), (4, 3), (5, 4)])
def test_each_sweep_gains_an_order(M, K):
    p = observed_orders(M, K, (0.1, 0.05, 0.025))
    assert p[-1] > min(K + 1, 2 * M - 2) - 0.2


@pytest.mark.parametrize("M,K", [(2, 1), (2, 3), (3, 3), (4, 5)])
def test_collocation_order_caps_the_gain(M, K):
    p = observed_orders(M, K, (0.1, 0.05, 0.025))
    assert abs(p[-1] - (2 * M - 2)) < 0.3
