"""SDC order on the cell models and the Newton bookkeeping of the oracle.

Paper section 4.2, table partitioned_order: without the correction the
partitioned scheme is first order, with one trapezoidal correction second
order.  Per vertex (diffusion fixed) the same holds for the M = 2, K = 1
scheme, and more sweeps/nodes give min(K+1, 2M-2).  Checked on a smooth,
unstimulated window from a perturbed state, against the oracle itself with
5 nodes and 8 sweeps (order 8) at a 4x finer step, far more accurate than
every tested run.  The settings of the benchmark workloads (3 nodes and 3
sweeps; 4 nodes and 3 sweeps) are checked for fourth order.
"""
import numpy as np
import pytest

from oracle import rest, tt06
from oracle.models import LR91, TT06
from oracle.sdc import advance


def perturbed(model):
    if model is LR91:
        x = rest.lr91_rest()
        x[0] = -72.0          # subthreshold depolarisation, gates out of equilibrium
    else:
        x = tt06.published_initial()
        x[0] = -75.0
    return x[:, None]


def orders(model, M, K, T=1.0, dts=(0.1, 0.05, 0.025)):
    X0 = perturbed(model)
    dref = dts[-1] / 4     # reference: 5 nodes, 8 sweeps (order 8)
    ref, _ = advance(model, X0, dt=dref, n_steps=int(round(T / dref)), n_nodes=5, n_sweeps=8, tol=1e-14)
    errs = []
    for dt in dts:
        X, _ = advance(model, X0, dt=dt, n_steps=int(round(T / dt)), n_nodes=M, n_sweeps=K, tol=1e-14)
        errs.append(abs(X[0, 0] - ref[0, 0]))
    errs = np.array(errs)
    return np.log2(errs[:-1] / errs[1:])


@pytest.mark.slow
@pytest.mark.parametrize("model", [LR91, TT06], ids=["LR91", "TT06"])
@pytest.mark.parametrize("M,K,p", [(2, 0, 1), (2, 1, 2), (3, 2, 3)], ids=["noSDC", "paperSDC", "M3K2"])
def test_order_on_cell_models(model, M, K, p):
    o = orders(model, M, K)
    assert o[-1] > p - 0.3


@pytest.mark.slow
@pytest.mark.parametrize("model", [LR91, TT06], ids=["LR91", "TT06"])
@pytest.mark.parametrize("M,K", [(3, 3), (4, 3)], ids=["M3K3", "M4K3"])
def test_fourth_order_at_the_benchmark_settings(model, M, K):
    """The slab's setting (3 nodes, 3 sweeps) and the spiral's (4 nodes, 3
    sweeps) are fourth order: min(K+1, 2M-2) = 4.  The stiff gates keep the
    coarse steps pre-asymptotic, so the order is the least-squares slope of
    log|V error| over four halvings from 0.1 ms; a dropped sweep, a wrong
    quadrature weight or node would leave it at 3 or below."""
    dts = np.array((0.1, 0.05, 0.025, 0.0125))
    X0 = perturbed(model)
    T, dref = 1.0, dts[-1] / 4
    ref, _ = advance(model, X0, dt=dref, n_steps=int(round(T / dref)), n_nodes=5, n_sweeps=8,
                     tol=1e-14)
    errs = []
    for dt in dts:
        X, _ = advance(model, X0, dt=dt, n_steps=int(round(T / dt)), n_nodes=M, n_sweeps=K,
                       tol=1e-14)
        errs.append(abs(X[0, 0] - ref[0, 0]))
    slope = np.polyfit(np.log2(dts), np.log2(errs), 1)[0]
    assert slope > 3.6, (errs, slope)


def test_newton_maxit_is_counted_not_raised():
    X0 = np.tile(rest.lr91_rest()[:, None], (1, 4))
    X, st = advance(LR91, X0, dt=0.02, n_steps=3, n_nodes=3, n_sweeps=1, tol=0.0, maxit=4)
    assert st.n_nonconverged == 4 * 3 * 2
    assert st.newton_it_max == 4
    assert np.all(np.isfinite(X))


def test_nonfinite_is_counted():
    X0 = np.tile(rest.lr91_rest()[:, None], (1, 4))
    d = np.zeros(4)
    d[1] = np.nan
    X, st = advance(LR91, X0, dt=0.02, n_steps=2, n_nodes=2, n_sweeps=1, i_diff=d)
    assert st.n_nonfinite == 1
    assert np.all(np.isfinite(X[:, [0, 2, 3]]))


def test_vertices_are_independent():
    X0 = np.tile(tt06.published_initial()[:, None], (1, 3))
    X0[0] += np.array([0.0, 20.0, -2.0])
    stim = np.array([-30.0, 0.0, -30.0])
    Xa, _ = advance(TT06, X0, dt=0.02, n_steps=5, n_nodes=3, n_sweeps=2, i_stim=stim, stim_on=0, stim_off=1)
    Xb, _ = advance(TT06, X0[:, 1:2], dt=0.02, n_steps=5, n_nodes=3, n_sweeps=2, i_stim=stim[1:2], stim_on=0, stim_off=1)
    assert np.array_equal(Xa[:, 1], Xb[:, 0])
