"""Pins of the oracle's adaptive time stepping with the ROS2 predictor (paper
section 3.3.1: the embedded solution chooses the next step; section 4: the
partitioned strategy uses adaptive steps capped at 0.05 ms).

The paper gives no controller, so these pin what any such controller must
satisfy, plus the behaviour that follows from the embedded order:
* every accepted attempt has err <= tol, every rejected one err > tol, the
  run ends exactly at t_end and no step exceeds dt_max;
* steps never cross a stimulus switching time; a step that reaches one ends
  there exactly;
* with the first-order embedding the local estimate is O(tau^2), so the step
  count grows like tol^(-1/2): a factor of 100 in tol is about a factor of 10
  in steps;
* a tighter tolerance gives a smaller global error, on a problem with a
  closed form;
* on a cell model the adaptive run reproduces a fine fixed-step run.
"""
import numpy as np
import pytest

from oracle import rest
from oracle.adaptive import Q_MAX, advance_adaptive, step_factor
from oracle.models import LR91, TEST_LINEAR, TEST_LOGISTIC
from oracle.sdc import advance
from oracle.testmodels import Logistic


def run_logistic(tol, **kw):
    mdl = TEST_LOGISTIC.with_params(rate=3.0)
    kw.setdefault("dt_init", 1e-3)
    kw.setdefault("dt_max", 0.5)
    return advance_adaptive(mdl, np.array([[0.05]]), t_end=2.0, err_tol=tol, **kw)


def test_bookkeeping_invariants():
    X, st = run_logistic(1e-5, dt_max=0.05)
    assert st.done and not st.failed and st.t == 2.0
    h = st.history
    assert st.accepted + st.rejected == len(h)
    for t, tau, err, ok in h:
        assert tau <= 0.05
        assert ok == (err <= 1e-5)
    acc = [r for r in h if r[3]]
    # accepted steps tile [0, 2]: each starts where the previous one ended
    for (t0, tau0, _, _), (t1, _, _, _) in zip(acc[:-1], acc[1:]):
        assert t1 == pytest.approx(t0 + tau0, abs=1e-14)
    assert acc[-1][0] + acc[-1][1] == pytest.approx(2.0, abs=1e-14)


def test_rejection_shrinks_and_retries():
    # a first step far too large for the tolerance is rejected and retried smaller
    X, st = run_logistic(1e-7, dt_init=0.5)
    t0, tau0, err0, ok0 = st.history[0]
    t1, tau1, _, _ = st.history[1]
    assert not ok0 and t1 == t0 == 0.0
    assert tau1 == pytest.approx(tau0 * step_factor(err0, 1e-7), rel=1e-15)
    assert tau1 < tau0


def test_loose_tolerance_grows_to_dt_max():
    mdl = TEST_LINEAR.with_params(lam=-0.1, b=0.0)
    X, st = advance_adaptive(mdl, np.array([[1.0]]), t_end=3.0, dt_init=0.01, dt_max=0.05,
                             err_tol=1.0)
    taus = [r[1] for r in st.history]
    assert st.rejected == 0
    assert taus[:3] == pytest.approx([0.01, 0.01 * Q_MAX, 0.01 * Q_MAX ** 2], rel=1e-15)
    assert max(taus) == 0.05


def test_step_count_scales_like_tol_to_minus_half():
    counts = [run_logistic(tol)[1].accepted for tol in (1e-4, 1e-6, 1e-8)]
    r = np.array(counts[1:]) / np.array(counts[:-1])
    assert np.all((r > 7.0) & (r < 13.0)), counts


def test_tighter_tolerance_smaller_error():
    exact = Logistic.exact(0.05, 2.0, dict(rate=3.0))
    errs = [abs(run_logistic(tol)[0][0, 0] - exact) for tol in (1e-3, 1e-5, 1e-7)]
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    assert errs[0] < 1e-3


def test_stimulus_switching_times_are_breakpoints():
    x = rest.lr91_rest()[:, None]
    X, st = advance_adaptive(LR91, x, t_end=3.0, dt_init=0.013, dt_max=0.05, err_tol=1e-3,
                             i_stim=np.array([-80.0]), stim_on=0.5, stim_off=1.5)
    acc = [r for r in st.history if r[3]]
    starts = [r[0] for r in acc]
    assert 0.5 in starts and 1.5 in starts
    for t, tau, _, _ in acc:
        assert not (t < 0.5 < t + tau - 1e-15) and not (t < 1.5 < t + tau - 1e-15)
    assert X[0, 0] > 0.0        # the stimulus fired an upstroke


@pytest.mark.slow
def test_adaptive_matches_fine_fixed_step_on_lr91():
    """LR91 single cell, stimulated, 10 ms through the upstroke: the adaptive
    ROS2 + SDC(M=2, K=1) run at tol 1e-5 against the Newton predictor with
    3 nodes and 3 sweeps at dt = 0.005 (order 4; halving its step moves V by
    1e-3 mV)."""
    x = rest.lr91_rest()[:, None]
    stim = dict(i_stim=np.array([-80.0]), stim_on=0.0, stim_off=1.0)
    ref, _ = advance(LR91, x, dt=0.005, n_steps=2000, n_nodes=3, n_sweeps=3, **stim)
    X, st = advance_adaptive(LR91, x, t_end=10.0, dt_init=0.01, dt_max=0.05, err_tol=1e-5, **stim)
    assert st.done and ref[0, 0] > -40.0           # in the plateau after the upstroke
    assert abs(X[0, 0] - ref[0, 0]) < 0.01          # mV
    assert st.accepted < 10.0 / 0.005               # fewer steps than the fixed fine run
