"""Pins of the oracle's Rush-Larsen predictor (exponential gating steps at
frozen state, backward Euler by Newton on the V/concentration core).

* Under voltage clamp every voltage-gated gate obeys a linear ODE with
  constant coefficients, which the exponential step integrates exactly: the
  predictor alone reproduces g_inf + (g0 - g_inf) exp(-t/tau) for any step,
  where backward Euler only approximates it.
* Without gating states (the scalar test problems) the predictor is the
  backward-Euler Newton predictor, to the last bit.
* The core states returned satisfy the backward-Euler equation of the core
  with the gates held, to the Newton tolerance.
* Orders on the cell models: first order alone, one more per sweep up to the
  Lobatto cap, like the other predictors.
"""
import numpy as np
import pytest

from oracle import lr91, rest, tt06
from oracle.models import LR91, TEST_LINEAR, TEST_LOGISTIC, TT06
from oracle.rush_larsen import phi, rush_larsen_be, split_states
from oracle.sdc import Stats, advance


def test_phi():
    z = np.array([0.0, 1e-12, -1e-6, -0.5, -30.0, 2.0])
    want = np.array([1.0, 1.0 + 5e-13, (np.exp(-1e-6) - 1) / -1e-6, (np.exp(-0.5) - 1) / -0.5,
                     (np.exp(-30.0) - 1) / -30.0, (np.exp(2.0) - 1) / 2.0])
    np.testing.assert_allclose(phi(z), want, rtol=1e-9)


def test_split():
    core, gating = split_states(TT06)
    assert [TT06.state_names[i] for i in core] == ["V", "Cai", "CaSR", "CaSS", "Nai", "Ki"]
    assert len(gating) == 13
    core, gating = split_states(LR91)
    assert [LR91.state_names[i] for i in core] == ["V", "Cai"] and len(gating) == 6


@pytest.mark.parametrize("model", ["LR91", "TT06"])
def test_gates_exact_under_voltage_clamp(model):
    if model == "LR91":
        mdl, V = LR91, np.array([-30.0, 10.0, -60.0])
        X0 = np.tile(rest.lr91_rest()[:, None], (1, 3))
        r = lr91.rates(V)
        kin = {g: (r["a" + g] / (r["a" + g] + r["b" + g]), r["a" + g] + r["b" + g]) for g in lr91.GATES}
    else:
        mdl, V = TT06, np.array([-30.0, 10.0, -70.0])
        X0 = np.tile(tt06.published_initial()[:, None], (1, 3))
        g = tt06.gate_kinetics(V)
        kin = {k: (g[k + "_inf"], 1.0 / g[k + "_tau"]) for k in tt06.V_GATES}
    X0[0] = V
    dt, n = 0.7, 12           # steps far beyond the fastest gate time constants
    X, _ = advance(mdl, X0, dt=dt, n_steps=n, n_nodes=2, n_sweeps=0, clamp_v=True, tol=1e-14,
                   predictor="rush_larsen")
    for name, (g_inf, rate) in kin.items():
        i = mdl.state_names.index(name)
        expect = g_inf + (X0[i] - g_inf) * np.exp(-rate * dt * n)
        np.testing.assert_allclose(X[i], expect, rtol=1e-11, atol=1e-14, err_msg=name)
    # at this step backward Euler's factor (1 + rate dt)^-n is far from exp(-rate t)
    # for some gate, so exactness is not a property of any implicit step
    gap = max(np.max(np.abs((1.0 + rate * dt) ** -n - np.exp(-rate * dt * n)))
              for g_inf, rate in kin.values())
    assert gap > 1e-3


@pytest.mark.parametrize("mdl", [TEST_LINEAR.with_params(lam=-3.0, b=0.5), TEST_LOGISTIC],
                         ids=["linear", "logistic"])
def test_no_gating_states_means_backward_euler_newton(mdl):
    x0 = np.array([[0.2, 0.7, 1.3]])
    a, sa = advance(mdl, x0, dt=0.3, n_steps=5, n_nodes=3, n_sweeps=2, predictor="rush_larsen")
    b, sb = advance(mdl, x0, dt=0.3, n_steps=5, n_nodes=3, n_sweeps=2)
    assert np.array_equal(a, b)
    assert sa.newton_iters_total == sb.newton_iters_total


@pytest.mark.parametrize("model", ["LR91", "TT06"])
def test_core_solves_backward_euler_with_gates_held(model):
    mdl = LR91 if model == "LR91" else TT06
    x = (rest.lr91_rest() if model == "LR91" else tt06.published_initial())[:, None].repeat(4, 1)
    x[0] = [-84.0, -60.0, -20.0, 15.0]
    dtau, stim, diff = 0.04, np.array([-50.0, 0.0, 0.0, 0.0]), np.array([0.0, 0.3, -0.2, 0.0])
    st = Stats(per_vertex_iters=np.zeros(4, dtype=np.int64))
    Y = rush_larsen_be(mdl, x, dtau, stim, diff, 1e-13, 20, False, st)
    core, gating = split_states(mdl)
    F = mdl.F(Y, stim, diff)
    resid = Y[core] - x[core] - dtau * F[core]
    scale = np.maximum(np.abs(Y[core]), mdl.newton_scale[core][:, None])
    assert np.max(np.abs(resid) / scale) < 1e-12
    assert st.n_nonconverged == 0


def _orders(model, M, K, T=1.0, dts=(0.1, 0.05, 0.025)):
    x = (rest.lr91_rest() if model is LR91 else tt06.published_initial()).copy()
    x[0] = -72.0 if model is LR91 else -75.0
    X0 = x[:, None]
    dref = dts[-1] / 4
    ref, _ = advance(model, X0, dt=dref, n_steps=int(round(T / dref)), n_nodes=5, n_sweeps=8,
                     tol=1e-14)
    errs = []
    for dt in dts:
        X, _ = advance(model, X0, dt=dt, n_steps=int(round(T / dt)), n_nodes=M, n_sweeps=K,
                       tol=1e-14, predictor="rush_larsen")
        errs.append(np.max(np.abs(X - ref) / np.maximum(np.abs(ref), model.newton_scale[:, None])))
    errs = np.array(errs)
    return np.log2(errs[:-1] / errs[1:])


@pytest.mark.slow
@pytest.mark.parametrize("model", [LR91, TT06], ids=["LR91", "TT06"])
@pytest.mark.parametrize("M,K,p", [(2, 0, 1), (3, 2, 3)], ids=["RL", "M3K2"])
def test_order_on_cell_models(model, M, K, p):
    o = _orders(model, M, K)
    assert o[-1] > p - 0.3


@pytest.mark.slow
def test_one_trapezoidal_sweep_tends_to_second_order():
    """The paper's correction on the Rush-Larsen value.  The splitting error of
    the exponential gate step is large, so second order shows only at small
    steps: the observed order climbs past 1.6 (1.70, then 1.82 at half the step,
    in the oracle's own run) where the predictor alone stays at 1."""
    o = _orders(LR91, 2, 1, T=0.25, dts=(0.0125, 0.00625, 0.003125))
    assert o[-1] > 1.6
    assert _orders(LR91, 2, 0, T=0.25, dts=(0.0125, 0.00625, 0.003125))[-1] < 1.3
