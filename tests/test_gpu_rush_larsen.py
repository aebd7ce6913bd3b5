"""GPU vs oracle for the Rush-Larsen predictor (exponential gating steps at
frozen state, backward Euler by Newton on the V/concentration core), through
the C ABI: every model x precision, several node and sweep counts, a vertex
count with a ragged tail, stimulated and diffusion-driven vertices.

Bar: fp64 max|dV| / max|V_ref| <= 1e-10 (other states <= 1e-9 of their
scale); mixed <= 1e-4 on V and the fp64-held concentrations, against the fp64
oracle.  Without gating states (the scalar test problems) the predictor must
give exactly what the Newton predictor gives."""
import numpy as np
import pytest

from gpu_helpers import MODEL_OF, gpu_tensor, rel_errors, say
from oracle.sdc import advance
from paper_2510_27447_amd.workloads import initial_state

pytestmark = pytest.mark.gpu

N_SMALL = 130


def inputs(model, N=N_SMALL, seed=31):
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.tile(initial_state(model)[:, None], (1, N))
    x0[0] += rng.uniform(-3.0, 3.0, N)
    stim = np.where(rng.random(N) < 0.3, -80.0 if model == "LR91" else -100.0, 0.0)
    diff = rng.normal(0.0, 0.5, N)
    return x0, stim, diff


def run(model, precision, x0, stim, diff, dt, n_steps, M, K, predictor):
    import torch
    from paper_2510_27447_amd import ionic as I
    sim = I.Simulation(model, x0, precision=precision)
    sim.set_predictor(predictor)
    sim.step(0.0, dt, n_steps, M, K, gpu_tensor(stim), 0.0, 0.5, gpu_tensor(diff))
    torch.cuda.synchronize()
    X, st = sim.readback(), sim.stats()
    sim.close()
    return X, st


@pytest.mark.parametrize("model", ["LR91", "TT06"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("M,K", [(2, 0), (2, 1), (3, 3), (4, 3)])
def test_rush_larsen_matches_oracle(model, precision, M, K):
    say("case rush-larsen", model, precision, M, K)
    x0, stim, diff = inputs(model)
    dt, n_steps = 0.02, 25
    Xg, st = run(model, precision, x0, stim, diff, dt, n_steps, M, K, "rush_larsen")
    Xo, so = advance(MODEL_OF[model], x0, dt=dt, n_steps=n_steps, n_nodes=M, n_sweeps=K,
                     i_stim=stim, stim_on=0.0, stim_off=0.5, i_diff=diff,
                     tol=1e-10, predictor="rush_larsen")
    err = rel_errors(Xg, Xo, list(range(Xo.shape[0])))
    say("  V max/rms", err[0], "worst", max(err.items(), key=lambda kv: kv[1][0]))
    if precision == "fp64":
        assert err[0][0] <= 1e-10
        assert max(e[0] for e in err.values()) <= 1e-9
        assert st["newton_iters"] == so.newton_iters_total
    else:
        n64 = 2 if model == "LR91" else 6
        for i in range(n64):
            assert err[i][0] <= 1e-4, i
        assert max(e[0] for e in err.values()) <= 1e-3
    assert st["newton_solves"] == N_SMALL * n_steps * (M - 1)
    assert st["n_nonfinite"] == 0


def test_without_gating_states_equals_newton_predictor():
    x0 = np.linspace(0.1, 0.9, 70)[None, :]
    a, sa = run("TEST_LOGISTIC", "fp64", x0, np.zeros(70), np.zeros(70), 0.2, 7, 3, 2, "rush_larsen")
    b, sb = run("TEST_LOGISTIC", "fp64", x0, np.zeros(70), np.zeros(70), 0.2, 7, 3, 2, "newton")
    assert np.array_equal(a, b)
    assert sa["newton_iters"] == sb["newton_iters"]


def test_fused_steps_equal_one_step_launches():
    """The whole step loop in one launch and one launch per step agree bitwise
    (no state other than X survives a step)."""
    import torch
    from paper_2510_27447_amd import ionic as I
    x0, stim, diff = inputs("TT06", N=90, seed=5)
    st, df = gpu_tensor(stim), gpu_tensor(diff)
    a = I.Simulation("TT06", x0)
    a.set_predictor("rush_larsen")
    a.step(0.0, 0.02, 20, 3, 2, st, 0.0, 0.5, df)
    b = I.Simulation("TT06", x0)
    b.set_predictor("rush_larsen")
    for k in range(20):
        b.step(k * 0.02, 0.02, 1, 3, 2, st, 0.0, 0.5, df)
    torch.cuda.synchronize()
    assert np.array_equal(a.readback(), b.readback())
    a.close()
    b.close()
