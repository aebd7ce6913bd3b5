"""GPU vs oracle for the ROS2 predictor (paper section 3.3.1, equation
rb_system) and the adaptive step control built on its embedded solution.

Fixed steps: every model x precision, the paper's scheme (2 nodes, 1
correction) and multi-node variants, a vertex count with a ragged tail,
stimulated and diffusion-driven vertices.  Bar: fp64 max|dV| / max|V_ref|
<= 1e-10 (other states <= 1e-9 of their scale); mixed <= 1e-4 on V and the
fp64-held concentrations, against the fp64 oracle.

Adaptive: the attempt history (t, tau, err, accepted) and the final state
against the oracle's controller on the same inputs.  Accept/reject decisions
must agree exactly; t and tau to 1e-9 relative (err is a maximum over
vertices of a cancelling difference, so it carries more rounding than the
states); the final state to the fixed-step bars.
"""
import numpy as np
import pytest

from gpu_helpers import MODEL_OF, gpu_tensor, rel_errors, say
from oracle.adaptive import advance_adaptive
from oracle.sdc import advance
from paper_2510_27447_amd.workloads import initial_state

pytestmark = pytest.mark.gpu

N_SMALL = 130


def inputs(model, N=N_SMALL, seed=11):
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.tile(initial_state(model)[:, None], (1, N))
    x0[0] += rng.uniform(-3.0, 3.0, N)
    stim = np.where(rng.random(N) < 0.3, -80.0 if model == "LR91" else -100.0, 0.0)
    diff = rng.normal(0.0, 0.5, N)
    return x0, stim, diff


def check(model, precision, Xg, Xo):
    err = rel_errors(Xg, Xo, list(range(Xo.shape[0])))
    say("  V max/rms", err[0], "worst", max(err.items(), key=lambda kv: kv[1][0]))
    if precision == "fp64":
        assert err[0][0] <= 1e-10
        assert max(e[0] for e in err.values()) <= 1e-9
    else:
        n64 = 2 if model == "LR91" else 6
        for i in range(n64):
            assert err[i][0] <= 1e-4, i
        assert max(e[0] for e in err.values()) <= 1e-3


@pytest.mark.parametrize("model", ["LR91", "TT06"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("M,K", [(2, 1), (2, 0), (3, 2), (4, 3)])
def test_fixed_step_ros2_matches_oracle(model, precision, M, K):
    import torch
    from paper_2510_27447_amd import ionic as I
    say("case ros2 fixed", model, precision, M, K)
    x0, stim, diff = inputs(model)
    dt, n_steps = 0.05, 12
    sim = I.Simulation(model, x0, precision=precision)
    sim.set_predictor("ros2")
    sim.step(0.0, dt, n_steps, M, K, gpu_tensor(stim), 0.0, 0.3, gpu_tensor(diff))
    torch.cuda.synchronize()
    Xg = sim.readback()
    st = sim.stats()
    sim.close()
    Xo, _ = advance(MODEL_OF[model], x0, dt=dt, n_steps=n_steps, n_nodes=M, n_sweeps=K,
                    i_stim=stim, stim_on=0.0, stim_off=0.3, i_diff=diff, predictor="ros2")
    check(model, precision, Xg, Xo)
    assert st["vertex_steps"] == N_SMALL * n_steps
    assert st["newton_iters"] == 0 and st["newton_solves"] == 0
    assert st["n_nonfinite"] == 0


@pytest.mark.parametrize("z", [-0.5, -3.0, 0.4])
def test_ros2_on_linear_problem(z):
    """y' = lam y: one ROS2 step (no sweeps) and the paper's scheme, on a
    problem where the oracle's result is a fixed rational function of z."""
    import torch
    from paper_2510_27447_amd import ionic as I
    dt = 0.1
    x0 = np.linspace(-1.0, 2.0, 67)[None, :]
    for K in (0, 1):
        sim = I.Simulation("TEST_LINEAR", x0, params=[z / dt, 0.0])
        sim.set_predictor("ros2")
        sim.step(0.0, dt, 3, 2, K)
        torch.cuda.synchronize()
        Xg = sim.readback()
        sim.close()
        Xo, _ = advance(MODEL_OF["TEST_LINEAR"].with_params(lam=z / dt, b=0.0), x0, dt=dt,
                        n_steps=3, n_nodes=2, n_sweeps=K, predictor="ros2")
        assert np.max(np.abs(Xg - Xo)) <= 1e-14 * np.max(np.abs(Xo))


def test_batch_with_ros2_is_identical_to_single_calls():
    import torch
    from paper_2510_27447_amd import ionic as I
    x0, stim, diff = inputs("TT06", N=100, seed=3)
    st, df = gpu_tensor(stim), gpu_tensor(diff)
    sims = [I.Simulation("TT06", x0[:, :70], precision="mixed"),
            I.Simulation("TT06", x0[:, 30:], precision="mixed")]
    for s, lo, hi in ((sims[0], 0, 70), (sims[1], 30, 100)):
        s.set_predictor("ros2")
        I.ionic_set_inputs(s.handle, 0.0, 0.05, 2, 1, st[lo:hi], 0.0, 0.5, df[lo:hi])
    I.reaction_sdc_step_batch([s.handle for s in sims], [6, 9])
    torch.cuda.synchronize()
    for s, lo, hi, k in ((sims[0], 0, 70, 6), (sims[1], 30, 100, 9)):
        ref = I.Simulation("TT06", x0[:, lo:hi], precision="mixed")
        ref.set_predictor("ros2")
        ref.step(0.0, 0.05, k, 2, 1, st[lo:hi], 0.0, 0.5, df[lo:hi])
        torch.cuda.synchronize()
        assert np.array_equal(s.readback(), ref.readback())
        ref.close()
        s.close()


def run_adaptive_pair(model, precision, t_end, err_tol, M=2, K=1, N=N_SMALL, seed=21,
                      dt_init=0.01, dt_max=0.05, max_attempts=4000, t_on=0.0, t_off=1.0):
    from paper_2510_27447_amd import ionic as I
    x0, stim, diff = inputs(model, N=N, seed=seed)
    sim = I.Simulation(model, x0, precision=precision)
    res, hist = sim.adaptive(0.0, t_end, dt_init, dt_max, err_tol, n_nodes=M, n_sweeps=K,
                             i_stim=gpu_tensor(stim), stim_t_on=t_on, stim_t_off=t_off,
                             i_diff=gpu_tensor(diff), max_attempts=max_attempts, history=True)
    Xg = sim.readback()
    sim.close()
    Xo, so = advance_adaptive(MODEL_OF[model], x0, t_end=t_end, dt_init=dt_init, dt_max=dt_max,
                              err_tol=err_tol, n_nodes=M, n_sweeps=K, i_stim=stim, stim_on=t_on,
                              stim_off=t_off, i_diff=diff, max_attempts=max_attempts)
    return res, hist, Xg, so, Xo


@pytest.mark.parametrize("model", ["LR91", "TT06"])
@pytest.mark.parametrize("M,K", [(2, 1), (3, 2)])
def test_adaptive_fp64_matches_oracle(model, M, K):
    say("case adaptive fp64", model, M, K)
    res, hist, Xg, so, Xo = run_adaptive_pair(model, "fp64", 4.0, 1e-3, M, K)
    say("  gpu", res, "oracle acc/rej", so.accepted, so.rejected)
    ho = np.array([(t, tau, err, 1.0 if ok else 0.0) for t, tau, err, ok in so.history])
    assert res["reached"] == 1 and res["failed"] == 0 and res["t"] == 4.0
    assert (res["accepted"], res["rejected"]) == (so.accepted, so.rejected)
    assert hist.shape == ho.shape
    assert np.array_equal(hist[:, 3], ho[:, 3])
    assert np.allclose(hist[:, 0], ho[:, 0], rtol=1e-9, atol=1e-12)
    assert np.allclose(hist[:, 1], ho[:, 1], rtol=1e-9, atol=0.0)
    assert np.allclose(hist[:, 2], ho[:, 2], rtol=1e-6, atol=1e-13)
    check(model, "fp64", Xg, Xo)


@pytest.mark.parametrize("model", ["LR91", "TT06"])
def test_adaptive_mixed_matches_fp64_oracle(model):
    say("case adaptive mixed", model)
    res, hist, Xg, so, Xo = run_adaptive_pair(model, "mixed", 4.0, 1e-3)
    say("  gpu", res, "oracle acc/rej", so.accepted, so.rejected)
    assert res["reached"] == 1 and res["t"] == 4.0
    assert abs(res["accepted"] - so.accepted) <= 2
    check(model, "mixed", Xg, Xo)


@pytest.mark.parametrize("t_end,n_acc", [(0.03, 2), (0.07, 3)])
def test_adaptive_result_lands_in_state_buffer(t_end, n_acc):
    """Even and odd accepted counts (the state ends in either buffer): with a
    loose tolerance every attempt is accepted and the step doubles, so the
    counts are known: 0.01 + 0.02 = 0.03; 0.01 + 0.02 + 0.04 (cut at 0.07)."""
    from paper_2510_27447_amd import ionic as I
    x0 = np.linspace(0.5, 1.5, 70)[None, :]
    sim = I.Simulation("TEST_LINEAR", x0, params=[-0.1, 0.0])
    res = sim.adaptive(0.0, t_end, 0.01, 0.05, 1.0)
    Xg = sim.readback()
    sim.close()
    Xo, so = advance_adaptive(MODEL_OF["TEST_LINEAR"].with_params(lam=-0.1, b=0.0), x0,
                              t_end=t_end, dt_init=0.01, dt_max=0.05, err_tol=1.0)
    assert res["accepted"] == so.accepted == n_acc and res["rejected"] == 0
    assert np.max(np.abs(Xg - Xo)) <= 1e-14


def test_adaptive_attempt_cap_keeps_last_accepted_state():
    say("case adaptive cap")
    res, hist, Xg, so, Xo = run_adaptive_pair("LR91", "fp64", 4.0, 1e-3, max_attempts=17)
    assert res["reached"] == 0 and res["failed"] == 1
    assert res["accepted"] + res["rejected"] == 17 == len(so.history)
    assert res["t"] == pytest.approx(so.t, rel=1e-12) and so.t < 4.0
    check("LR91", "fp64", Xg, Xo)
