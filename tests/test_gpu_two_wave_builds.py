"""The step kernels held to two wavefronts per SIMD (256 registers per lane)
run only in launches of at least 2048 workgroups; smaller launches take the
one-wavefront build of the same instantiation.  Every such instantiation (LR91
with 2 and 3 nodes, both precisions, each predictor; TT06 mixed with 2 nodes,
ROS2 and Rush-Larsen) is run here on 2048 x 64 + 37 vertices (a ragged tail),
and a seeded sample of its vertices is compared (a) with the same vertices run
alone, which is a launch of one workgroup and so the one-wavefront build: the
two builds differ only in register allocation, so the states must agree bit
for bit; and (b) with the fp64 oracle at the parity bars (fp64: V within 1e-10
of max|V|, every state within 1e-9 of its scale; mixed: V and the fp64-held
concentrations within 1e-4, gates within 1e-3)."""
import numpy as np
import pytest

from gpu_helpers import MODEL_OF, gpu_tensor, say
from oracle.sdc import advance
from paper_2510_27447_amd.workloads import initial_state

pytestmark = pytest.mark.gpu

N_BIG = 2048 * 64 + 37
CASES = ([("LR91", p, M, pred) for p in ("fp64", "mixed") for M in (2, 3)
          for pred in ("newton", "ros2", "rush_larsen")]
         + [("TT06", "mixed", 2, "ros2"), ("TT06", "mixed", 2, "rush_larsen")])


def run(model, precision, pred, M, K, x0, stim, diff, dt, n_steps):
    import torch
    from paper_2510_27447_amd import ionic as I
    sim = I.Simulation(model, x0, precision=precision)
    sim.set_predictor(pred)
    sim.step(0.0, dt, n_steps, M, K, gpu_tensor(stim), 0.0, 0.3, gpu_tensor(diff))
    torch.cuda.synchronize()
    X = sim.readback()
    st = sim.stats()
    sim.close()
    return X, st


@pytest.mark.parametrize("model,precision,M,pred", CASES,
                         ids=["%s-%s-M%d-%s" % c for c in CASES])
def test_two_wavefront_build_matches(model, precision, M, pred):
    rng = np.random.Generator(np.random.PCG64(29))
    x0 = np.tile(initial_state(model)[:, None], (1, N_BIG))
    x0[0] += rng.uniform(-3.0, 3.0, N_BIG)
    stim = np.where(rng.random(N_BIG) < 0.2, -80.0 if model == "LR91" else -100.0, 0.0)
    diff = rng.normal(0.0, 0.5, N_BIG)
    K = M - 1
    dt, n_steps = (0.02, 20) if pred != "ros2" else (0.05, 12)
    say("case", model, precision, M, K, pred, N_BIG)
    Xb, st = run(model, precision, pred, M, K, x0, stim, diff, dt, n_steps)
    assert st["n_nonfinite"] == 0
    idx = np.unique(np.concatenate([[0, 1, N_BIG - 1, N_BIG - 37],
                                    rng.choice(np.nonzero(stim)[0], 6, replace=False),
                                    rng.choice(N_BIG, 10, replace=False)]))
    Xs, _ = run(model, precision, pred, M, K, x0[:, idx], stim[idx], diff[idx], dt, n_steps)
    same = np.array_equal(Xb[:, idx], Xs)
    say("  bitwise equal to the one-wavefront build:", same)
    assert same
    Xo, _ = advance(MODEL_OF[model], x0[:, idx], dt=dt, n_steps=n_steps, n_nodes=M, n_sweeps=K,
                    i_stim=stim[idx], stim_on=0.0, stim_off=0.3, i_diff=diff[idx],
                    predictor=pred)
    mdl = MODEL_OF[model]
    Xg = Xb[:, idx]
    ev = np.max(np.abs(Xg[0] - Xo[0])) / np.max(np.abs(Xo[0]))
    scale = np.maximum(np.max(np.abs(Xo), axis=1), mdl.newton_scale)
    serr = np.max(np.abs(Xg - Xo), axis=1) / scale
    say("  V %.2e, worst state %.2e" % (ev, serr.max()))
    if precision == "fp64":
        assert ev <= 1e-10 and np.all(serr <= 1e-9), serr
    else:
        n64 = len(mdl.fp64_states)
        assert ev <= 1e-4 and np.all(serr[:n64] <= 1e-4) and np.all(serr <= 1e-3), serr
