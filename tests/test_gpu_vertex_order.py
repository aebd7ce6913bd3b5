"""A processing order of the vertices (ionic_set_vertex_order) changes only
which vertices share a wavefront (the mixed kernels take it; the fp64 ones
keep the identity mapping): every state must come out bit for bit as in the
identity order, for fp64 and mixed, every predictor, a ragged tail, a
blocked order of a structured grid and a random permutation, in a launch of
the one-wavefront build and in one of the two-wavefront build; the batched and
adaptive entries take the order too; a non-permutation is rejected."""
import numpy as np
import pytest

from gpu_helpers import gpu_tensor, say
from paper_2510_27447_amd.workloads import blocked_order, initial_state

pytestmark = pytest.mark.gpu


def inputs(model, n, seed=41):
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.tile(initial_state(model)[:, None], (1, n))
    x0[0] += rng.uniform(-3.0, 3.0, n)
    stim = np.where(rng.random(n) < 0.2, -80.0 if model == "LR91" else -100.0, 0.0)
    diff = rng.normal(0.0, 0.5, n)
    return x0, stim, diff


def run(model, precision, pred, M, K, x0, stim, diff, order=None, dt=0.02, n_steps=12):
    import torch
    from paper_2510_27447_amd import ionic as I
    sim = I.Simulation(model, x0, precision=precision)
    sim.set_predictor(pred)
    if order is not None:
        sim.set_vertex_order(order)
    sim.step(0.0, dt, n_steps, M, K, gpu_tensor(stim), 0.0, 0.3, gpu_tensor(diff))
    torch.cuda.synchronize()
    X = sim.readback()
    st = sim.stats()
    sim.close()
    return X, st


@pytest.mark.parametrize("model,precision,M,pred", [
    ("TT06", "mixed", 3, "newton"), ("TT06", "fp64", 3, "newton"), ("TT06", "mixed", 3, "rush_larsen"),
    ("TT06", "mixed", 2, "ros2"), ("LR91", "fp64", 3, "newton"), ("LR91", "mixed", 2, "ros2"),
    # kernels that keep the predictor's rows at node 1 in LDS for the first sweep
    ("TT06", "mixed", 4, "newton"), ("LR91", "mixed", 3, "newton")])
@pytest.mark.parametrize("shape", [(13, 11, 9), (64, 64, 33)], ids=["small", "two_wave"])
def test_order_changes_nothing(model, precision, M, pred, shape):
    n = int(np.prod(shape))
    x0, stim, diff = inputs(model, n)
    K = M - 1
    ref, st0 = run(model, precision, pred, M, K, x0, stim, diff)
    blocked = blocked_order(*shape)
    assert np.array_equal(np.sort(blocked), np.arange(n))
    rand = np.random.Generator(np.random.PCG64(5)).permutation(n).astype(np.int32)
    for name, order in (("blocked", blocked), ("random", rand)):
        X, st = run(model, precision, pred, M, K, x0, stim, diff, order)
        say(model, precision, M, pred, shape, name, "equal:", np.array_equal(X, ref))
        assert np.array_equal(X, ref)
        assert st["vertex_steps"] == st0["vertex_steps"]
        assert st["newton_iters"] == st0["newton_iters"]


def test_batched_and_adaptive_entries_take_the_order():
    import torch
    from paper_2510_27447_amd import ionic as I
    shape = (20, 17, 5)
    n = int(np.prod(shape))
    x0, stim, diff = inputs("TT06", n)
    order = blocked_order(*shape)
    outs = []
    for use in (False, True):
        sims = [I.Simulation("TT06", x0, precision="mixed") for _ in range(2)]
        s_t, d_t = gpu_tensor(stim), gpu_tensor(diff)
        for s in sims:
            if use:
                s.set_vertex_order(order)
            I.ionic_set_inputs(s.handle, 0.0, 0.02, 3, 2, s_t, 0.0, 0.3, d_t)
        I.reaction_sdc_step_batch([s.handle for s in sims], [7, 9])
        torch.cuda.synchronize()
        outs.append([s.readback() for s in sims])
        for s in sims:
            s.close()
    assert all(np.array_equal(a, b) for a, b in zip(outs[0], outs[1]))
    res = []
    for use in (False, True):
        sim = I.Simulation("TT06", x0, precision="fp64")
        if use:
            sim.set_vertex_order(order)
        r = sim.adaptive(0.0, 0.5, 0.01, 0.05, 1e-3, i_stim=gpu_tensor(stim), stim_t_on=0.0,
                         stim_t_off=0.3, i_diff=gpu_tensor(diff))
        res.append((r, sim.readback()))
        sim.close()
    assert res[0][0]["accepted"] == res[1][0]["accepted"]
    assert np.array_equal(res[0][1], res[1][1])


def test_non_permutations_are_rejected():
    import torch
    from paper_2510_27447_amd import ionic as I
    n = 100
    x0, _, _ = inputs("LR91", n)
    sim = I.Simulation("LR91", x0, precision="fp64")
    bad = [np.r_[np.arange(n - 1), 0], np.r_[np.arange(n - 1), n], np.r_[np.arange(n - 1), -1]]
    for b in bad:
        with pytest.raises(I.IonicError):
            sim.set_vertex_order(b.astype(np.int32))
    with pytest.raises(I.IonicError):
        sim.set_vertex_order(np.arange(n - 1, dtype=np.int32))
    sim.set_vertex_order(None)
    sim.close()
