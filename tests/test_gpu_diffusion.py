"""GPU vs oracle for the diffusion current on structured grids (paper section
3.1, Q1 elements with lumped mass) and for reaction-diffusion stepping (the
current of the V field at the start of each step held over one reaction
step), through the C ABI.

Bars: the current alone to 1e-12 of its scale (it is a short sum of fp64
products); coupled runs as the other parity tests (fp64 1e-10 on V, mixed
1e-4 against the fp64 oracle)."""
import numpy as np
import pytest

from gpu_helpers import MODEL_OF, gpu_tensor, rel_errors, say
from oracle.diffusion import Diffusion, advance_coupled
from paper_2510_27447_amd.workloads import initial_state

pytestmark = pytest.mark.gpu


# (70, 9, 13): wavefronts of 62 nodes spanning several x-rows and planes;
# (63, 1, 4100) and (1, 1, 8193): long grids along z, one node wide in y (and x)
@pytest.mark.parametrize("shape", [(17, 1, 1), (13, 9, 1), (7, 6, 5), (1, 1, 1), (2, 3, 2),
                                   (70, 9, 13), (63, 1, 4100), (1, 1, 8193)])
def test_diffusion_current_matches_oracle(shape):
    import torch
    from paper_2510_27447_amd import ionic as I
    n = int(np.prod(shape))
    rng = np.random.Generator(np.random.PCG64(3))
    x0 = np.tile(initial_state("TT06")[:, None], (1, n))
    x0[0] = rng.uniform(-85.0, 30.0, n)
    h, sigma = 0.01, 0.75e-3
    want = Diffusion(shape, h, sigma).current(x0[0])
    for prec in ("fp64", "mixed"):
        sim = I.Simulation("TT06", x0, precision=prec)
        out = torch.zeros(n, dtype=torch.float64, device="cuda")
        I.ionic_diffusion_current(sim.handle, I.make_grid(*shape, h=h, sigma=sigma), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        sim.close()
        scale = max(np.max(np.abs(want)), 1e-300)
        say("grid", shape, prec, "max rel", np.max(np.abs(got - want)) / scale)
        assert np.max(np.abs(got - want)) <= 1e-12 * scale + 1e-300


@pytest.mark.parametrize("model,shape", [("LR91", (20, 15, 1)), ("TT06", (8, 7, 6))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("predictor", ["newton", "rush_larsen"])
def test_reaction_diffusion_matches_oracle(model, shape, precision, predictor):
    import torch
    from paper_2510_27447_amd import ionic as I
    say("case reaction-diffusion", model, shape, precision, predictor)
    n = int(np.prod(shape))
    x0 = np.tile(initial_state(model)[:, None], (1, n))
    stim = np.zeros(n)
    stim[np.arange(n) % shape[0] < 2] = -100.0     # planar stimulus at x = 0, 1
    h, sigma, dt, n_steps, M, K = 0.01, 0.75e-3, 0.02, 60, 3, 2
    sim = I.Simulation(model, x0, precision=precision)
    sim.set_predictor(predictor)
    work = torch.zeros(n, dtype=torch.float64, device="cuda")
    I.reaction_diffusion_step(sim.handle, I.make_grid(*shape, h=h, sigma=sigma), 0.0, dt, n_steps,
                              M, K, work, gpu_tensor(stim), 0.0, 1.0)
    torch.cuda.synchronize()
    Xg = sim.readback()
    st = sim.stats()
    sim.close()
    Xo, _ = advance_coupled(MODEL_OF[model], x0, Diffusion(shape, h, sigma), dt=dt,
                            n_steps=n_steps, n_nodes=M, n_sweeps=K, i_stim=stim, stim_on=0.0,
                            stim_off=1.0, predictor=predictor)
    err = rel_errors(Xg, Xo, list(range(Xo.shape[0])))
    say("  V max/rms", err[0], "V range", Xo[0].min(), Xo[0].max())
    assert Xo[0].max() > -40.0        # the stimulated columns have depolarised
    if precision == "fp64":
        assert err[0][0] <= 1e-10
        assert max(e[0] for e in err.values()) <= 1e-9
    else:
        n64 = 2 if model == "LR91" else 6
        for i in range(n64):
            assert err[i][0] <= 1e-4, i
    assert st["vertex_steps"] == n * n_steps and st["n_nonfinite"] == 0


def test_unstable_step_and_bad_grid_are_rejected():
    import torch
    from paper_2510_27447_amd import ionic as I
    x0 = np.tile(initial_state("LR91")[:, None], (1, 24))
    sim = I.Simulation("LR91", x0)
    work = torch.zeros(24, dtype=torch.float64, device="cuda")
    g = I.make_grid(6, 4, 1, h=0.005, sigma=0.75e-3)       # limit h^2/(2 sigma) = 0.0167 ms
    with pytest.raises(I.IonicError, match="unstable"):
        I.reaction_diffusion_step(sim.handle, g, 0.0, 0.02, 1, 3, 2, work)
    I.reaction_diffusion_step(sim.handle, g, 0.0, 0.015, 2, 3, 2, work)
    with pytest.raises(I.IonicError, match="vertex count"):
        I.ionic_diffusion_current(sim.handle, I.make_grid(5, 4, 1), work)
    torch.cuda.synchronize()
    sim.close()
