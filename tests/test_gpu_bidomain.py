"""GPU vs oracle for the elliptic equation of the partitioned step (paper
section 3.1, equation semi-elliptic; Algorithm 2, first box) and for
partitioned bidomain stepping (one pass of Algorithm 2 per step), through
the C ABI, on structured grids with diagonal conductivity tensors.

Grids of at most 512 nodes use the Jacobi preconditioner, larger ones the
multigrid cycle.  Bars: u against the oracle's direct solve to 1e-9 of its scale at a CG
tolerance of 1e-13 (random fields); coupled runs at a CG tolerance of 1e-11; the solve reproducible bit for bit; coupled runs as the
other parity tests (fp64 1e-10 on V, mixed 1e-4 against the fp64 oracle);
sigma_e = sigma_i equal to monodomain stepping."""
import numpy as np
import pytest

from gpu_helpers import MODEL_OF, gpu_tensor, rel_errors, say
from oracle.diffusion import Bidomain, advance_bidomain
from paper_2510_27447_amd.workloads import initial_state

pytestmark = pytest.mark.gpu

SI = (1.5e-3, 0.5e-3, 1.0e-3)
SE = (1.0e-3, 2.0e-3, 0.7e-3)


def _buffers(shape, max_iter):
    import torch
    from paper_2510_27447_amd import ionic as I
    n = int(np.prod(shape))
    wb = I.ionic_elliptic_work_bytes(*shape, max_iter)
    return (torch.zeros(n, dtype=torch.float64, device="cuda"),
            torch.zeros(wb, dtype=torch.uint8, device="cuda"), wb,
            torch.zeros(n, dtype=torch.float64, device="cuda"))


# (9, 8, 5) ... (70, 3, 2): at most 512 nodes, Jacobi-preconditioned; (24, 20, 3)
# and (30, 24, 10): multigrid with 2 and 3 levels; (5000, 1, 1) and (60, 50, 1):
# multigrid on a cable (5 levels) and a sheet (3 levels), directions with one node
@pytest.mark.parametrize("shape", [(9, 8, 5), (13, 11, 1), (40, 1, 1), (70, 3, 2), (24, 20, 3),
                                   (30, 24, 10), (5000, 1, 1), (60, 50, 1)])
def test_elliptic_solve_matches_direct_solve(shape):
    from paper_2510_27447_amd import ionic as I
    n = int(np.prod(shape))
    h = 0.02
    rng = np.random.Generator(np.random.PCG64(8))
    x0 = np.tile(initial_state("TT06")[:, None], (1, n))
    x0[0] = rng.uniform(-85.0, 30.0, n)
    sim = I.Simulation("TT06", x0, precision="mixed")
    u, work, wb, _ = _buffers(shape, 4000)
    g = I.make_bidomain_grid(*shape, h=h, sigma_i=SI, sigma_e=SE)
    info = I.ionic_elliptic_solve(sim.handle, g, u, work, wb, rtol=1e-13, max_iter=4000)
    ug = u.cpu().numpy()
    # the same solve again from the same guess: the same bits
    u.zero_()
    I.ionic_elliptic_solve(sim.handle, g, u, work, wb, rtol=1e-13, max_iter=4000)
    assert np.array_equal(u.cpu().numpy(), ug)
    # warm start from the solution: no iteration needed
    info2 = I.ionic_elliptic_solve(sim.handle, g, u, work, wb, rtol=1e-9, max_iter=4000)
    sim.close()
    uo = Bidomain(shape, h, SI, SE).elliptic(x0[0])
    say("grid", shape, info, "max |du|/max|u|", np.max(np.abs(ug - uo)) / np.max(np.abs(uo)))
    assert info["converged"] == 1 and info["relative_residual"] <= 1e-13
    assert np.max(np.abs(ug - uo)) <= 1e-9 * np.max(np.abs(uo))
    assert info2["cg_iterations"] == 0


def test_iteration_count_and_reported_residual():
    """The solve stops at the first iteration that meets rtol, reports the
    residual it stopped on (checked against b - A_ie u from the oracle's
    matrices), and with one iteration fewer allowed it ends unconverged."""
    from paper_2510_27447_amd import ionic as I
    shape, h, rtol = (20, 15, 6), 0.02, 1e-6
    n = int(np.prod(shape))
    rng = np.random.Generator(np.random.PCG64(12))
    x0 = np.tile(initial_state("TT06")[:, None], (1, n))
    x0[0] = rng.uniform(-85.0, 30.0, n)
    sim = I.Simulation("TT06", x0, precision="fp64")
    u, work, wb, _ = _buffers(shape, 400)
    g = I.make_bidomain_grid(*shape, h=h, sigma_i=SI, sigma_e=SE)
    info = I.ionic_elliptic_solve(sim.handle, g, u, work, wb, rtol=rtol, max_iter=400)
    k = info["cg_iterations"]
    B = Bidomain(shape, h, SI, SE)
    b = -(B.Ai @ x0[0])
    true_rel = np.linalg.norm(b - B.Aie @ u.cpu().numpy()) / np.linalg.norm(b)
    say("iterations", k, "reported", info["relative_residual"], "true", true_rel)
    assert info["converged"] == 1 and 1 < k < 400
    assert info["relative_residual"] <= rtol
    assert abs(true_rel - info["relative_residual"]) <= 1e-4 * true_rel
    u.zero_()
    short = I.ionic_elliptic_solve(sim.handle, g, u, work, wb, rtol=rtol, max_iter=k - 1)
    sim.close()
    assert short["converged"] == 0 and short["cg_iterations"] == k - 1
    assert short["relative_residual"] > rtol


@pytest.mark.parametrize("model,shape", [("LR91", (16, 12, 1)), ("TT06", (8, 7, 6)),
                                         ("LR91", (24, 20, 3))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bidomain_stepping_matches_oracle(model, shape, precision):
    import torch
    from paper_2510_27447_amd import ionic as I
    say("case bidomain", model, shape, precision)
    n = int(np.prod(shape))
    x0 = np.tile(initial_state(model)[:, None], (1, n))
    stim = np.where(np.arange(n) % shape[0] < 2, -100.0, 0.0)
    h, dt, n_steps, M, K = 0.01, 0.02, 40, 3, 2
    sim = I.Simulation(model, x0, precision=precision)
    u, work, wb, idiff = _buffers(shape, 4000)
    g = I.make_bidomain_grid(*shape, h=h, sigma_i=SI, sigma_e=SE)
    info = I.reaction_bidomain_step(sim.handle, g, 0.0, dt, n_steps, M, K, u, work, wb, idiff,
                                    gpu_tensor(stim), 0.0, 1.0, rtol=1e-11, max_iter=4000)
    torch.cuda.synchronize()
    Xg, ug = sim.readback(), u.cpu().numpy()
    sim.close()
    Xo, uo, _ = advance_bidomain(MODEL_OF[model], x0, Bidomain(shape, h, SI, SE), dt=dt,
                                 n_steps=n_steps, n_nodes=M, n_sweeps=K, i_stim=stim, stim_on=0.0,
                                 stim_off=1.0)
    err = rel_errors(Xg, Xo, list(range(Xo.shape[0])))
    say("  V max/rms", err[0], "cg", info, "V range", Xo[0].min(), Xo[0].max())
    assert info["converged"] == 1
    assert Xo[0].max() > -40.0
    if precision == "fp64":
        assert err[0][0] <= 1e-10
        assert np.max(np.abs(ug - uo)) <= 1e-8 * np.max(np.abs(uo))
    else:
        n64 = 2 if model == "LR91" else 6
        for i in range(n64):
            assert err[i][0] <= 1e-4, i


def test_equal_ratios_equal_monodomain_stepping():
    import torch
    from paper_2510_27447_amd import ionic as I
    shape = (14, 10, 1)
    n = int(np.prod(shape))
    x0 = np.tile(initial_state("LR91")[:, None], (1, n))
    stim = gpu_tensor(np.where(np.arange(n) % shape[0] < 2, -100.0, 0.0))
    a = I.Simulation("LR91", x0)
    u, work, wb, idiff = _buffers(shape, 4000)
    I.reaction_bidomain_step(a.handle, I.make_bidomain_grid(*shape, h=0.01), 0.0, 0.02, 30, 3, 2,
                             u, work, wb, idiff, stim, 0.0, 1.0, rtol=1e-11, max_iter=4000)
    b = I.Simulation("LR91", x0)
    I.reaction_diffusion_step(b.handle, I.make_grid(*shape, h=0.01, sigma=0.75e-3), 0.0, 0.02, 30,
                              3, 2, idiff, stim, 0.0, 1.0)
    torch.cuda.synchronize()
    Xa, Xb = a.readback(), b.readback()
    a.close()
    b.close()
    assert np.max(np.abs(Xa[0] - Xb[0])) <= 1e-10 * np.max(np.abs(Xb[0]))


def test_bidomain_rejections():
    import torch
    from paper_2510_27447_amd import ionic as I
    shape = (6, 4, 1)
    x0 = np.tile(initial_state("LR91")[:, None], (1, 24))
    sim = I.Simulation("LR91", x0)
    u, work, wb, idiff = _buffers(shape, 50)
    g = I.make_bidomain_grid(*shape, h=0.005, sigma_i=(1.5e-3,) * 3, sigma_e=(1.5e-3,) * 3)
    with pytest.raises(I.IonicError, match="unstable"):
        I.reaction_bidomain_step(sim.handle, g, 0.0, 0.02, 1, 3, 2, u, work, wb, idiff)
    with pytest.raises(I.IonicError, match="work buffer too small"):
        I.ionic_elliptic_solve(sim.handle, g, u, work, wb, max_iter=5000)
    torch.cuda.synchronize()
    sim.close()
