"""GPU vs oracle on small inputs: every model x precision x node count, a
vertex count spanning several workgroups with a ragged tail, states spread
over the physiological range (some vertices stimulated, some with a diffusion
current), and the degenerate cases of the method (no sweeps, one node pair).

Bar (the stated targets of the build): fp64 path max|dV| / max|V_ref| <= 1e-10
(other states <= 1e-9 of their own scale); mixed path <= 1e-4 on V and the
fp64-held concentrations, measured against the fp64 oracle."""
import numpy as np
import pytest

from gpu_helpers import rel_errors, run_gpu, run_oracle, say
from paper_2510_27447_amd.workloads import Workload, initial_state

pytestmark = pytest.mark.gpu

N_SMALL = 130  # two full wavefronts and a tail of 2


def small_workload(model, precision, M, K, n_steps=25, seed=1, N=N_SMALL):
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.tile(initial_state(model)[:, None], (1, N))
    x0[0] += rng.uniform(-3.0, 3.0, N)
    stim = np.where(rng.random(N) < 0.3, -80.0 if model == "LR91" else -100.0, 0.0)
    diff = rng.normal(0.0, 0.5, N)
    return Workload("small-%s-%s-M%dK%d" % (model, precision, M, K), model, precision, x0, 0.02,
                    n_steps, M, K, 1e-10, 10, stim, 0.0, 0.5, diff, seed=seed)


@pytest.mark.parametrize("model", ["LR91", "TT06"])
@pytest.mark.parametrize("M,K", [(2, 1), (3, 2), (3, 3), (4, 3), (5, 2), (3, 0)])
def test_fp64_matches_oracle(model, M, K):
    w = small_workload(model, "fp64", M, K)
    say("case", w.name)
    Xg, st = run_gpu(w)
    Xo = run_oracle(w)
    names = list(range(w.x0.shape[0]))
    err = rel_errors(Xg, Xo, names)
    say("  V max/rms", err[0], "worst state", max(err.items(), key=lambda kv: kv[1][0]))
    assert err[0][0] <= 1e-10
    assert max(e[0] for e in err.values()) <= 1e-9
    assert st["n_nonfinite"] == 0
    assert st["vertex_steps"] == w.n * w.n_steps
    assert st["newton_solves"] == w.n * w.n_steps * (M - 1)


# (3, 1), (4, 1), (5, 2), (4, 0): the kernels that take the predictor's F and
# J at node 1 into the first sweep (LR91 with 3 nodes, TT06 with 4 and 5),
# with one sweep only, with later sweeps, and with none
@pytest.mark.parametrize("model", ["LR91", "TT06"])
@pytest.mark.parametrize("M,K", [(2, 1), (3, 2), (3, 3), (4, 3), (3, 1), (4, 1), (5, 2), (4, 0)])
def test_mixed_matches_fp64_oracle(model, M, K):
    w = small_workload(model, "mixed", M, K)
    say("case", w.name)
    Xg, st = run_gpu(w)
    Xo = run_oracle(w)
    n64 = 2 if model == "LR91" else 6
    err = rel_errors(Xg, Xo, list(range(w.x0.shape[0])))
    say("  V max/rms", err[0], "fp64-held", [err[i] for i in range(n64)])
    for i in range(n64):
        assert err[i][0] <= 1e-4, i
    assert max(e[0] for e in err.values()) <= 1e-3
    assert st["n_nonfinite"] == 0


@pytest.mark.parametrize("model", ["LR91", "TT06"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_jacobian_matches_oracle(model, precision):
    from gpu_helpers import MODEL_OF
    from paper_2510_27447_amd import ionic as I
    w = small_workload(model, precision, 3, 2, N=70, seed=4)
    # spread V wider, including the h/j branch point and removable singularities
    w.x0[0, :8] = [-40.0, -47.13, -77.0, 15.0, -39.999, -85.0, 20.0, -60.0]
    sim = I.Simulation(model, w.x0, precision=precision)
    mdl = MODEL_OF[model]
    tol = 1e-12 if precision == "fp64" else 2e-4
    for v in range(0, 70, 3):
        Fg, Jg = sim.debug_jacobian(v, i_stim=-7.0, i_diff=0.25)
        Fo, Jo = mdl.FJ(w.x0[:, v:v + 1], np.array([-7.0]), np.array([0.25]))
        Fo, Jo = Fo[:, 0], Jo[0]
        # row-scaled comparison (entries J_ik * scale_k)
        s = np.maximum(np.abs(w.x0[:, v]), mdl.newton_scale)
        A, B = Jg * s[None, :], Jo * s[None, :]
        rs = np.max(np.abs(B), axis=1) + np.abs(Fo) + 1e-300
        assert np.max(np.abs(A - B) / rs[:, None]) <= tol, v
        assert np.max(np.abs(Fg - Fo) / rs) <= tol, v
        assert np.all((Jg != 0) <= (Jo != 0) | (np.abs(Jg) < 1e-300))
    sim.close()
