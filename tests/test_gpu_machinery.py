"""Device SDC machinery against textbook results, batching, resume and the
statistics, through the C ABI.

* TEST_LINEAR: predictor alone = backward-Euler product, many sweeps = the
  (M-1, M-1) Pade approximant (Lobatto IIIA collocation);
* TEST_LOGISTIC: observed order under dt-halving against the closed form;
* continuous batching: a handle advanced inside a batch, in chunks, equals the
  same handle advanced alone in one call, bit for bit;
* resume: n steps = n/2 steps, readback, re-init, n/2 steps, bit for bit;
* Newton bookkeeping: tol = 0 counts every solve as non-converged, a NaN
  input is counted as non-finite.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_tensor, run_gpu, say
from oracle.models import TEST_LINEAR
from oracle.sdc import advance
from paper_2510_27447_amd import ionic as I
from paper_2510_27447_amd.workloads import Workload, initial_state

pytestmark = pytest.mark.gpu

PADE = {
    2: ([1, 1 / 2], [1, -1 / 2]),
    3: ([1, 1 / 2, 1 / 12], [1, -1 / 2, 1 / 12]),
    4: ([1, 1 / 2, 1 / 10, 1 / 120], [1, -1 / 2, 1 / 10, -1 / 120]),
    5: ([1, 1 / 2, 3 / 28, 1 / 84, 1 / 1680], [1, -1 / 2, 3 / 28, -1 / 84, 1 / 1680]),
}


def pade(M, z):
    num, den = PADE[M]
    return sum(a * z ** k for k, a in enumerate(num)) / sum(b * z ** k for k, b in enumerate(den))


def lobatto_nodes(M):
    s5, s21 = np.sqrt(5.0), np.sqrt(21.0)
    return {2: [0, 1], 3: [0, .5, 1], 4: [0, (5 - s5) / 10, (5 + s5) / 10, 1],
            5: [0, (7 - s21) / 14, .5, (7 + s21) / 14, 1]}[M]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("M", [2, 3, 4, 5])
def test_linear_problem_limits(M, precision):
    dt = 0.25
    for z in (-0.5, -1.5):
        lam = z / dt
        y0 = np.linspace(0.5, 2.0, 100)[None, :]
        sim = I.Simulation("TEST_LINEAR", y0, precision=precision, newton_tol=1e-14,
                           params=[lam, 0.0])
        sim.step(0.0, dt, 1, M, 0)
        be = np.prod([1.0 / (1.0 - d * dt * lam) for d in np.diff(lobatto_nodes(M))])
        got = sim.readback()[0] / y0[0]
        tol = 1e-14 if precision == "fp64" else 1e-6
        np.testing.assert_allclose(got, be, rtol=tol)
        sim.close()
        sim = I.Simulation("TEST_LINEAR", y0, precision=precision, newton_tol=1e-14,
                           params=[lam, 0.0])
        sim.step(0.0, dt, 1, M, 16)
        got = sim.readback()[0] / y0[0]
        # 16 sweeps (the largest count the library accepts) against the oracle's
        # 16 sweeps, and against the collocation limit where 16 sweeps converge
        ref, _ = advance(TEST_LINEAR.with_params(lam=lam, b=0.0), np.array([[1.0]]), dt=dt,
                         n_steps=1, n_nodes=M, n_sweeps=16, tol=1e-15)
        np.testing.assert_allclose(got, ref[0, 0], rtol=1e-13 if precision == "fp64" else 1e-6)
        if z == -0.5:
            np.testing.assert_allclose(got, pade(M, z), rtol=1e-12 if precision == "fp64" else 1e-6)
        sim.close()


@pytest.mark.parametrize("M,K,p", [(2, 1, 2), (3, 2, 3), (3, 3, 4), (4, 3, 4)])
def test_logistic_order(M, K, p):
    rate, y0, T = 3.0, 0.05, 2.0
    exact = y0 * np.exp(rate * T) / (1 - y0 + y0 * np.exp(rate * T))
    errs = []
    for dt in (0.1, 0.05, 0.025):
        sim = I.Simulation("TEST_LOGISTIC", np.full((1, 64), y0), newton_tol=1e-15, params=[rate])
        sim.step(0.0, dt, int(round(T / dt)), M, K)
        errs.append(abs(sim.readback()[0, 0] - exact))
        sim.close()
    order = np.log2(errs[-2] / errs[-1])
    say("order", M, K, order)
    assert order > p - 0.2


def _tissue(model, N, seed, precision):
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.tile(initial_state(model)[:, None], (1, N))
    x0[0] += rng.uniform(-1, 1, N)
    stim = np.zeros(N)
    stim[: N // 8] = -80.0 if model == "LR91" else -100.0
    diff = rng.normal(0, 0.5, N)
    return x0, stim, diff


@pytest.mark.parametrize("model", ["LR91", "TT06"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_alone_bitwise(model, precision):
    import torch
    sizes = [300, 64, 1000]
    steps = [40, 25, 33]
    alone, batched = [], []
    inputs = [_tissue(model, n, 10 + k, precision) for k, n in enumerate(sizes)]
    for (x0, stim, diff), ns in zip(inputs, steps):
        s = I.Simulation(model, x0, precision=precision)
        st, df = gpu_tensor(stim), gpu_tensor(diff)
        s.step(0.0, 0.02, ns, 3, 2, st, 0.0, 0.3, df)
        alone.append(s.readback())
        s.close()
    sims, keep = [], []
    for (x0, stim, diff) in inputs:
        s = I.Simulation(model, x0, precision=precision)
        st, df = gpu_tensor(stim), gpu_tensor(diff)
        keep += [st, df]
        I.ionic_set_inputs(s.handle, 0.0, 0.02, 3, 2, st, 0.0, 0.3, df)
        sims.append(s)
    # two chunks of unequal length, as the serving loop would issue them
    first = [min(10, n) for n in steps]
    I.reaction_sdc_step_batch([s.handle for s in sims], first)
    I.reaction_sdc_step_batch([s.handle for s in sims], [n - f for n, f in zip(steps, first)])
    torch.cuda.synchronize()
    for k, s in enumerate(sims):
        out = s.readback()
        assert np.array_equal(out, alone[k]), k
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_is_bitwise(precision):
    x0, stim, diff = _tissue("TT06", 200, 3, precision)
    st, df = gpu_tensor(stim), gpu_tensor(diff)
    a = I.Simulation("TT06", x0, precision=precision)
    a.step(0.0, 0.02, 100, 3, 3, st, 0.0, 1.0, df)
    full = a.readback()
    b = I.Simulation("TT06", x0, precision=precision)
    b.step(0.0, 0.02, 50, 3, 3, st, 0.0, 1.0, df)
    mid = b.readback()
    c = I.Simulation("TT06", mid, precision=precision)
    c.step(50 * 0.02, 0.02, 50, 3, 3, st, 0.0, 1.0, df)
    assert np.array_equal(c.readback(), full)


def test_newton_bookkeeping():
    x0, stim, diff = _tissue("LR91", 100, 5, "fp64")
    s = I.Simulation("LR91", x0, newton_tol=0.0, newton_maxit=3)
    s.step(0.0, 0.02, 4, 3, 1)
    st = s.stats()
    assert st["n_nonconverged"] == 100 * 4 * 2
    assert st["newton_it_max"] == 3
    assert st["newton_iters"] == 100 * 4 * 2 * 3
    d = np.zeros(100)
    d[7] = np.nan
    s2 = I.Simulation("LR91", x0)
    s2.step(0.0, 0.02, 2, 2, 1, i_diff=gpu_tensor(d))
    assert s2.stats()["n_nonfinite"] == 1


def test_steady_gates_match_oracle():
    from oracle import tt06 as ot
    V = np.linspace(-90, 40, 130)
    x0 = np.tile(initial_state("TT06")[:, None], (1, 130))
    x0[0] = V
    s = I.Simulation("TT06", x0)
    I.ionic_gates_to_steady_state(s.handle)
    X = s.readback()
    ss = ot.gate_steady_state(V, x0[3])
    for k, v in ss.items():
        np.testing.assert_allclose(X[ot.STATE_NAMES.index(k)], v, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("model", ["LR91", "TT06"])
def test_init_without_x0_loads_rest_state(model, precision):
    """ionic_init(x0 = NULL): LR91 at the oracle's resting state X* (F(X*) = 0, the
    GPU's own Newton solve), TT06 at the published initial conditions; every
    vertex (a ragged 130) holds it, in the precision layout."""
    from oracle import rest as orest
    from oracle import tt06 as ot
    ref = orest.lr91_rest() if model == "LR91" else ot.published_initial()
    s = I.Simulation(model, None, precision=precision, n_vertices=130)
    X = s.readback()
    s.close()
    assert X.shape == (len(ref), 130)
    n64 = 2 if model == "LR91" else 6
    for i, r in enumerate(ref):
        tol = 1e-12 if (precision == "fp64" or i < n64) else 6e-8  # fp32 gates: one rounding
        np.testing.assert_allclose(X[i], r, rtol=tol, atol=1e-300, err_msg=str(i))
    if model == "TT06" and precision == "fp64":
        assert np.array_equal(X, np.tile(np.asarray(ref)[:, None], (1, 130)))


def test_init_from_device_x0_equals_host_x0():
    """The asynchronous device-x0 path loads exactly what the host path loads."""
    import torch
    x0, _, _ = _tissue("TT06", 150, 9, "mixed")
    for precision in ("fp64", "mixed"):
        a = I.Simulation("TT06", x0, precision=precision)
        b = I.Simulation("TT06", torch.as_tensor(x0).cuda(), precision=precision)
        assert np.array_equal(a.readback(), b.readback())
        a.close()
        b.close()
