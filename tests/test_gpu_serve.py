"""Serving loop on the GPU: every request's result in the continuous-batching
mix (other requests of its class in the same launches, other classes on other
streams, chunked steps) equals the same request run alone, bit for bit, and a
seeded sample of every request's vertices matches the fp64 oracle (fp64
requests: V within 1e-10 of max|V|, every state within 1e-9 of its scale;
mixed requests: V and the fp64-held concentrations within 1e-4, gates within
1e-3).  The V the loop hands back is the V of that state."""
import numpy as np
import pytest

from gpu_helpers import MODEL_OF, gpu_tensor, run_oracle, say
from paper_2510_27447_amd import ionic as I
from paper_2510_27447_amd.serve import Server, summarize
from paper_2510_27447_amd.workloads import Request

pytestmark = pytest.mark.gpu


def small_trace():
    rng = np.random.Generator(np.random.PCG64(5))
    reqs = []
    t = 0.0
    for k in range(14):
        t += rng.exponential(0.01)
        reqs.append(Request(k, t, "LR91" if k % 2 else "TT06", "fp64" if k % 3 else "mixed",
                            int(rng.integers(100, 3000)), 0.01 if k % 4 else 0.02,
                            int(rng.integers(20, 90)), int(rng.integers(0, 2 ** 31))))
    return reqs


def test_results_in_the_mix_equal_results_alone():
    trace = small_trace()
    srv = Server(chunk_steps=16, quantum_vertices=1000, split_small=True, slots=6, keep_state=True)
    res = {r.rid: r for r in srv.run(trace)}
    say("serving summary", summarize(list(res.values())))
    assert len(res) == len(trace)
    rng = np.random.Generator(np.random.PCG64(17))
    for req in trace:
        w = req.materialize()
        sim = I.Simulation(w.model, w.x0, precision=w.precision)
        sim.step(0.0, w.dt, w.n_steps, w.n_nodes, w.n_sweeps, gpu_tensor(w.i_stim), w.stim_t_on,
                 w.stim_t_off, gpu_tensor(w.i_diff))
        alone = sim.readback()
        sim.close()
        got = res[req.rid]
        assert np.array_equal(got.state, alone), req.rid
        assert np.array_equal(got.V, got.state[0]), req.rid
        # a seeded vertex sample against the oracle: stimulated and unstimulated
        # vertices, the first and the last
        stim_idx = np.nonzero(w.i_stim)[0]
        idx = np.unique(np.concatenate([[0, w.n - 1], rng.choice(stim_idx, 2),
                                        rng.choice(w.n, 4, replace=False)]))
        Xo = run_oracle(w.subset(idx))
        mdl = MODEL_OF[w.model]
        n64 = len(mdl.fp64_states)
        Xs = got.state[:, idx]
        scale = np.maximum(np.max(np.abs(Xo), axis=1), mdl.newton_scale)
        serr = np.max(np.abs(Xs - Xo), axis=1) / scale
        ev = np.max(np.abs(Xs[0] - Xo[0])) / np.max(np.abs(Xo[0]))
        say("  req %d %s %s N=%d steps=%d: V %.2e, worst state %.2e" % (
            req.rid, w.model, w.precision, w.n, w.n_steps, ev, serr.max()))
        if w.precision == "fp64":
            assert ev <= 1e-10 and np.all(serr <= 1e-9), (req.rid, serr)
        else:
            assert ev <= 1e-4 and np.all(serr[:n64] <= 1e-4) and np.all(serr <= 1e-3), (
                req.rid, serr)
