"""Serving loop on the GPU: every request's result in the continuous-batching
mix (other requests of its class in the same launches, other classes on other
streams, chunked steps) equals the same request run alone, bit for bit."""
import numpy as np
import pytest

from gpu_helpers import gpu_tensor, say
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
    srv = Server(chunk_steps=16, slots=6, keep_state=True)
    res = {r.rid: r for r in srv.run(trace)}
    say("serving summary", summarize(list(res.values())))
    assert len(res) == len(trace)
    for req in trace:
        w = req.materialize()
        sim = I.Simulation(w.model, w.x0, precision=w.precision)
        sim.step(0.0, w.dt, w.n_steps, w.n_nodes, w.n_sweeps, gpu_tensor(w.i_stim), w.stim_t_on,
                 w.stim_t_off, gpu_tensor(w.i_diff))
        alone = sim.readback()
        sim.close()
        assert np.array_equal(res[req.rid].state, alone), req.rid
