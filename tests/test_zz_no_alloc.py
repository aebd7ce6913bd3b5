"""state_readback_noalloc (the entry point for callers that cannot allocate)
against state_readback, through the C ABI: two calls in a row on one handle,
the second on a smaller vertex range, in both precision layouts; both must
return the same values bit for bit (the same widening kernel runs in both,
only the staging buffer differs).  A readback beyond the 8 MiB static buffer
is rejected before any GPU work."""
import numpy as np
import pytest

from gpu_helpers import gpu_tensor, say
from paper_2510_27447_amd import ionic as I
from paper_2510_27447_amd.workloads import initial_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("model", ["TT06", "LR91"])
def test_noalloc_readback_equals_readback(model, precision):
    import torch
    N = 70_000  # beyond the static buffer for TT06 whole, within it for a sub-range
    rng = np.random.Generator(np.random.PCG64(21))
    x0 = np.tile(initial_state(model)[:, None], (1, N))
    x0[0] += rng.uniform(-5.0, 5.0, N)
    stim = np.where(np.arange(N) < N // 10, -80.0, 0.0)
    sim = I.Simulation(model, x0, precision=precision)
    sim.step(0.0, 0.02, 20, 3, 2, gpu_tensor(stim), 0.0, 1.0, gpu_tensor(rng.normal(0, 0.5, N)))
    torch.cuda.synchronize()
    ns = sim.n_states
    cap = (8 << 20) // (8 * ns)
    first_count = min(N - 5, cap)          # largest range the buffer holds
    ranges = [(5, first_count), (1234, 777)]  # the second call smaller
    for first, count in ranges:
        say("case", model, precision, "first", first, "count", count)
        ref = I.state_readback(sim.handle, ns, first, count)
        got = I.state_readback_noalloc(sim.handle, ns, first, count)
        assert got.shape == (ns, count)
        assert np.array_equal(got, ref)
    if ns * N * 8 > (8 << 20):
        with pytest.raises(I.IonicError) as ei:
            I.state_readback_noalloc(sim.handle, ns, 0, N)
        assert ei.value.status == -1 and "static staging buffer" in str(ei.value)
    sim.close()
