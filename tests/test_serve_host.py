"""Admission policy of the serving loop, on the CPU: FIFO order, the slot
limit, the HBM byte budget, and rejection of a request larger than the whole
budget; plus the request trace's shape."""
from collections import deque

import numpy as np

from paper_2510_27447_amd.serve import Admission
from paper_2510_27447_amd.workloads import c5_trace


def test_fifo_slots_and_budget():
    pol = Admission(budget_bytes=100, slots=3)
    waiting = deque([("a", 40), ("b", 40), ("c", 30), ("d", 10)])
    adm, rej = pol.take(waiting, lambda r: r[1])
    assert [r[0] for r in adm] == ["a", "b"]          # c does not fit: head-of-line blocks d
    assert pol.resident == 80 and pol.active == 2
    pol.release(40)
    adm, _ = pol.take(waiting, lambda r: r[1])
    assert [r[0] for r in adm] == ["c", "d"]
    assert pol.active == 3
    waiting = deque([("e", 1)])
    adm, _ = pol.take(waiting, lambda r: r[1])
    assert adm == [] and len(waiting) == 1              # slots exhausted


def test_oversized_request_is_rejected():
    pol = Admission(budget_bytes=100, slots=8)
    waiting = deque([("huge", 101), ("ok", 50)])
    adm, rej = pol.take(waiting, lambda r: r[1])
    assert [r[0] for r in rej] == ["huge"]
    assert [r[0] for r in adm] == ["ok"]


def test_trace_shape():
    tr = c5_trace()
    assert len(tr) == 256
    gaps = np.diff([r.arrival for r in tr])
    assert 0.035 < gaps.mean() < 0.065                  # Poisson at 20/s
    ns = np.array([r.n for r in tr])
    assert ns.min() >= 1000 and ns.max() <= 2_000_000
    assert 0.35 < np.mean([r.model == "LR91" for r in tr]) < 0.65
    assert 0.35 < np.mean([r.precision == "fp64" for r in tr]) < 0.65
    assert set(r.dt for r in tr) == {0.01, 0.02}
    assert all(100 <= r.n_steps <= 1000 for r in tr)
    # every request fits a 200 GB budget by far
    assert sum(r.footprint_bytes() for r in tr) < 200e9
    w = tr[3].materialize()
    assert w.x0.shape[1] == tr[3].n and np.count_nonzero(w.i_stim) == max(1, tr[3].n // 10)


def test_chunk_sizes():
    from paper_2510_27447_amd.serve import chunk_for
    # large jobs take the plain chunk, small ones the same vertex-steps, capped by what is left
    assert chunk_for(2_000_000, 1000, 100, 200_000) == 100
    assert chunk_for(200_000, 1000, 100, 200_000) == 100
    assert chunk_for(100_000, 1000, 100, 200_000) == 200
    assert chunk_for(1_000, 1000, 100, 200_000) == 1000
    assert chunk_for(1_000, 37, 100, 200_000) == 37
    assert chunk_for(5_000, 0, 100, 200_000) == 0
    # without a quantum every job takes the plain chunk
    assert chunk_for(1_000, 1000, 100, 0) == 100
