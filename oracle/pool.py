"""The oracle's stepper run over disjoint vertex subsets in worker processes
(test infrastructure: the CPU baseline of the benchmark).  Vertices are
independent in the reaction stage, so each worker advances its own columns
with oracle.sdc.advance unchanged, one numpy thread per process."""
from __future__ import annotations

import multiprocessing as mp
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _worker(args):
    model_name, x0, stim, diff, kw = args
    from threadpoolctl import threadpool_limits

    from .models import BY_NAME
    from .sdc import advance
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        X, _ = advance(BY_NAME[model_name], x0, i_stim=stim, i_diff=diff, **kw)
        return X, time.perf_counter() - t0


def advance_parallel(model_name, x0, i_stim, i_diff, workers, **kw):
    """advance() of every column of x0 (n, N), split into `workers` contiguous
    parts run in spawned processes.  Returns (X (n, N), per-worker seconds,
    wall seconds)."""
    parts = np.array_split(np.arange(x0.shape[1]), workers)
    jobs = [(model_name, np.ascontiguousarray(x0[:, p]),
             None if i_stim is None else i_stim[p], None if i_diff is None else i_diff[p], kw)
            for p in parts]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_worker, jobs))
    wall = time.perf_counter() - t0
    return np.concatenate([r[0] for r in res], axis=1), [r[1] for r in res], wall
