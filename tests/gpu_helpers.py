"""Shared helpers of the GPU tests: run a workload through the C-ABI library
and, separately, through the oracle; compare the two.  Inputs are built once
(paper_2510_27447_amd.workloads) and handed to both sides."""
from __future__ import annotations

import sys

import numpy as np

from oracle import models as omodels
from oracle import lr91 as olr91
from oracle import tt06 as ott06
from oracle.sdc import advance

MODEL_OF = {"LR91": omodels.LR91, "TT06": omodels.TT06,
            "TEST_LINEAR": omodels.TEST_LINEAR, "TEST_LOGISTIC": omodels.TEST_LOGISTIC}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_tensor(a):
    import torch
    if a is None:
        return None
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run_gpu(w, stream=None, return_sim=False):
    """Run workload w on the GPU through the library; returns (X (n, N), stats)."""
    import torch
    from paper_2510_27447_amd import ionic as I
    sim = I.Simulation(w.model, w.x0, precision=w.precision, newton_tol=w.newton_tol,
                       newton_maxit=w.newton_maxit)
    if w.steady_gates:
        I.ionic_gates_to_steady_state(sim.handle)
    stim = gpu_tensor(w.i_stim)
    if w.i_diff_series:
        diffs = [gpu_tensor(d) for d in w.i_diff_series]
        done = 0
        k = 0
        while done < w.n_steps:
            n = min(w.diff_period, w.n_steps - done)
            sim.step(done * w.dt, w.dt, n, w.n_nodes, w.n_sweeps, stim, w.stim_t_on, w.stim_t_off,
                     diffs[k])
            done += n
            k += 1
    else:
        sim.step(0.0, w.dt, w.n_steps, w.n_nodes, w.n_sweeps, stim, w.stim_t_on, w.stim_t_off,
                 gpu_tensor(w.i_diff))
    torch.cuda.synchronize()
    X = sim.readback()
    st = sim.stats()
    if return_sim:
        return X, st, sim
    sim.close()
    return X, st


def oracle_initial(w):
    """Initial state as the oracle sees it (gates to steady state with its own kinetics)."""
    X0 = w.x0.copy()
    if w.steady_gates:
        if w.model == "TT06":
            ss = ott06.gate_steady_state(X0[0], X0[3])
            for k, v in ss.items():
                X0[ott06.STATE_NAMES.index(k)] = v
        else:
            ss = olr91.gate_steady_state(X0[0])
            for k, v in ss.items():
                X0[olr91.STATE_NAMES.index(k)] = v
    return X0


def run_oracle(w):
    model = MODEL_OF[w.model]
    X = oracle_initial(w)
    if w.i_diff_series:
        done, k = 0, 0
        while done < w.n_steps:
            n = min(w.diff_period, w.n_steps - done)
            X, _ = advance(model, X, t0=done * w.dt, dt=w.dt, n_steps=n, n_nodes=w.n_nodes,
                           n_sweeps=w.n_sweeps, i_stim=w.i_stim, stim_on=w.stim_t_on,
                           stim_off=w.stim_t_off, i_diff=w.i_diff_series[k], tol=w.newton_tol,
                           maxit=w.newton_maxit)
            done += n
            k += 1
        return X
    X, _ = advance(model, X, t0=0.0, dt=w.dt, n_steps=w.n_steps, n_nodes=w.n_nodes,
                   n_sweeps=w.n_sweeps, i_stim=w.i_stim, stim_on=w.stim_t_on,
                   stim_off=w.stim_t_off, i_diff=w.i_diff, tol=w.newton_tol, maxit=w.newton_maxit)
    return X


def rel_errors(Xg, Xo, names):
    """Per state: max |diff| / max |ref| and RMS |diff| / max |ref|."""
    out = {}
    for i, nm in enumerate(names):
        scale = max(np.max(np.abs(Xo[i])), 1e-300)
        d = np.abs(Xg[i] - Xo[i])
        out[nm] = (float(np.max(d) / scale), float(np.sqrt(np.mean(d * d)) / scale))
    return out
