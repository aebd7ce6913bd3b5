"""Adaptive time stepping of the reaction stage with the ROS2 predictor, fp64
(oracle; test infrastructure).

Paper, section 3.3.1: the second (embedded) ROS2 solution X_hat serves to
choose the next step size; section 4: the partitioned strategy runs with
adaptive time steps capped at 0.05 ms.  In the partitioned strategy the whole
tissue shares one step, so here one step size serves every vertex of the
call.  One attempt from t with step tau is a full sdc_step (ROS2 predictor on
every Gauss-Lobatto sub-interval, then K correction sweeps); the paper's own
scheme is M = 2, K = 1.

The paper prints no controller.  Readings:
* error of an attempt: err = max over vertices, sub-intervals and states of
  |X_i - X_hat_i| / max(|X_i|, scale_i)  (scale_i: the per-state floor of the
  Newton stop), the embedded estimate of the ROS2 predictor;
* the attempt is accepted iff err <= tol;
* next step: tau * min(Q_MAX, max(Q_MIN, SAFETY * (tol / err)^(1/2))), the
  exponent 1/(phat + 1) of the embedded order phat = 1; err == 0 gives Q_MAX;
  a non-finite err rejects the attempt with Q_MIN; the result is capped at
  dt_max;
* breakpoints: the stimulus switching times and t_end.  A step never crosses
  one: if the proposed step reaches the next breakpoint b > t, the step is
  b - t and on acceptance t becomes b exactly;
* the stimulus is constant over a step, on iff t_on <= t + tau/2 < t_off;
* at most max_attempts attempts; the run also stops (failed) when the step
  falls below dt_min.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lobatto import integration_matrix, nodes
from .sdc import Stats, sdc_step

SAFETY = 0.9
Q_MIN = 0.2
Q_MAX = 2.0


@dataclass
class AdaptStats:
    accepted: int = 0
    rejected: int = 0
    t: float = 0.0
    done: bool = False
    failed: bool = False
    # one row per attempt: (t at the start, step, err, accepted)
    history: list = field(default_factory=list)


def next_breakpoint(t, t_on, t_off, t_end):
    b = t_end
    for x in (t_on, t_off):
        if t < x < b:
            b = x
    return b


def step_factor(err, tol):
    if not np.isfinite(err):
        return Q_MIN
    if err == 0.0:
        return Q_MAX
    return min(Q_MAX, max(Q_MIN, SAFETY * np.sqrt(tol / err)))


def advance_adaptive(model, X0, *, t0=0.0, t_end, dt_init, dt_max=0.05, err_tol,
                     n_nodes=2, n_sweeps=1, i_stim=None, stim_on=0.0, stim_off=0.0,
                     i_diff=None, max_attempts=100000, dt_min=1e-12, clamp_v=False):
    """Advance X0 (n, N) from t0 to t_end; returns (X, AdaptStats)."""
    X = np.array(X0, dtype=np.float64, copy=True)
    n, N = X.shape
    if n != model.n:
        raise ValueError("state has %d rows, model %s has %d states" % (n, model.name, model.n))
    stim_amp = np.zeros(N) if i_stim is None else np.asarray(i_stim, dtype=np.float64)
    diff = np.zeros(N) if i_diff is None else np.asarray(i_diff, dtype=np.float64)
    c = nodes(n_nodes)
    S = integration_matrix(n_nodes)
    st = AdaptStats(t=float(t0))
    scratch = Stats(per_vertex_iters=np.zeros(N, dtype=np.int64))
    t = float(t0)
    dt_try = min(float(dt_init), float(dt_max))
    while t < t_end:
        if len(st.history) >= max_attempts:
            st.failed = True
            break
        b = next_breakpoint(t, stim_on, stim_off, t_end)
        hit = dt_try >= b - t
        tau = b - t if hit else dt_try
        if tau < dt_min:
            st.failed = True
            break
        t_mid = t + 0.5 * tau
        stim = stim_amp if (stim_on <= t_mid < stim_off) else np.zeros(N)
        Xn, err_v = sdc_step(model, X, stim, tau, n_nodes, n_sweeps, diff, 0.0, 1, clamp_v,
                             scratch, S, c, predictor="ros2")
        err = float(np.max(err_v)) if np.all(np.isfinite(err_v)) else float("inf")
        ok = err <= err_tol
        st.history.append((t, tau, err, ok))
        q = step_factor(err, err_tol)
        if ok:
            X = Xn
            t = b if hit else t + tau
            st.accepted += 1
        else:
            st.rejected += 1
        dt_try = min(float(dt_max), tau * q)
    st.t = t
    st.done = t >= t_end
    return X, st
