"""Reaction stage with spectral deferred correction, fp64 (oracle; test infrastructure).

Paper, section 3.3.2.  With the extracellular potential (here: the fixed
per-vertex diffusion current I_diff) held over the step, the vertices
decouple and each one integrates dX/dt = F(X) (equation genODE, M~ = I after
nodal evaluation of the reaction terms).  One step from t_n to t_n + dt:

1. nodes c_0 = 0 < ... < c_{M-1} = 1 (Gauss-Lobatto), sub-steps
   dtau_m = (c_{m+1} - c_m) dt, quadrature S * dt (module lobatto);
2. predictor, X_0 = X_n and, on each sub-interval, either
   (a) backward Euler Y - X_m - dtau_m F(Y) = 0 solved by local Newton
       (I - dtau_m J(Y)) delta = -(Y - X_m - dtau_m F(Y)),  Y += delta,
       stopping once max_i |delta_i| / max(|Y_i|, scale_i) <= tol (at least
       one iteration, at most maxit, the last iterate kept): the first-order
       implicit integrator the paper's correction equation uses; or
   (b) one step of the Rosenbrock method ROS2 (equation rb_system, module
       ros2), the paper's own predictor, which also yields the scaled
       embedded error max_i |X_i - X_hat_i| / max(|X_i|, scale_i) used for
       step-size control; or
   (c) Rush-Larsen (module rush_larsen): exponential steps for the gating
       states at frozen X_m, then backward Euler by Newton on the core;
3. K sweeps of the linearised implicit correction (equations residual,
   sdc_ode, sdc generalised from the trapezoid to M nodes):
   F^k_j = F(X^k_j);  X^{k+1}_0 = X_n;  for m = 0..M-2
   r = X^{k+1}_m - X^k_{m+1} + sum_j S_mj F^k_j
   (I - dtau_m J(X^k_{m+1})) delta = r,  X^{k+1}_{m+1} = X^k_{m+1} + delta;
   with M = 2 and K = 1 this is equation sdc with M~ = I;
4. X_{n+1} = X^K_{M-1}.

The stimulus is constant over a step and applied iff
t_on <= t0 + (n + 1/2) dt < t_off.  Everything is vectorised over vertices;
every vertex follows its own Newton iteration count.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lobatto import integration_matrix, nodes
from .ros2 import ros2_step
from .rush_larsen import rush_larsen_be


@dataclass
class Stats:
    newton_iters_total: int = 0
    newton_solves: int = 0
    newton_it_max: int = 0
    n_nonconverged: int = 0
    n_nonfinite: int = 0
    per_vertex_iters: np.ndarray = field(default=None, repr=False)
    embedded_error: list = field(default_factory=list, repr=False)


def _solve(A, b):
    return np.linalg.solve(A, b[..., None])[..., 0]


def stimulus_on(t0, dt, n, t_on, t_off):
    t_mid = t0 + (n + 0.5) * dt
    return (t_on <= t_mid) and (t_mid < t_off)


def newton_be(model, Xm, dtau, i_stim, i_diff, tol, maxit, clamp_v, stats):
    """Backward Euler on one sub-interval by local Newton (per-vertex stop)."""
    n, N = Xm.shape
    Y = Xm.copy()
    it = np.zeros(N, dtype=np.int64)
    active = np.ones(N, dtype=bool)
    converged = np.zeros(N, dtype=bool)
    I = np.eye(n)
    scale = model.newton_scale[:, None]
    while active.any():
        idx = np.nonzero(active)[0]
        Ya = Y[:, idx]
        F, J = model.FJ(Ya, _pick(i_stim, idx), _pick(i_diff, idx), clamp_v)
        G = Ya - Xm[:, idx] - dtau * F
        delta = _solve(I[None] - dtau * J, -G.T).T
        Ynew = Ya + delta
        Y[:, idx] = Ynew
        it[idx] += 1
        err = np.max(np.abs(delta) / np.maximum(np.abs(Ynew), scale), axis=0)
        done = err <= tol
        converged[idx] = done
        active[idx] = ~(done | (it[idx] >= maxit))
    stats.newton_iters_total += int(it.sum())
    stats.newton_solves += N
    stats.newton_it_max = max(stats.newton_it_max, int(it.max(initial=0)))
    stats.n_nonconverged += int((~converged).sum())
    stats.per_vertex_iters += it
    return Y


def _pick(a, idx):
    if np.ndim(a) == 0:
        return a
    return a[idx]


def embedded_error(model, X, X_hat):
    """Scaled embedded error per vertex: max_i |X_i - X_hat_i| / max(|X_i|, scale_i)."""
    scale = model.newton_scale[:, None]
    return np.max(np.abs(X - X_hat) / np.maximum(np.abs(X), scale), axis=0)


PREDICTORS = ("newton", "ros2", "rush_larsen")


def sdc_step(model, Xn, i_stim, dt, M, K, i_diff, tol, maxit, clamp_v, stats, S, c,
             predictor="newton"):
    """One step; returns X_{n+1} and, for the ROS2 predictor, the embedded error
    per vertex (largest over the sub-intervals; None for Newton)."""
    n, N = Xn.shape
    I = np.eye(n)
    dtau = np.diff(c) * dt
    Sdt = S * dt
    # predictor
    Xk = [Xn]
    err = None
    if predictor == "newton":
        for m in range(M - 1):
            Xk.append(newton_be(model, Xk[m], dtau[m], i_stim, i_diff, tol, maxit, clamp_v, stats))
    elif predictor == "ros2":
        err = np.zeros(N)
        for m in range(M - 1):
            Xnew, Xhat, _ = ros2_step(model, Xk[m], dtau[m], i_stim, i_diff, clamp_v)
            err = np.maximum(err, embedded_error(model, Xnew, Xhat))
            Xk.append(Xnew)
    elif predictor == "rush_larsen":
        for m in range(M - 1):
            Xk.append(rush_larsen_be(model, Xk[m], dtau[m], i_stim, i_diff, tol, maxit, clamp_v,
                                     stats))
    else:
        raise ValueError("unknown predictor %r" % (predictor,))
    # corrections
    F0 = model.F(Xn, i_stim, i_diff, clamp_v)
    for _ in range(K):
        Fk = [F0] + [model.F(Xk[j], i_stim, i_diff, clamp_v) for j in range(1, M)]
        Xnew = [Xn]
        for m in range(M - 1):
            r = Xnew[m] - Xk[m + 1]
            for j in range(M):
                r = r + Sdt[m, j] * Fk[j]
            _, J = model.FJ(Xk[m + 1], i_stim, i_diff, clamp_v)
            delta = _solve(I[None] - dtau[m] * J, r.T).T
            Xnew.append(Xk[m + 1] + delta)
        Xk = Xnew
    return Xk[M - 1], err


def advance(model, X0, *, t0=0.0, dt, n_steps, n_nodes, n_sweeps,
            i_stim=None, stim_on=0.0, stim_off=0.0, i_diff=None,
            tol=1e-10, maxit=10, clamp_v=False, predictor="newton"):
    """Advance X0 (n, N) by n_steps steps of size dt; returns (X, Stats).  With
    the ROS2 predictor, Stats.embedded_error holds the largest scaled embedded
    error over the vertices, one entry per step."""
    X = np.array(X0, dtype=np.float64, copy=True)
    n, N = X.shape
    if n != model.n:
        raise ValueError("state has %d rows, model %s has %d states" % (n, model.name, model.n))
    stim_amp = np.zeros(N) if i_stim is None else np.asarray(i_stim, dtype=np.float64)
    diff = np.zeros(N) if i_diff is None else np.asarray(i_diff, dtype=np.float64)
    c = nodes(n_nodes)
    S = integration_matrix(n_nodes)
    stats = Stats(per_vertex_iters=np.zeros(N, dtype=np.int64))
    for step in range(n_steps):
        stim = stim_amp if stimulus_on(t0, dt, step, stim_on, stim_off) else np.zeros(N)
        X, err = sdc_step(model, X, stim, dt, n_nodes, n_sweeps, diff, tol, maxit, clamp_v, stats,
                          S, c, predictor)
        if err is not None:
            stats.embedded_error.append(float(np.max(err, initial=0.0)))
    stats.n_nonfinite = int((~np.isfinite(X).all(axis=0)).sum())
    return X, stats
