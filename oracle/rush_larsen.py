"""Rush-Larsen predictor, fp64 (oracle; test infrastructure).

A predictor for one Gauss-Lobatto sub-interval of length dtau that treats the
two kinds of state differently, as the per-vertex reaction stage allows:

1. gating states (every state outside the intracellular core: the gates, and
   for TT06 also fCass and Rbar).  Each of their rows is linear in the state
   itself, F_g = a_g(x) - b_g(x) g.  With every other state frozen at X_m the
   exact solution over dtau is the exponential step
       g_new = g + dtau F_g(X_m) phi(dtau J_gg(X_m)),  phi(z) = (e^z - 1)/z,
   phi(0) = 1, where J_gg = -b_g is the diagonal Jacobian entry (Rush and
   Larsen's scheme, written for any row linear in its own state);
2. the core (V and the intracellular concentrations: the states the model
   lists as fp64 states).  Backward Euler with the gates held at g_new,
       Y_c - X_c,m - dtau F_c(Y_c, g_new) = 0,
   solved by local Newton on the core block of the Jacobian only, with the
   same stop rule as the full Newton predictor (scaled max-norm of the
   update over the core states, at least one and at most maxit iterations,
   the last iterate kept).

The sweeps that follow are unchanged.  For a model without gating states (the
scalar test problems) this is the backward-Euler Newton predictor.
"""
from __future__ import annotations

import numpy as np


def _solve(A, b):
    return np.linalg.solve(A, b[..., None])[..., 0]


def phi(z):
    """(e^z - 1) / z with phi(0) = 1."""
    zs = np.where(z == 0.0, 1.0, z)
    return np.where(z == 0.0, 1.0, np.expm1(zs) / zs)


def split_states(model):
    core = [model.state_names.index(s) for s in model.fp64_states]
    gating = [i for i in range(model.n) if i not in core]
    return core, gating


def rush_larsen_be(model, Xm, dtau, i_stim, i_diff, tol, maxit, clamp_v, stats):
    n, N = Xm.shape
    core, gating = split_states(model)
    F, J = model.FJ(Xm, i_stim, i_diff, clamp_v)
    Y = Xm.copy()
    for g in gating:
        Y[g] = Xm[g] + dtau * F[g] * phi(dtau * J[:, g, g])
    # backward Euler on the core, gates held
    nc = len(core)
    Ic = np.eye(nc)
    scale = model.newton_scale[core][:, None]
    it = np.zeros(N, dtype=np.int64)
    active = np.ones(N, dtype=bool)
    converged = np.zeros(N, dtype=bool)
    while active.any():
        idx = np.nonzero(active)[0]
        Ya = Y[:, idx]
        F, J = model.FJ(Ya, _pick(i_stim, idx), _pick(i_diff, idx), clamp_v)
        Jc = J[:, core][:, :, core]
        G = Ya[core] - Xm[core][:, idx] - dtau * F[core]
        delta = _solve(Ic[None] - dtau * Jc, -G.T).T
        Yc = Ya[core] + delta
        Y[np.ix_(core, idx)] = Yc
        it[idx] += 1
        err = np.max(np.abs(delta) / np.maximum(np.abs(Yc), scale), axis=0)
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
