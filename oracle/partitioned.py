"""Partitioned bidomain stepping with the parabolic term inside the ROS2 stages
and the inner iterations of Algorithm 2, fp64 (oracle; test infrastructure).

Paper section 3.3.2, Algorithm 2 (partitioned strategy with SDC) and the solver
paragraph after it; section 3.3.1, equations rb_system and second_sol;
equation sdc.  On a structured grid (module diffusion: Q1 stiffness A_i, A_ie,
lumped mass M_L, homogeneous Neumann boundaries) one time step t^n -> t^n + tau
from (X^n, u^n) is

  k = 0, X^0 = X^n; repeat
    1. u^{k+1} solves the elliptic equation A_ie u = -A_i v^k (lumped-mass mean 0);
    2. ROS2 over the whole step from X^n for dX/dt = G(X; u^{k+1}), where
           G(X; u) = F(X; I_stim, I_diff = -M_L^{-1} A_i (v + u))
       is the cell model's right-hand side with the parabolic current of
       equation semi-parabolic (mass lumped: M~ = I per vertex), and its
       Jacobian J_G is the block-diagonal cell Jacobian plus -M_L^{-1} A_i in the
       (v, v) block: the term -A_i v stays implicit in both stages;
    3. the correction of equation sdc,
           (I - tau J_G(X~)) eps = X^n - X~ + tau/2 (G(X^n; u^n) + G(X~; u^{k+1})),
       X^{k+1} = X~ + eps, X~ the ROS2 result;
    4. stop once max_i |X^{k+1}_i - X^k_i| / max(|X^{k+1}_i|, s_i) <= tol (s_i the
       per-state Newton scale) or after max_inner passes;
  X^{n+1} = X^{k+1}, u^{n+1} = u^{k+1}.

Every linear system (the two ROS2 stages share one matrix, the correction has
its own) is global -- the diffusion couples the v of neighbouring vertices --
and is solved here directly (sparse LU), its plain definition; the paper uses
BiCGSTAB with block Jacobi.  The stimulus is on for a step iff
t_on <= t^n + tau/2 < t_off.  Unknowns are ordered state-major (state i of
vertex p at i N + p), the layout of the state planes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ros2 import A21, C21, GAMMA, M1, M2


@dataclass
class PartitionedStats:
    inner_iterations: list = field(default_factory=list)   # passes per step
    inner_change: list = field(default_factory=list)       # last scaled change per step
    converged: bool = True


def _global_jacobian(J, L):
    """Block-diagonal cell Jacobian J (N, n, n) plus -L in the (v, v) block, as a
    sparse (nN x nN) matrix in state-major order."""
    N, n, _ = J.shape
    p, i, k = np.nonzero(J)
    rows = i * N + p
    cols = k * N + p
    Jc = sp.csr_matrix((J[p, i, k], (rows, cols)), shape=(n * N, n * N))
    Lc = sp.csr_matrix(L)
    D = sp.bmat([[-Lc, None], [None, sp.csr_matrix((N * (n - 1), N * (n - 1)))]], format="csr")
    return Jc + D


def _flat(X):
    return np.ascontiguousarray(X).reshape(-1)


def _unflat(x, n, N):
    return x.reshape(n, N)


def rhs_G(model, X, u, bidomain, stim):
    """G(X; u): the cell right-hand side with I_diff = -M_L^{-1} A_i (v + u)."""
    return model.F(X, stim, bidomain.current(X[0], u))


def ros2_sdc_pass(model, Xn, Fn, u_new, bidomain, tau, stim):
    """Steps 2 and 3 of one inner pass: ROS2 from X^n with u^{k+1}, then the
    correction.  Fn = G(X^n; u^n).  Returns X^{k+1}."""
    n, N = Xn.shape
    L = sp.diags(1.0 / bidomain.ml) @ bidomain.Ai
    Inn = sp.identity(n * N, format="csc")
    # ROS2, both stages on (I - gamma tau J_G(X^n))
    Fx, Jx = model.FJ(Xn, stim, bidomain.current(Xn[0], u_new))
    A = (Inn - (GAMMA * tau) * _global_jacobian(Jx, L)).tocsc()
    lu = spla.splu(A)
    k1 = _unflat(lu.solve(_flat((GAMMA * tau) * Fx)), n, N)
    X2 = Xn + A21 * k1
    F2 = rhs_G(model, X2, u_new, bidomain, stim)
    k2 = _unflat(lu.solve(_flat((GAMMA * tau) * F2 - (GAMMA * C21) * k1)), n, N)
    Xt = Xn + M1 * k1 + M2 * k2
    # correction, equation sdc with the Jacobian at X~
    Ft, Jt = model.FJ(Xt, stim, bidomain.current(Xt[0], u_new))
    B = (Inn - tau * _global_jacobian(Jt, L)).tocsc()
    r = Xn - Xt + 0.5 * tau * (Fn + Ft)
    eps = _unflat(spla.splu(B).solve(_flat(r)), n, N)
    return Xt + eps


def advance_partitioned(model, X0, u0, bidomain, *, t0=0.0, dt, n_steps, i_stim=None,
                        stim_on=0.0, stim_off=0.0, tol=1e-8, max_inner=20):
    """Algorithm 2 with ROS2 and one trapezoidal correction per inner pass, the
    parabolic term implicit.  u0 is u^0 (for example the elliptic solution of
    v^0).  Returns (X, u, PartitionedStats)."""
    X = np.array(X0, dtype=np.float64, copy=True)
    u = np.array(u0, dtype=np.float64, copy=True)
    n, N = X.shape
    amp = np.zeros(N) if i_stim is None else np.asarray(i_stim, dtype=np.float64)
    scale = model.newton_scale[:, None]
    st = PartitionedStats()
    for step in range(n_steps):
        t_mid = t0 + (step + 0.5) * dt
        stim = amp if (stim_on <= t_mid < stim_off) else np.zeros(N)
        Fn = rhs_G(model, X, u, bidomain, stim)
        Xk = X
        change = np.inf
        for k in range(max_inner):
            u_new = bidomain.elliptic(Xk[0])
            Xk1 = ros2_sdc_pass(model, X, Fn, u_new, bidomain, dt, stim)
            change = float(np.max(np.abs(Xk1 - Xk) / np.maximum(np.abs(Xk1), scale)))
            Xk = Xk1
            if change <= tol:
                break
        st.inner_iterations.append(k + 1)
        st.inner_change.append(change)
        st.converged = st.converged and change <= tol
        X, u = Xk, u_new
    return X, u, st
