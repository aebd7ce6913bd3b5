"""ROS2 Rosenbrock predictor, fp64 (oracle; test infrastructure).

Paper section 3.3.1, equations rb_system and second_sol: an s-stage
Rosenbrock method in the form

    (I/(tau gamma) - J) k_j = F(X + sum_{l<j} a_jl k_l) - sum_{l<j} (c_jl / tau) k_l,
    X_new = X + sum_l m_l k_l,     X_hat = X + sum_l mhat_l k_l,

with M~ = I per vertex and J the exact Jacobian at X.  The paper uses ROS2
(two stages, second order, L-stable) and takes the second solution X_hat to
choose the next step size, but prints no coefficients.  Reading: ROS2 is the
two-stage method with gamma = 1 + 1/sqrt(2) whose stability function

    R(z) = (1 + (1 - 2 gamma) z) / (1 - gamma z)^2

agrees with exp(z) to second order and vanishes at infinity (L-stable
because gamma^2 - 2 gamma + 1/2 = 0), with the first-order embedded solution
X_hat = X + k_1 / gamma.  In the form above that is

    a_21 = 1/gamma,  c_21 = 2/gamma,  m_1 = 3/(2 gamma),  m_2 = 1/(2 gamma),
    mhat_1 = 1/gamma,  mhat_2 = 0.

The per-vertex right-hand side does not depend on time inside a step (the
stimulus is constant over a step, the diffusion current over the call), so
the stage times alpha_j and the time-derivative term drop out.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.0 + 1.0 / math.sqrt(2.0)
A21 = 1.0 / GAMMA
C21 = 2.0 / GAMMA
M1 = 3.0 / (2.0 * GAMMA)
M2 = 1.0 / (2.0 * GAMMA)
MHAT1 = 1.0 / GAMMA
MHAT2 = 0.0


def _solve(A, b):
    return np.linalg.solve(A, b[..., None])[..., 0]


def ros2_step(model, X, tau, i_stim, i_diff, clamp_v=False):
    """One ROS2 step of length tau from X (n, N).

    Returns (X_new, X_hat, F(X)); F(X) is returned because the correction
    sweeps that follow need it at the left end of the step."""
    n, N = X.shape
    F0, J = model.FJ(X, i_stim, i_diff, clamp_v)
    A = np.eye(n)[None] / (tau * GAMMA) - J                    # (N, n, n)
    k1 = _solve(A, F0.T).T
    F2 = model.F(X + A21 * k1, i_stim, i_diff, clamp_v)
    k2 = _solve(A, (F2 - (C21 / tau) * k1).T).T
    X_new = X + M1 * k1 + M2 * k2
    X_hat = X + MHAT1 * k1 + MHAT2 * k2
    return X_new, X_hat, F0
