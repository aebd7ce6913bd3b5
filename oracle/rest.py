"""Resting states and the TT06 charge invariant (oracle; test infrastructure).

LR91: the resting state X* solves F(X*) = 0 with I_stim = I_diff = 0; Newton's
method with the exact Jacobian, started near -84 mV.

TT06 conserves charge exactly:
    Q(X) = C_m V - F (V_c (Na_i + K_i) + 2 (V_c Ca_i,tot + V_sr Ca_SR,tot + V_ss Ca_SS,tot))
is constant along every solution (each ion flux of the voltage equation
reappears in a concentration equation with its valence and volume factor), so
F(X) = 0 has a one-parameter family of solutions and J(X*) is singular in
one direction.  Without pacing the model drifts for minutes (the SR unloads,
Na_i falls) towards the member of that family on the invariant level of its
published initial conditions; ``tt06_unpaced_fixed_point`` solves for it by
Newton with the K_i row replaced by Q(X) = Q(X_published).  The workloads do
not start there: like the paper's simulations they start from the published
initial conditions, the quiescent state of a paced cell, whose slow drift is
irrelevant over the simulated milliseconds.
"""
from __future__ import annotations

import numpy as np

from . import lr91, tt06
from .ad import seed, split
from .models import LR91, TT06


def solve_rest(model, x_start, tol=1e-15, maxit=50):
    """Newton on F(x) = 0 for a single cell."""
    x = np.array(x_start, dtype=np.float64).reshape(-1, 1)
    zero = np.zeros(1)
    for _ in range(maxit):
        F, J = model.FJ(x, zero, zero)
        delta = np.linalg.solve(J[0], -F[:, 0])
        x[:, 0] += delta
        if np.max(np.abs(delta) / np.maximum(np.abs(x[:, 0]), model.newton_scale)) < tol:
            break
    return x[:, 0]


def lr91_rest():
    return solve_rest(LR91, lr91.rest_guess())


def tt06_charge(x, p=tt06.PARAMS):
    """Charge invariant Q of TT06 (works on arrays and Duals)."""
    V, Cai, CaSR, CaSS, Nai, Ki = x[:6]
    CaiT = Cai + p["Buf_c"] * Cai / (Cai + p["K_bufc"])
    CaSRT = CaSR + p["Buf_sr"] * CaSR / (CaSR + p["K_bufsr"])
    CaSST = CaSS + p["Buf_ss"] * CaSS / (CaSS + p["K_bufss"])
    return p["Cm"] * V - p["F"] * (p["Vc"] * (Nai + Ki)
                                   + 2.0 * (p["Vc"] * CaiT + p["Vsr"] * CaSRT + p["Vss"] * CaSST))


def tt06_unpaced_fixed_point(x_start, level, tol=1e-15, maxit=50):
    """F(X) = 0 on the invariant level Q(X) = level (K_i row replaced by the invariant)."""
    x = np.array(x_start, dtype=np.float64)
    iK = TT06.state_names.index("Ki")
    zero = np.zeros(1)
    for _ in range(maxit):
        xs = seed(x.reshape(-1, 1))
        F, J = split(TT06._rhs(xs, zero, zero, TT06.params, False), TT06.n, 1)
        F, J = F[:, 0], J[0]
        q = tt06_charge(xs)
        F[iK] = q.v[0] - level
        J[iK, :] = q.d[:, 0]
        delta = np.linalg.solve(J, -F)
        x += delta
        if np.max(np.abs(delta) / np.maximum(np.abs(x), TT06.newton_scale)) < tol:
            break
    return x
