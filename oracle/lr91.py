"""Luo-Rudy phase-1 ventricular membrane model (oracle; test infrastructure).

Paper, section 2 ("Luo-Rody model (LR91)"): six currents I_Na, I_si, I_K,
I_K1, I_Kp, I_b; Hodgkin-Huxley gates m, h, j, d, f, X with
dk/dt = alpha_k(v)(1-k) - beta_k(v) k; one concentration ODE for [Ca]_i; eight
states in total.  The paper names the model but does not print its
equations: the rate functions, reversal potentials and constants below are
restated from the model's original publication (Luo and Rudy, Circ. Res. 68,
1991), which the paper cites.  Section 4 (Numerics, opening paragraph)
modifies three conductances to obtain spiral waves: G_si = 0.02, G_Na = 4.0
and G_K = 0.423; that "paper" set is the default here, the publication's
values are the "original" set.  G_K = 0.423 replaces the whole prefactor
0.282 sqrt(K_o/5.4) of I_K.

Units: V in mV, t in ms, currents in uA/cm^2 with C_m = 1 uF/cm^2 (so a current
is also a rate in mV/ms), [Ca]_i in mM.

State order (plane order of the GPU layout): V, Cai, m, h, j, d, f, X.
"""
from __future__ import annotations

import numpy as np

from .ad import exp, expm1, log, sqrt, val, where

NAME = "LR91"
STATE_NAMES = ("V", "Cai", "m", "h", "j", "d", "f", "X")
N_STATES = 8
# in the mixed-precision layout these states are stored and accumulated in fp64
FP64_STATES = ("V", "Cai")

PARAMS_ORIGINAL = dict(
    R=8314.0, T=310.0, F=96485.0,            # mJ/(mol K), K, C/mol
    Nao=140.0, Nai=18.0, Ko=5.4, Ki=145.0,   # mM
    PR_NaK=0.01833,
    G_Na=23.0, G_si=0.09, G_K=0.282,         # G_K here already includes sqrt(Ko/5.4) = 1
    G_K1=0.6047, G_Kp=0.0183, G_b=0.03921, E_b=-59.87,
)
# paper section 4: G_si = 0.02, G_Na = 4.0, G_K = 0.423
PARAMS_PAPER = dict(PARAMS_ORIGINAL, G_Na=4.0, G_si=0.02, G_K=0.423)

# Scale for the Newton stopping rule: s_i = max(|Y_i|, SCALE_i)
NEWTON_SCALE = np.array([100.0, 1e-4, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])

# Near-rest starting guess for the resting-state solve (not a stored rest state)
REST_GUESS_V = -84.0
REST_GUESS_CAI = 2e-4


def _x_over_1mexp(x, a):
    """x / (1 - exp(-a x)); removable singularity at x == 0 (limit 1/a, slope 1/2)."""
    xv = val(x)
    zero = xv == 0.0
    xs = where(zero, np.ones_like(xv), x)
    regular = xs / (-expm1(-a * xs))
    limit = 1.0 / a + 0.5 * x
    return where(zero, limit, regular)


def _expm1_over_x(x, a):
    """(exp(a x) - 1) / x; removable singularity at x == 0 (limit a, slope a^2/2)."""
    xv = val(x)
    zero = xv == 0.0
    xs = where(zero, np.ones_like(xv), x)
    regular = expm1(a * xs) / xs
    limit = a + 0.5 * a * a * x
    return where(zero, limit, regular)


def rates(V):
    """alpha, beta for m, h, j, d, f, X as functions of V (publication's forms)."""
    Vv = val(V)
    r = {}
    r["am"] = 0.32 * _x_over_1mexp(V + 47.13, 0.1)
    r["bm"] = 0.08 * exp(-V / 11.0)
    hi = Vv >= -40.0  # branch includes equality
    r["ah"] = where(hi, 0.0 * V, 0.135 * exp((80.0 + V) / -6.8))
    r["bh"] = where(hi, 1.0 / (0.13 * (1.0 + exp((V + 10.66) / -11.1))),
                    3.56 * exp(0.079 * V) + 3.1e5 * exp(0.35 * V))
    r["aj"] = where(hi, 0.0 * V,
                    (-1.2714e5 * exp(0.2444 * V) - 3.474e-5 * exp(-0.04391 * V))
                    * (V + 37.78) / (1.0 + exp(0.311 * (V + 79.23))))
    r["bj"] = where(hi, 0.3 * exp(-2.535e-7 * V) / (1.0 + exp(-0.1 * (V + 32.0))),
                    0.1212 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14))))
    r["ad"] = 0.095 * exp(-0.01 * (V - 5.0)) / (1.0 + exp(-0.072 * (V - 5.0)))
    r["bd"] = 0.07 * exp(-0.017 * (V + 44.0)) / (1.0 + exp(0.05 * (V + 44.0)))
    r["af"] = 0.012 * exp(-0.008 * (V + 28.0)) / (1.0 + exp(0.15 * (V + 28.0)))
    r["bf"] = 0.0065 * exp(-0.02 * (V + 30.0)) / (1.0 + exp(-0.2 * (V + 30.0)))
    r["aX"] = 0.0005 * exp(0.083 * (V + 50.0)) / (1.0 + exp(0.057 * (V + 50.0)))
    r["bX"] = 0.0013 * exp(-0.06 * (V + 20.0)) / (1.0 + exp(-0.04 * (V + 20.0)))
    return r


GATES = ("m", "h", "j", "d", "f", "X")


def gate_steady_state(V):
    """Steady state alpha/(alpha+beta) of every gate at voltage V (for initial fields)."""
    r = rates(V)
    return {g: r["a" + g] / (r["a" + g] + r["b" + g]) for g in GATES}


def rhs(x, i_stim, i_diff, p=PARAMS_PAPER, clamp_v=False):
    """F(X): dV/dt = -(I_ion + I_stim) + I_diff; gates; d[Ca]_i/dt.

    ``x`` is a sequence of the 8 states (arrays or Duals), i_stim and i_diff
    are per-vertex arrays (or scalars).  ``clamp_v`` freezes V (dV/dt = 0),
    used only by the voltage-clamp tests.
    """
    V, Cai, m, h, j, d, f, X = x
    RTF = p["R"] * p["T"] / p["F"]

    # fast sodium current
    E_Na = RTF * np.log(p["Nao"] / p["Nai"])
    I_Na = p["G_Na"] * m * m * m * h * j * (V - E_Na)

    # slow inward current
    E_si = 7.7 - 13.0287 * log(Cai)
    I_si = p["G_si"] * d * f * (V - E_si)

    # time-dependent potassium current
    E_K = RTF * np.log((p["Ko"] + p["PR_NaK"] * p["Nao"]) / (p["Ki"] + p["PR_NaK"] * p["Nai"]))
    Vv = val(V)
    Xi_regular = 2.837 * _expm1_over_x(V + 77.0, 0.04) * exp(-0.04 * (V + 35.0))
    Xi = where(Vv > -100.0, Xi_regular, 1.0 + 0.0 * V)
    I_K = p["G_K"] * X * Xi * (V - E_K)

    # time-independent potassium current
    E_K1 = RTF * np.log(p["Ko"] / p["Ki"])
    G_K1 = p["G_K1"] * np.sqrt(p["Ko"] / 5.4)
    a_K1 = 1.02 / (1.0 + exp(0.2385 * (V - E_K1 - 59.215)))
    b_K1 = (0.49124 * exp(0.08032 * (V - E_K1 + 5.476))
            + exp(0.06175 * (V - E_K1 - 594.31))) / (1.0 + exp(-0.5143 * (V - E_K1 + 4.753)))
    K1_inf = a_K1 / (a_K1 + b_K1)
    I_K1 = G_K1 * K1_inf * (V - E_K1)

    # plateau potassium current
    E_Kp = E_K1
    Kp = 1.0 / (1.0 + exp((7.488 - V) / 5.98))
    I_Kp = p["G_Kp"] * Kp * (V - E_Kp)

    # background current
    I_b = p["G_b"] * (V - p["E_b"])

    I_ion = I_Na + I_si + I_K + I_K1 + I_Kp + I_b

    r = rates(V)
    dV = -(I_ion + i_stim) + i_diff
    if clamp_v:
        dV = 0.0 * V
    out = [dV,
           -1e-4 * I_si + 0.07 * (1e-4 - Cai)]
    for g, k in zip(GATES, (m, h, j, d, f, X)):
        out.append(r["a" + g] * (1.0 - k) - r["b" + g] * k)
    return out


def rest_guess():
    """A starting point for the resting-state Newton solve: V = -84 mV, gates at
    their steady state there, [Ca]_i = 2e-4 mM."""
    V = np.array([REST_GUESS_V])
    ss = gate_steady_state(V)
    return np.array([V[0], REST_GUESS_CAI] + [float(ss[g][0]) for g in GATES])
