"""ten Tusscher-Panfilov 2006 human ventricular model, epicardial cell
(oracle; test infrastructure).

Paper, section 2 (its subsection on the ten Tusscher model): 19 states (one voltage,
gating and concentration variables) and 12 currents: fast Na, L-type Ca,
rapid and slow delayed rectifier K, inward rectifier K, transient outward K,
plateau K, Na-Ca exchanger, Na-K pump, sarcolemmal Ca pump, background Na and
background Ca.  The paper takes the epicardial parameter set of the original
publication and prints no equations; the forms and constants below are
restated from that publication (ten Tusscher and Panfilov, Am. J. Physiol.
Heart 291, 2006).

Readings (listed with the other readings of the paper in the design notes):
  * the state holds FREE concentrations of [Ca]_i, [Ca]_SR and [Ca]_SS;
    buffering enters through the rapid-equilibrium factor
    1 / (1 + Buf K / (Ca + K)^2), the time derivative of the publication's
    total-to-free relation;
  * dV/dt = -(I_ion + I_stim) + I_diff, currents in pA/pF and C_m = 1 uF/cm^2
    in the voltage equation (paper equation parabolic with the diffusion
    held fixed); the stimulus and the fixed diffusion current are carried by
    K+ in d[K]_i/dt (the publication's printed K_i equation with I_ax = I_diff);
  * the removable singularity of I_CaL at V = 15 mV is evaluated through
    u / expm1(2u) with the limit 1/2 at u == 0.

State order (plane order of the GPU layout):
  V, Cai, CaSR, CaSS, Nai, Ki, m, h, j, xr1, xr2, xs, r, s, d, f, f2, fCass, Rbar
"""
from __future__ import annotations

import numpy as np

from .ad import exp, expm1, log, sqrt, val, where

NAME = "TT06"
STATE_NAMES = ("V", "Cai", "CaSR", "CaSS", "Nai", "Ki",
               "m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d", "f", "f2", "fCass", "Rbar")
N_STATES = 19
FP64_STATES = ("V", "Cai", "CaSR", "CaSS", "Nai", "Ki")

PARAMS = dict(
    R=8314.472, T=310.0, F=96485.3415,       # mJ/(K mol), K, C/mol
    Cm=0.185, Vc=0.016404, Vsr=0.001094, Vss=0.00005468,
    Ko=5.4, Nao=140.0, Cao=2.0,
    G_Na=14.838, G_K1=5.405, G_to=0.294, G_Kr=0.153, G_Ks=0.392, p_KNa=0.03,
    G_CaL=3.980e-5, k_NaCa=1000.0, gamma=0.35, Km_Ca=1.38, Km_Nai=87.5,
    k_sat=0.1, alpha=2.5, P_NaK=2.724, Km_K=1.0, Km_Na=40.0,
    G_pK=0.0146, G_pCa=0.1238, K_pCa=0.0005, G_bNa=0.00029, G_bCa=0.000592,
    Vmax_up=0.006375, K_up=0.00025, V_rel=0.102, k1p=0.15, k2p=0.045,
    k3=0.060, k4=0.005, EC=1.5, max_sr=2.5, min_sr=1.0,
    V_leak=0.00036, V_xfer=0.0038,
    Buf_c=0.2, K_bufc=0.001, Buf_sr=10.0, K_bufsr=0.3, Buf_ss=0.4, K_bufss=0.00025,
)

NEWTON_SCALE = np.array([100.0, 1e-4, 1.0, 1e-4, 10.0, 100.0] + [1.0] * 13)

# Initial conditions printed with the publication (epicardial cell); used only
# as the starting point of the resting-state solve.
PUBLISHED_INITIAL = dict(
    V=-85.23, Cai=0.000126, CaSR=3.64, CaSS=0.00036, Nai=8.604, Ki=136.89,
    m=0.00172, h=0.7444, j=0.7045, xr1=0.00621, xr2=0.4712, xs=0.0095,
    r=2.42e-8, s=0.999998, d=3.373e-5, f=0.7888, f2=0.9755, fCass=0.9953,
    Rbar=0.9073,
)

V_GATES = ("m", "h", "j", "xr1", "xr2", "xs", "r", "s", "d", "f", "f2")


def gate_kinetics(V):
    """Steady states x_inf(V) and time constants tau_x(V) of the 11 voltage gates."""
    Vv = val(V)
    g = {}
    # I_Na gates
    g["m_inf"] = 1.0 / ((1.0 + exp((-56.86 - V) / 9.03)) ** 2)
    a_m = 1.0 / (1.0 + exp((-60.0 - V) / 5.0))
    b_m = 0.1 / (1.0 + exp((V + 35.0) / 5.0)) + 0.10 / (1.0 + exp((V - 50.0) / 200.0))
    g["m_tau"] = a_m * b_m
    hj_inf = 1.0 / ((1.0 + exp((V + 71.55) / 7.43)) ** 2)
    g["h_inf"] = hj_inf
    g["j_inf"] = hj_inf
    hi = Vv >= -40.0  # branch includes equality
    a_h = where(hi, 0.0 * V, 0.057 * exp(-(V + 80.0) / 6.8))
    b_h = where(hi, 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1))),
                2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V))
    g["h_tau"] = 1.0 / (a_h + b_h)
    a_j = where(hi, 0.0 * V,
                (-2.5428e4 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V))
                * (V + 37.78) / (1.0 + exp(0.311 * (V + 79.23))))
    b_j = where(hi, 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0))),
                0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14))))
    g["j_tau"] = 1.0 / (a_j + b_j)
    # I_Kr gates
    g["xr1_inf"] = 1.0 / (1.0 + exp((-26.0 - V) / 7.0))
    a_xr1 = 450.0 / (1.0 + exp((-45.0 - V) / 10.0))
    b_xr1 = 6.0 / (1.0 + exp((V + 30.0) / 11.5))
    g["xr1_tau"] = a_xr1 * b_xr1
    g["xr2_inf"] = 1.0 / (1.0 + exp((V + 88.0) / 24.0))
    a_xr2 = 3.0 / (1.0 + exp((-60.0 - V) / 20.0))
    b_xr2 = 1.12 / (1.0 + exp((V - 60.0) / 20.0))
    g["xr2_tau"] = a_xr2 * b_xr2
    # I_Ks gate
    g["xs_inf"] = 1.0 / (1.0 + exp((-5.0 - V) / 14.0))
    a_xs = 1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0))
    b_xs = 1.0 / (1.0 + exp((V - 35.0) / 15.0))
    g["xs_tau"] = a_xs * b_xs + 80.0
    # I_to gates (epicardial)
    g["r_inf"] = 1.0 / (1.0 + exp((20.0 - V) / 6.0))
    g["r_tau"] = 9.5 * exp(-((V + 40.0) ** 2) / 1800.0) + 0.8
    g["s_inf"] = 1.0 / (1.0 + exp((V + 20.0) / 5.0))
    g["s_tau"] = 85.0 * exp(-((V + 45.0) ** 2) / 320.0) + 5.0 / (1.0 + exp((V - 20.0) / 5.0)) + 3.0
    # I_CaL gates
    g["d_inf"] = 1.0 / (1.0 + exp((-8.0 - V) / 7.5))
    a_d = 1.4 / (1.0 + exp((-35.0 - V) / 13.0)) + 0.25
    b_d = 1.4 / (1.0 + exp((V + 5.0) / 5.0))
    c_d = 1.0 / (1.0 + exp((50.0 - V) / 20.0))
    g["d_tau"] = a_d * b_d + c_d
    g["f_inf"] = 1.0 / (1.0 + exp((V + 20.0) / 7.0))
    a_f = 1102.5 * exp(-((V + 27.0) ** 2) / 225.0)
    b_f = 200.0 / (1.0 + exp((13.0 - V) / 10.0))
    c_f = 180.0 / (1.0 + exp((V + 30.0) / 10.0)) + 20.0
    g["f_tau"] = a_f + b_f + c_f
    g["f2_inf"] = 0.67 / (1.0 + exp((V + 35.0) / 7.0)) + 0.33
    a_f2 = 600.0 * exp(-((V + 25.0) ** 2) / 170.0)
    b_f2 = 31.0 / (1.0 + exp((25.0 - V) / 10.0))
    c_f2 = 16.0 / (1.0 + exp((V + 30.0) / 10.0))
    g["f2_tau"] = a_f2 + b_f2 + c_f2
    return g


def fcass_kinetics(CaSS):
    q = 1.0 + (CaSS / 0.05) ** 2
    return 0.6 / q + 0.4, 80.0 / q + 2.0


def gate_steady_state(V, CaSS):
    """x_inf of the 11 voltage gates at V and fCass_inf at CaSS (initial fields)."""
    g = gate_kinetics(V)
    out = {k: g[k + "_inf"] for k in V_GATES}
    out["fCass"] = fcass_kinetics(CaSS)[0]
    return out


def rhs(x, i_stim, i_diff, p=PARAMS, clamp_v=False):
    """F(X) for the 19 states; see the module docstring for the readings."""
    (V, Cai, CaSR, CaSS, Nai, Ki,
     m, h, j, xr1, xr2, xs, r, s, d, f, f2, fCass, Rbar) = x
    RTF = p["R"] * p["T"] / p["F"]
    FRT = 1.0 / RTF

    # reversal potentials
    E_Na = RTF * log(p["Nao"] / Nai)
    E_K = RTF * log(p["Ko"] / Ki)
    E_Ca = 0.5 * RTF * log(p["Cao"] / Cai)
    E_Ks = RTF * log((p["Ko"] + p["p_KNa"] * p["Nao"]) / (Ki + p["p_KNa"] * Nai))

    # currents (pA/pF)
    I_Na = p["G_Na"] * m * m * m * h * j * (V - E_Na)
    I_to = p["G_to"] * r * s * (V - E_K)
    I_Kr = p["G_Kr"] * np.sqrt(p["Ko"] / 5.4) * xr1 * xr2 * (V - E_K)
    I_Ks = p["G_Ks"] * xs * xs * (V - E_Ks)

    a_K1 = 0.1 / (1.0 + exp(0.06 * (V - E_K - 200.0)))
    b_K1 = (3.0 * exp(0.0002 * (V - E_K + 100.0)) + exp(0.1 * (V - E_K - 10.0))) \
        / (1.0 + exp(-0.5 * (V - E_K)))
    xK1_inf = a_K1 / (a_K1 + b_K1)
    I_K1 = p["G_K1"] * np.sqrt(p["Ko"] / 5.4) * xK1_inf * (V - E_K)

    # L-type Ca: G d f f2 fCass 4 (V-15) F^2/(RT) (0.25 CaSS e^{2u} - Cao)/(e^{2u} - 1),
    # u = (V-15) F/(RT); written as 4 F (0.25 CaSS e^{2u} - Cao) * u/expm1(2u)
    u = (V - 15.0) * FRT
    uv = val(u)
    zero = uv == 0.0
    us = where(zero, np.ones_like(uv), u)
    ghk = where(zero, 0.5 - 0.5 * u, us / expm1(2.0 * us))   # limit 1/2, slope -1/2
    e2u = exp(2.0 * u)
    I_CaL = p["G_CaL"] * d * f * f2 * fCass * 4.0 * p["F"] * (0.25 * CaSS * e2u - p["Cao"]) * ghk

    eg = exp(p["gamma"] * V * FRT)
    eg1 = exp((p["gamma"] - 1.0) * V * FRT)
    I_NaCa = p["k_NaCa"] * (eg * Nai ** 3 * p["Cao"] - eg1 * p["Nao"] ** 3 * Cai * p["alpha"]) \
        / ((p["Km_Nai"] ** 3 + p["Nao"] ** 3) * (p["Km_Ca"] + p["Cao"]) * (1.0 + p["k_sat"] * eg1))

    I_NaK = p["P_NaK"] * p["Ko"] / (p["Ko"] + p["Km_K"]) * Nai / (Nai + p["Km_Na"]) \
        / (1.0 + 0.1245 * exp(-0.1 * V * FRT) + 0.0353 * exp(-V * FRT))

    I_pCa = p["G_pCa"] * Cai / (p["K_pCa"] + Cai)
    I_pK = p["G_pK"] * (V - E_K) / (1.0 + exp((25.0 - V) / 5.98))
    I_bNa = p["G_bNa"] * (V - E_Na)
    I_bCa = p["G_bCa"] * (V - E_Ca)

    I_ion = (I_Na + I_K1 + I_to + I_Kr + I_Ks + I_CaL + I_NaCa + I_NaK
             + I_pCa + I_pK + I_bNa + I_bCa)

    # calcium handling
    k_casr = p["max_sr"] - (p["max_sr"] - p["min_sr"]) / (1.0 + (p["EC"] / CaSR) ** 2)
    k1 = p["k1p"] / k_casr
    k2 = p["k2p"] * k_casr
    O = k1 * CaSS * CaSS * Rbar / (p["k3"] + k1 * CaSS * CaSS)
    I_rel = p["V_rel"] * O * (CaSR - CaSS)
    I_up = p["Vmax_up"] / (1.0 + p["K_up"] ** 2 / (Cai * Cai))
    I_leak = p["V_leak"] * (CaSR - Cai)
    I_xfer = p["V_xfer"] * (CaSS - Cai)

    beta_c = 1.0 / (1.0 + p["Buf_c"] * p["K_bufc"] / ((Cai + p["K_bufc"]) ** 2))
    beta_sr = 1.0 / (1.0 + p["Buf_sr"] * p["K_bufsr"] / ((CaSR + p["K_bufsr"]) ** 2))
    beta_ss = 1.0 / (1.0 + p["Buf_ss"] * p["K_bufss"] / ((CaSS + p["K_bufss"]) ** 2))

    cF_c = p["Cm"] / (p["Vc"] * p["F"])
    dCai = beta_c * (-(I_bCa + I_pCa - 2.0 * I_NaCa) * 0.5 * cF_c
                     + (I_leak - I_up) * p["Vsr"] / p["Vc"] + I_xfer)
    dCaSR = beta_sr * (I_up - I_leak - I_rel)
    dCaSS = beta_ss * (-I_CaL * p["Cm"] / (2.0 * p["Vss"] * p["F"])
                       + I_rel * p["Vsr"] / p["Vss"] - I_xfer * p["Vc"] / p["Vss"])
    dNai = -(I_Na + I_bNa + 3.0 * I_NaK + 3.0 * I_NaCa) * cF_c
    dKi = -(I_K1 + I_to + I_Kr + I_Ks - 2.0 * I_NaK + I_pK + i_stim - i_diff) * cF_c

    dRbar = -k2 * CaSS * Rbar + p["k4"] * (1.0 - Rbar)

    g = gate_kinetics(V)
    fc_inf, fc_tau = fcass_kinetics(CaSS)

    dV = -(I_ion + i_stim) + i_diff
    if clamp_v:
        dV = 0.0 * V
    out = [dV, dCai, dCaSR, dCaSS, dNai, dKi]
    for name, k in zip(V_GATES, (m, h, j, xr1, xr2, xs, r, s, d, f, f2)):
        out.append((g[name + "_inf"] - k) / g[name + "_tau"])
    out.append((fc_inf - fCass) / fc_tau)
    out.append(dRbar)
    return out


def published_initial():
    return np.array([PUBLISHED_INITIAL[k] for k in STATE_NAMES])
