// ten Tusscher-Panfilov 2006 human ventricular model, epicardial cell,
// device form (paper section 2, "Ten Tusscher model (TP06)").
//
// 19 states; 12 currents: I_Na, I_CaL, I_Kr, I_Ks, I_K1, I_to, I_pK, I_NaCa,
// I_NaK, I_pCa, I_bNa, I_bCa.  The paper takes the epicardial parameter set
// of the model's publication and does not print it; the forms and constants
// are restated from that publication (Am. J. Physiol. Heart 291, 2006).  Readings shared with the reference implementation used for testing:
// free [Ca]_i, [Ca]_SR, [Ca]_SS as states with rapid-equilibrium buffering
// factors; dV/dt = -(I_ion + I_stim) + I_diff with C_m = 1 uF/cm^2 and
// currents in pA/pF; stimulus and diffusion current carried by K+ in d[K]_i/dt;
// the removable singularity of I_CaL at V = 15 mV through u / expm1(2u).
//
// Plane order: V, Cai, CaSR, CaSS, Nai, Ki (double in the mixed layout), then
// the gates m, h, j, xr1, xr2, xs, r, s, d, f, f2, fCass and Rbar.
//
// Compile-time Jacobian pattern (CTSM), 76 of 361 entries:
//   V     -> all states but CaSR and Rbar        (17)
//   Cai   -> V, Nai, Cai, CaSR, CaSS
//   CaSR  -> Cai, CaSR, CaSS, Rbar
//   CaSS  -> V, d, f, f2, fCass, CaSS, CaSR, Rbar, Cai
//   Nai   -> V, m, h, j, Nai, Cai
//   Ki    -> V, r, s, xr1, xr2, xs, Nai, Ki
//   voltage gates -> V, itself;  fCass -> CaSS, itself;  Rbar -> CaSS, CaSR, Rbar
#pragma once

#include <cmath>

#include "dual.h"

namespace ionic {

struct TT06 {
  static constexpr int N = 19;
  static constexpr int N64 = 6;
  enum : int { V = 0, Cai, CaSR, CaSS, Nai, Ki, m, h, j, xr1, xr2, xs, r, s, d, f, f2, fCass, Rbar };

  static constexpr uint32_t ROW[N] = {
      0x7FFFFu & ~(bit(CaSR) | bit(Rbar)),                                   // V
      bit(V) | bit(Nai) | bit(Cai) | bit(CaSR) | bit(CaSS),                  // Cai
      bit(Cai) | bit(CaSR) | bit(CaSS) | bit(Rbar),                          // CaSR
      bit(V) | bit(d) | bit(f) | bit(f2) | bit(fCass) | bit(CaSS) | bit(CaSR) | bit(Rbar) |
          bit(Cai),                                                          // CaSS
      bit(V) | bit(m) | bit(h) | bit(j) | bit(Nai) | bit(Cai),               // Nai
      bit(V) | bit(r) | bit(s) | bit(xr1) | bit(xr2) | bit(xs) | bit(Nai) | bit(Ki),  // Ki
      bit(V) | bit(m), bit(V) | bit(h), bit(V) | bit(j), bit(V) | bit(xr1), bit(V) | bit(xr2), bit(V) | bit(xs),
      bit(V) | bit(r), bit(V) | bit(s), bit(V) | bit(d), bit(V) | bit(f), bit(V) | bit(f2),
      bit(CaSS) | bit(fCass),                                                // fCass
      bit(CaSS) | bit(CaSR) | bit(Rbar)};                                    // Rbar

  static constexpr double SCALE[N] = {100.0, 1e-4, 1.0, 1e-4, 10.0, 100.0, 1.0, 1.0, 1.0, 1.0,
                                      1.0,   1.0,  1.0, 1.0,  1.0,  1.0,   1.0, 1.0, 1.0};

  // Resting state loaded by ionic_init when no initial state is given: the
  // epicardial initial conditions printed with the model's publication (the
  // quiescent state of a paced cell).  F(X) = 0 is not used: the model
  // conserves charge exactly, so its equilibria form a one-parameter family.
  static constexpr bool REST_BY_NEWTON = false;
  static constexpr double REST_GUESS[N] = {
      -85.23, 0.000126, 3.64,    0.00036, 8.604,  136.89, 0.00172,  0.7444,   0.7045, 0.00621,
      0.4712, 0.0095,   2.42e-8, 0.999998, 3.373e-5, 0.7888, 0.9755, 0.9953, 0.9073};

  static constexpr int N_PARAMS = 47;
  static constexpr const char* PARAM_NAMES[N_PARAMS] = {
      "R", "T", "F", "Cm", "Vc", "Vsr", "Vss", "Ko", "Nao", "Cao", "G_Na", "G_K1", "G_to",
      "G_Kr", "G_Ks", "p_KNa", "G_CaL", "k_NaCa", "gamma", "Km_Ca", "Km_Nai", "k_sat", "alpha",
      "P_NaK", "Km_K", "Km_Na", "G_pK", "G_pCa", "K_pCa", "G_bNa", "G_bCa", "Vmax_up", "K_up",
      "V_rel", "k1p", "k2p", "k3", "k4", "EC", "max_sr", "min_sr", "V_leak", "V_xfer", "Buf_c",
      "K_bufc", "Buf_sr", "K_bufsr"};
  // (Buf_ss and K_bufss follow as the last two raw entries, not overridable)
  static constexpr double PARAM_DEFAULTS[N_PARAMS + 2] = {
      8314.472, 310.0,  96485.3415, 0.185,    0.016404, 0.001094, 0.00005468, 5.4,   140.0, 2.0,
      14.838,   5.405,  0.294,      0.153,    0.392,    0.03,     3.980e-5,   1000.0, 0.35, 1.38,
      87.5,     0.1,    2.5,        2.724,    1.0,      40.0,     0.0146,     0.1238, 0.0005,
      0.00029,  0.000592, 0.006375, 0.00025,  0.102,    0.15,     0.045,      0.060, 0.005, 1.5,
      2.5,      1.0,    0.00036,    0.0038,   0.2,      0.001,    10.0,       0.3,   0.4,   0.00025};

  template <class T>
  struct Params {
    T RTF, FRT, halfRTF, Ko, Nao, Cao, logNao, logKo, logCao, ks_num;
    T G_Na, G_K1s, G_to, G_Krs, G_Ks, p_KNa;
    T G_CaL4F;                 // G_CaL * 4 F
    T naca_c1, naca_c2, gamma, gamma1, k_sat;   // I_NaCa: k/((Km^3+Nao^3)(KmCa+Cao)) * Cao, * Nao^3 alpha
    T nak_c;                   // P_NaK Ko/(Ko + Km_K)
    T Km_Na, G_pK, G_pCa, K_pCa, G_bNa, G_bCa;
    T Vmax_up, K_up2, V_rel, k1p, k2p, k3, k4, EC2, max_sr, dsr, V_leak, V_xfer;
    T bc, K_bufc, bsr, K_bufsr, bss, K_bufss;   // Buf*K products
    T cF_c, halfcF_c, caL_ss, sr_ss, c_ss, sr_c;  // volume / capacitance ratios
  };

  template <class T>
  static Params<T> derive(const double* q) {
    const double R = q[0], Tk = q[1], F = q[2], Cm = q[3], Vc = q[4], Vsr = q[5], Vss = q[6];
    const double Ko = q[7], Nao = q[8], Cao = q[9];
    const double RTF = R * Tk / F;
    Params<T> p;
    p.RTF = T(RTF);
    p.FRT = T(1.0 / RTF);
    p.halfRTF = T(0.5 * RTF);
    p.Ko = T(Ko);
    p.Nao = T(Nao);
    p.Cao = T(Cao);
    p.logNao = T(std::log(Nao));
    p.logKo = T(std::log(Ko));
    p.logCao = T(std::log(Cao));
    p.ks_num = T(std::log(Ko + q[15] * Nao));
    p.G_Na = T(q[10]);
    p.G_K1s = T(q[11] * std::sqrt(Ko / 5.4));
    p.G_to = T(q[12]);
    p.G_Krs = T(q[13] * std::sqrt(Ko / 5.4));
    p.G_Ks = T(q[14]);
    p.p_KNa = T(q[15]);
    p.G_CaL4F = T(q[16] * 4.0 * F);
    const double kNaCa = q[17], gam = q[18], KmCa = q[19], KmNai = q[20], ksat = q[21], alp = q[22];
    const double den = (KmNai * KmNai * KmNai + Nao * Nao * Nao) * (KmCa + Cao);
    p.naca_c1 = T(kNaCa * Cao / den);
    p.naca_c2 = T(kNaCa * Nao * Nao * Nao * alp / den);
    p.gamma = T(gam);
    p.gamma1 = T(gam - 1.0);
    p.k_sat = T(ksat);
    p.nak_c = T(q[23] * Ko / (Ko + q[24]));
    p.Km_Na = T(q[25]);
    p.G_pK = T(q[26]);
    p.G_pCa = T(q[27]);
    p.K_pCa = T(q[28]);
    p.G_bNa = T(q[29]);
    p.G_bCa = T(q[30]);
    p.Vmax_up = T(q[31]);
    p.K_up2 = T(q[32] * q[32]);
    p.V_rel = T(q[33]);
    p.k1p = T(q[34]);
    p.k2p = T(q[35]);
    p.k3 = T(q[36]);
    p.k4 = T(q[37]);
    p.EC2 = T(q[38] * q[38]);
    p.max_sr = T(q[39]);
    p.dsr = T(q[39] - q[40]);
    p.V_leak = T(q[41]);
    p.V_xfer = T(q[42]);
    p.bc = T(q[43] * q[44]);
    p.K_bufc = T(q[44]);
    p.bsr = T(q[45] * q[46]);
    p.K_bufsr = T(q[46]);
    p.bss = T(q[47] * q[48]);
    p.K_bufss = T(q[48]);
    p.cF_c = T(Cm / (Vc * F));
    p.halfcF_c = T(0.5 * Cm / (Vc * F));
    p.caL_ss = T(Cm / (2.0 * Vss * F));
    p.sr_ss = T(Vsr / Vss);
    p.c_ss = T(Vc / Vss);
    p.sr_c = T(Vsr / Vc);
    return p;
  }

  // Steady state and inverse time constant of the 11 voltage gates at V.
  template <class TV>
  struct GateKin {
    decltype(TV{} * 1.0) inf[11], rtau[11];
  };

  template <class T, class TV>
  IONIC_DEV static GateKin<TV> gate_kinetics(const TV& Vm) {
    GateKin<TV> k;
    const bool hi = Vm.v >= T(-40);
    const auto zero = Vm * 0.0;
    // m
    const auto em = 1.0 + exp((-56.86 - Vm) * (1.0 / 9.03));
    k.inf[0] = 1.0 / (em * em);
    const auto a_m = 1.0 / (1.0 + exp((-60.0 - Vm) * (1.0 / 5.0)));
    const auto b_m = 0.1 / (1.0 + exp((Vm + 35.0) * (1.0 / 5.0))) +
                     0.10 / (1.0 + exp((Vm - 50.0) * (1.0 / 200.0)));
    k.rtau[0] = 1.0 / (a_m * b_m);
    // h, j (same steady state)
    const auto ehj = 1.0 + exp((Vm + 71.55) * (1.0 / 7.43));
    const auto hj_inf = 1.0 / (ehj * ehj);
    k.inf[1] = hj_inf;
    k.inf[2] = hj_inf;
    const auto a_h = select(hi, zero, 0.057 * exp((Vm + 80.0) * (-1.0 / 6.8)));
    const auto b_h = select(hi, 0.77 / (0.13 * (1.0 + exp((Vm + 10.66) * (-1.0 / 11.1)))),
                            2.7 * exp(0.079 * Vm) + 3.1e5 * exp(0.3485 * Vm));
    k.rtau[1] = a_h + b_h;
    const auto a_j = select(hi, zero,
                            (-2.5428e4 * exp(0.2444 * Vm) - 6.948e-6 * exp(-0.04391 * Vm)) *
                                (Vm + 37.78) / (1.0 + exp(0.311 * (Vm + 79.23))));
    const auto b_j = select(hi, 0.6 * exp(0.057 * Vm) / (1.0 + exp(-0.1 * (Vm + 32.0))),
                            0.02424 * exp(-0.01052 * Vm) / (1.0 + exp(-0.1378 * (Vm + 40.14))));
    k.rtau[2] = a_j + b_j;
    // xr1, xr2
    k.inf[3] = 1.0 / (1.0 + exp((-26.0 - Vm) * (1.0 / 7.0)));
    const auto a_xr1 = 450.0 / (1.0 + exp((-45.0 - Vm) * (1.0 / 10.0)));
    const auto b_xr1 = 6.0 / (1.0 + exp((Vm + 30.0) * (1.0 / 11.5)));
    k.rtau[3] = 1.0 / (a_xr1 * b_xr1);
    k.inf[4] = 1.0 / (1.0 + exp((Vm + 88.0) * (1.0 / 24.0)));
    const auto a_xr2 = 3.0 / (1.0 + exp((-60.0 - Vm) * (1.0 / 20.0)));
    const auto b_xr2 = 1.12 / (1.0 + exp((Vm - 60.0) * (1.0 / 20.0)));
    k.rtau[4] = 1.0 / (a_xr2 * b_xr2);
    // xs
    k.inf[5] = 1.0 / (1.0 + exp((-5.0 - Vm) * (1.0 / 14.0)));
    const auto a_xs = 1400.0 / sqrt(1.0 + exp((5.0 - Vm) * (1.0 / 6.0)));
    const auto b_xs = 1.0 / (1.0 + exp((Vm - 35.0) * (1.0 / 15.0)));
    k.rtau[5] = 1.0 / (a_xs * b_xs + 80.0);
    // r, s (epicardial)
    k.inf[6] = 1.0 / (1.0 + exp((20.0 - Vm) * (1.0 / 6.0)));
    const auto v40 = Vm + 40.0;
    k.rtau[6] = 1.0 / (9.5 * exp((v40 * v40) * (-1.0 / 1800.0)) + 0.8);
    k.inf[7] = 1.0 / (1.0 + exp((Vm + 20.0) * (1.0 / 5.0)));
    const auto v45 = Vm + 45.0;
    k.rtau[7] = 1.0 / (85.0 * exp((v45 * v45) * (-1.0 / 320.0)) +
                       5.0 / (1.0 + exp((Vm - 20.0) * (1.0 / 5.0))) + 3.0);
    // d
    k.inf[8] = 1.0 / (1.0 + exp((-8.0 - Vm) * (1.0 / 7.5)));
    const auto a_d = 1.4 / (1.0 + exp((-35.0 - Vm) * (1.0 / 13.0))) + 0.25;
    const auto b_d = 1.4 / (1.0 + exp((Vm + 5.0) * (1.0 / 5.0)));
    const auto c_d = 1.0 / (1.0 + exp((50.0 - Vm) * (1.0 / 20.0)));
    k.rtau[8] = 1.0 / (a_d * b_d + c_d);
    // f, f2 (share exp((V+30)/10))
    const auto e30 = exp((Vm + 30.0) * (1.0 / 10.0));
    k.inf[9] = 1.0 / (1.0 + exp((Vm + 20.0) * (1.0 / 7.0)));
    const auto v27 = Vm + 27.0;
    const auto a_f = 1102.5 * exp((v27 * v27) * (-1.0 / 225.0));
    const auto b_f = 200.0 / (1.0 + exp((13.0 - Vm) * (1.0 / 10.0)));
    const auto c_f = 180.0 / (1.0 + e30) + 20.0;
    k.rtau[9] = 1.0 / (a_f + b_f + c_f);
    k.inf[10] = 0.67 / (1.0 + exp((Vm + 35.0) * (1.0 / 7.0))) + 0.33;
    const auto v25 = Vm + 25.0;
    const auto a_f2 = 600.0 * exp((v25 * v25) * (-1.0 / 170.0));
    const auto b_f2 = 31.0 / (1.0 + exp((25.0 - Vm) * (1.0 / 10.0)));
    const auto c_f2 = 16.0 / (1.0 + e30);
    k.rtau[10] = 1.0 / (a_f2 + b_f2 + c_f2);
    return k;
  }

  template <class T, class Sink, class A0, class A1, class A2, class A3, class A4, class A5,
            class A6, class A7, class A8, class A9, class A10, class A11, class A12, class A13,
            class A14, class A15, class A16, class A17, class A18>
  IONIC_DEV static void rhs(const Params<T>& p, T stim, T diff, Sink& out, const A0& Vm,
                            const A1& cai, const A2& casr, const A3& cass, const A4& nai,
                            const A5& ki, const A6& gm, const A7& gh, const A8& gj,
                            const A9& gxr1, const A10& gxr2, const A11& gxs, const A12& gr,
                            const A13& gs, const A14& gd, const A15& gf, const A16& gf2,
                            const A17& gfc, const A18& rbar) {
    // rows eliminated first (gates, fCass, Rbar) are emitted before the core rows
    const auto k_casr = double(p.max_sr) - double(p.dsr) / (1.0 + double(p.EC2) / (casr * casr));
    const auto cass2 = cass * cass;
    const auto g = gate_kinetics<T>(Vm);
    out.template put<m>((g.inf[0] - gm) * g.rtau[0]);
    out.template put<h>((g.inf[1] - gh) * g.rtau[1]);
    out.template put<j>((g.inf[2] - gj) * g.rtau[2]);
    out.template put<xr1>((g.inf[3] - gxr1) * g.rtau[3]);
    out.template put<xr2>((g.inf[4] - gxr2) * g.rtau[4]);
    out.template put<xs>((g.inf[5] - gxs) * g.rtau[5]);
    out.template put<r>((g.inf[6] - gr) * g.rtau[6]);
    out.template put<s>((g.inf[7] - gs) * g.rtau[7]);
    out.template put<d>((g.inf[8] - gd) * g.rtau[8]);
    out.template put<f>((g.inf[9] - gf) * g.rtau[9]);
    out.template put<f2>((g.inf[10] - gf2) * g.rtau[10]);
    const auto qf = 1.0 + cass2 * 400.0;  // 1 + (CaSS/0.05)^2
    const auto rq = 1.0 / qf;
    out.template put<fCass>((0.6 * rq + 0.4 - gfc) / (80.0 * rq + 2.0));
    out.template put<Rbar>(-(double(p.k2p) * k_casr) * cass * rbar + double(p.k4) * (1.0 - rbar));

    // reversal potentials: RT/F log(out/in)
    const auto E_Na = double(p.RTF) * (double(p.logNao) - log(nai));
    const auto E_K = double(p.RTF) * (double(p.logKo) - log(ki));
    const auto E_Ca = double(p.halfRTF) * (double(p.logCao) - log(cai));
    const auto E_Ks = double(p.RTF) * (double(p.ks_num) - log(ki + double(p.p_KNa) * nai));

    const auto VmEK = Vm - E_K;
    const auto I_Na = double(p.G_Na) * (gm * gm * gm * gh * gj) * (Vm - E_Na);
    const auto I_to = double(p.G_to) * (gr * gs) * VmEK;
    const auto I_Kr = double(p.G_Krs) * (gxr1 * gxr2) * VmEK;
    const auto I_Ks = double(p.G_Ks) * (gxs * gxs) * (Vm - E_Ks);

    const auto a_K1 = 0.1 / (1.0 + exp(0.06 * (VmEK - 200.0)));
    const auto b_K1 = (3.0 * exp(0.0002 * (VmEK + 100.0)) + exp(0.1 * (VmEK - 10.0))) /
                      (1.0 + exp(-0.5 * VmEK));
    const auto I_K1 = double(p.G_K1s) * (a_K1 / (a_K1 + b_K1)) * VmEK;

    // L-type Ca: G 4F d f f2 fCass (0.25 CaSS e^{2u} - Cao) u / (e^{2u} - 1), u = (V-15) F/RT
    const auto u = (Vm - 15.0) * double(p.FRT);
    const auto e2u = exp(2.0 * u);
    const auto I_CaL = double(p.G_CaL4F) * (gd * gf * gf2 * gfc) *
                       ((0.25 * cass) * e2u - double(p.Cao)) * u_over_expm1_2u(u);

    const auto uv = Vm * double(p.FRT);
    const auto eg = exp(double(p.gamma) * uv);
    const auto eg1 = exp(double(p.gamma1) * uv);
    const auto I_NaCa = (double(p.naca_c1) * eg * (nai * nai * nai) - double(p.naca_c2) * eg1 * cai) /
                        (1.0 + double(p.k_sat) * eg1);
    const auto I_NaK = double(p.nak_c) * nai /
                       ((nai + double(p.Km_Na)) * (1.0 + 0.1245 * exp(-0.1 * uv) + 0.0353 * exp(-uv)));
    const auto I_pCa = double(p.G_pCa) * cai / (cai + double(p.K_pCa));
    const auto I_pK = double(p.G_pK) * VmEK / (1.0 + exp((25.0 - Vm) * (1.0 / 5.98)));
    const auto I_bNa = double(p.G_bNa) * (Vm - E_Na);
    const auto I_bCa = double(p.G_bCa) * (Vm - E_Ca);

    // calcium handling
    const auto k1 = double(p.k1p) / k_casr;
    const auto O = (k1 * cass2 * rbar) / (double(p.k3) + k1 * cass2);
    const auto I_rel = double(p.V_rel) * O * (casr - cass);
    const auto I_up = double(p.Vmax_up) / (1.0 + double(p.K_up2) / (cai * cai));
    const auto I_leak = double(p.V_leak) * (casr - cai);
    const auto I_xfer = double(p.V_xfer) * (cass - cai);

    const auto cb = cai + double(p.K_bufc);
    const auto beta_c = 1.0 / (1.0 + double(p.bc) / (cb * cb));
    const auto srb = casr + double(p.K_bufsr);
    const auto beta_sr = 1.0 / (1.0 + double(p.bsr) / (srb * srb));
    const auto ssb = cass + double(p.K_bufss);
    const auto beta_ss = 1.0 / (1.0 + double(p.bss) / (ssb * ssb));

    const auto I_ion = ((I_Na + I_K1) + (I_to + I_Kr) + (I_Ks + I_CaL)) + ((I_NaCa + I_NaK) + (I_pCa + I_pK)) +
                       (I_bNa + I_bCa);
    out.template put<V>((I_ion + double(stim)) * -1.0 + double(diff));
    out.template put<Cai>(beta_c * ((I_bCa + I_pCa - 2.0 * I_NaCa) * -double(p.halfcF_c) +
                                    (I_leak - I_up) * double(p.sr_c) + I_xfer));
    out.template put<CaSR>(beta_sr * (I_up - I_leak - I_rel));
    out.template put<CaSS>(beta_ss * (I_CaL * -double(p.caL_ss) + I_rel * double(p.sr_ss) -
                                      I_xfer * double(p.c_ss)));
    out.template put<Nai>((I_Na + I_bNa + 3.0 * I_NaK + 3.0 * I_NaCa) * -double(p.cF_c));
    out.template put<Ki>((I_K1 + I_to + I_Kr + I_Ks - 2.0 * I_NaK + I_pK + double(stim - diff)) *
                         -double(p.cF_c));

  }

  template <class T>
  IONIC_DEV static void steady_gates(const Params<T>&, T* x) {
    const auto k = gate_kinetics<T>(plain(x[V]));
    constexpr int gates[11] = {m, h, j, xr1, xr2, xs, r, s, d, f, f2};
    for (int i = 0; i < 11; ++i) x[gates[i]] = k.inf[i].v;
    const T q = T(1) + x[CaSS] * x[CaSS] * T(400);
    x[fCass] = T(0.6) / q + T(0.4);
  }
};

}  // namespace ionic
