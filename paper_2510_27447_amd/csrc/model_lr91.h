// Luo-Rudy phase-1 ventricular model, device form (paper section 2, "LR91").
//
// Eight states: V, [Ca]_i and the Hodgkin-Huxley gates m, h, j, d, f, X with
// dk/dt = alpha_k(V)(1 - k) - beta_k(V) k.  Six currents
// I_ion = I_Na + I_si + I_K + I_K1 + I_Kp + I_b.  The paper prints the model
// only by reference; rate functions and constants are restated from the
// model's publication (Luo and Rudy, Circ. Res. 68, 1991).  Default
// parameters are the paper's modified conductances (section 4): G_si = 0.02,
// G_Na = 4.0, G_K = 0.423 (G_K replaces the whole 0.282 sqrt(K_o/5.4) factor).
// Units: mV, ms, uA/cm^2 with C_m = 1 uF/cm^2, mM.
//
// Compile-time Jacobian pattern (CTSM): row V is full, each gate row touches
// {V, itself}, row Cai touches {V, d, f, Cai}: 24 of 64 entries.
#pragma once

#include "dual.h"

namespace ionic {

struct LR91 {
  static constexpr int N = 8;
  static constexpr int N64 = 2;  // V and Cai stay double in the mixed layout
  enum : int { V = 0, Cai, m, h, j, d, f, X };

  static constexpr uint32_t ROW[N] = {
      0xFFu,                                  // V
      bit(V) | bit(d) | bit(f) | bit(Cai),    // Cai
      bit(V) | bit(m), bit(V) | bit(h), bit(V) | bit(j),
      bit(V) | bit(d), bit(V) | bit(f), bit(V) | bit(X)};

  // Newton stop scale s_i = max(|Y_i|, SCALE_i)
  static constexpr double SCALE[N] = {100.0, 1e-4, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};

  // Resting state loaded by ionic_init when no initial state is given: the
  // solution X* of F(X) = 0 (no stimulus, no diffusion current), found by
  // Newton's method from V = -84 mV, [Ca]_i = 2e-4 mM and every gate at its
  // steady state at that V (the gate entries below are replaced by it).
  static constexpr bool REST_BY_NEWTON = true;
  static constexpr double REST_GUESS[N] = {-84.0, 2e-4, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

  // Overridable raw parameters, in this order.
  static constexpr int N_PARAMS = 15;
  static constexpr const char* PARAM_NAMES[N_PARAMS] = {
      "G_Na", "G_si", "G_K", "G_K1", "G_Kp", "G_b", "E_b", "Nao", "Nai", "Ko", "Ki",
      "PR_NaK", "R", "T", "F"};
  static constexpr double PARAM_DEFAULTS[N_PARAMS] = {
      4.0, 0.02, 0.423, 0.6047, 0.0183, 0.03921, -59.87, 140.0, 18.0, 5.4, 145.0,
      0.01833, 8314.0, 310.0, 96485.0};

  template <class T>
  struct Params {
    T G_Na, G_si, G_K, G_K1s, G_Kp, G_b, E_b, E_Na, E_K, E_K1;
  };

  // Host: derived constants (reversal potentials with fixed Na/K concentrations).
  template <class T>
  static Params<T> derive(const double* raw) {
    const double G_Na = raw[0], G_si = raw[1], G_K = raw[2], G_K1 = raw[3], G_Kp = raw[4];
    const double G_b = raw[5], E_b = raw[6], Nao = raw[7], Nai = raw[8], Ko = raw[9];
    const double Ki = raw[10], PR = raw[11], R = raw[12], Tk = raw[13], F = raw[14];
    const double RTF = R * Tk / F;
    Params<T> p;
    p.G_Na = T(G_Na);
    p.G_si = T(G_si);
    p.G_K = T(G_K);
    p.G_K1s = T(G_K1 * std::sqrt(Ko / 5.4));
    p.G_Kp = T(G_Kp);
    p.G_b = T(G_b);
    p.E_b = T(E_b);
    p.E_Na = T(RTF * std::log(Nao / Nai));
    p.E_K = T(RTF * std::log((Ko + PR * Nao) / (Ki + PR * Nai)));
    p.E_K1 = T(RTF * std::log(Ko / Ki));
    return p;
  }

  // alpha_k, beta_k of the six gates at V (V >= -40 takes the upper branch).
  template <class T, class TV>
  struct Rates {
    decltype(TV{} * 1.0) am, bm, ah, bh, aj, bj, ad, bd, af, bf, aX, bX;
  };

  template <class T, class TV>
  IONIC_DEV static Rates<T, TV> rates(const TV& Vm) {
    Rates<T, TV> r;
    const bool hi = Vm.v >= T(-40);
    const auto zero = Vm * 0.0;
    r.am = 0.32 * x_over_1mexp(Vm + 47.13, 0.1);
    r.bm = 0.08 * exp(Vm * (-1.0 / 11.0));
    r.ah = select(hi, zero, 0.135 * exp((80.0 + Vm) * (-1.0 / 6.8)));
    r.bh = select(hi, 1.0 / (0.13 * (1.0 + exp((Vm + 10.66) * (-1.0 / 11.1)))),
                  3.56 * exp(0.079 * Vm) + 3.1e5 * exp(0.35 * Vm));
    r.aj = select(hi, zero,
                  (-1.2714e5 * exp(0.2444 * Vm) - 3.474e-5 * exp(-0.04391 * Vm)) * (Vm + 37.78) /
                      (1.0 + exp(0.311 * (Vm + 79.23))));
    r.bj = select(hi, 0.3 * exp(-2.535e-7 * Vm) / (1.0 + exp(-0.1 * (Vm + 32.0))),
                  0.1212 * exp(-0.01052 * Vm) / (1.0 + exp(-0.1378 * (Vm + 40.14))));
    r.ad = 0.095 * exp(-0.01 * (Vm - 5.0)) / (1.0 + exp(-0.072 * (Vm - 5.0)));
    r.bd = 0.07 * exp(-0.017 * (Vm + 44.0)) / (1.0 + exp(0.05 * (Vm + 44.0)));
    r.af = 0.012 * exp(-0.008 * (Vm + 28.0)) / (1.0 + exp(0.15 * (Vm + 28.0)));
    r.bf = 0.0065 * exp(-0.02 * (Vm + 30.0)) / (1.0 + exp(-0.2 * (Vm + 30.0)));
    r.aX = 0.0005 * exp(0.083 * (Vm + 50.0)) / (1.0 + exp(0.057 * (Vm + 50.0)));
    r.bX = 0.0013 * exp(-0.06 * (Vm + 20.0)) / (1.0 + exp(-0.04 * (Vm + 20.0)));
    return r;
  }

  // F(X): writes row i through out.template put<i>(value_with_partials).
  template <class T, class Sink, class A0, class A1, class A2, class A3, class A4, class A5,
            class A6, class A7>
  IONIC_DEV static void rhs(const Params<T>& p, T stim, T diff, Sink& out, const A0& Vm,
                            const A1& Ca, const A2& gm, const A3& gh, const A4& gj, const A5& gd,
                            const A6& gf, const A7& gX) {
    // gate rows (eliminated first) are emitted before the V and Cai rows
    const auto r = rates<T>(Vm);
    out.template put<m>(r.am * (1.0 - gm) - r.bm * gm);
    out.template put<h>(r.ah * (1.0 - gh) - r.bh * gh);
    out.template put<j>(r.aj * (1.0 - gj) - r.bj * gj);
    out.template put<d>(r.ad * (1.0 - gd) - r.bd * gd);
    out.template put<f>(r.af * (1.0 - gf) - r.bf * gf);
    out.template put<X>(r.aX * (1.0 - gX) - r.bX * gX);
    const auto I_Na = p.G_Na * (gm * gm * gm * gh * gj) * (Vm - double(p.E_Na));
    const auto E_si = 7.7 - 13.0287 * log(Ca);
    const auto I_si = p.G_si * (gd * gf) * (Vm - E_si);
    const bool above = Vm.v > T(-100);
    const auto Xi = select(above,
                           2.837 * expm1_over_x(Vm + 77.0, 0.04) * exp(-0.04 * (Vm + 35.0)),
                           Vm * 0.0 + 1.0);
    const auto I_K = p.G_K * gX * Xi * (Vm - double(p.E_K));
    const auto dK1 = Vm - double(p.E_K1);
    const auto a_K1 = 1.02 / (1.0 + exp(0.2385 * (dK1 - 59.215)));
    const auto b_K1 = (0.49124 * exp(0.08032 * (dK1 + 5.476)) + exp(0.06175 * (dK1 - 594.31))) /
                      (1.0 + exp(-0.5143 * (dK1 + 4.753)));
    const auto I_K1 = p.G_K1s * (a_K1 / (a_K1 + b_K1)) * dK1;
    const auto Kp = 1.0 / (1.0 + exp((7.488 - Vm) * (1.0 / 5.98)));
    const auto I_Kp = p.G_Kp * Kp * dK1;
    const auto I_b = p.G_b * (Vm - double(p.E_b));

    out.template put<V>(((((I_Na + I_si) + I_K) + I_K1) + I_Kp + I_b + double(stim)) * -1.0 +
                        double(diff));
    out.template put<Cai>(-1e-4 * I_si + 0.07 * (1e-4 - Ca));
  }

  // Gates at their steady state alpha / (alpha + beta) for the current V.
  template <class T>
  IONIC_DEV static void steady_gates(const Params<T>&, T* x) {
    const auto r = rates<T>(plain(x[V]));
    x[m] = (r.am / (r.am + r.bm)).v;
    x[h] = (r.ah / (r.ah + r.bh)).v;
    x[j] = (r.aj / (r.aj + r.bj)).v;
    x[d] = (r.ad / (r.ad + r.bd)).v;
    x[f] = (r.af / (r.af + r.bf)).v;
    x[X] = (r.aX / (r.aX + r.bX)).v;
  }
};

}  // namespace ionic
