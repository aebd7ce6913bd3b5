// Scalar test problems with closed-form solutions, used to check the SDC
// machinery on the device against textbook results (backward-Euler products,
// Lobatto IIIA / Pade limits, observed order).  Not part of the paper.
//   TestLinear   y' = lam * y + b + I_diff
//   TestLogistic y' = rate * y * (1 - y) + I_diff
#pragma once

#include "dual.h"

namespace ionic {

struct TestLinear {
  static constexpr int N = 1;
  static constexpr int N64 = 1;
  static constexpr uint32_t ROW[N] = {1u};
  static constexpr double SCALE[N] = {1.0};
  static constexpr bool REST_BY_NEWTON = false;  // y = 0 when no initial state is given
  static constexpr double REST_GUESS[N] = {0.0};
  static constexpr int N_PARAMS = 2;
  static constexpr const char* PARAM_NAMES[N_PARAMS] = {"lam", "b"};
  static constexpr double PARAM_DEFAULTS[N_PARAMS] = {-1.0, 0.0};
  template <class T>
  struct Params {
    T lam, b;
  };
  template <class T>
  static Params<T> derive(const double* q) {
    return Params<T>{T(q[0]), T(q[1])};
  }
  template <class T, class Sink, class A0>
  IONIC_DEV static void rhs(const Params<T>& p, T, T diff, Sink& out, const A0& y) {
    out.template put<0>(double(p.lam) * y + double(p.b + diff));
  }
  template <class T>
  IONIC_DEV static void steady_gates(const Params<T>&, T*) {}
};

struct TestLogistic {
  static constexpr int N = 1;
  static constexpr int N64 = 1;
  static constexpr uint32_t ROW[N] = {1u};
  static constexpr double SCALE[N] = {1.0};
  static constexpr bool REST_BY_NEWTON = false;  // y = 0 when no initial state is given
  static constexpr double REST_GUESS[N] = {0.0};
  static constexpr int N_PARAMS = 1;
  static constexpr const char* PARAM_NAMES[N_PARAMS] = {"rate"};
  static constexpr double PARAM_DEFAULTS[N_PARAMS] = {1.0};
  template <class T>
  struct Params {
    T rate;
  };
  template <class T>
  static Params<T> derive(const double* q) {
    return Params<T>{T(q[0])};
  }
  template <class T, class Sink, class A0>
  IONIC_DEV static void rhs(const Params<T>& p, T, T diff, Sink& out, const A0& y) {
    out.template put<0>(double(p.rate) * y * (1.0 - y) + double(diff));
  }
  template <class T>
  IONIC_DEV static void steady_gates(const Params<T>&, T*) {}
};

}  // namespace ionic
