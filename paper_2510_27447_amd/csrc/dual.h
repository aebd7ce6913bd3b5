// Compile-time sparse forward-mode dual numbers for the device models.
//
// The paper's CTSM technique (section 3.3.2) stores each local block of the
// Jacobian with a sparsity fixed at compile time.  Here the sparsity is a
// template argument: D<T, Mask> carries a value and the partial derivatives
// with respect to the states whose bits are set in Mask, packed densely
// (popcount(Mask) entries).  Every operation combines the masks of its
// operands at compile time, so a gate that depends on V only carries one
// partial, and no arithmetic is ever spent on a structural zero.  With every
// function force-inlined the packed arrays become plain registers.
//
// A model is written once against these types.  Evaluating F alone seeds
// every state as D<T, 0> (no partials); evaluating F and J seeds state i as
// D<T, 1 << i>.  Plain double literals are converted to T inside the
// operators, so float evaluation never silently widens to double.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#define IONIC_DEV __device__ __forceinline__

namespace ionic {

// ---- compile-time loops -----------------------------------------------------
template <class F, int... I>
IONIC_DEV void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
IONIC_DEV void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int popc(uint32_t m) { return __builtin_popcount(m); }
constexpr bool has(uint32_t m, int i) { return (m >> i) & 1u; }
constexpr int rank(uint32_t m, int i) { return __builtin_popcount(m & ((1u << i) - 1u)); }
constexpr uint32_t bit(int i) { return 1u << i; }

template <uint32_t M, class F>
IONIC_DEV void for_bits(F&& f) {
  static_for<32>([&](auto I) {
    if constexpr (has(M, I)) f(I);
  });
}

// ---- precision-specific elementary functions ----------------------------------
// double: the device math library (about 1 ulp); reciprocals from the hardware
//         estimate refined by two Newton-Raphson steps (within about 1 ulp, finite
//         non-zero arguments), instead of a correctly rounded division sequence.
// float:  hardware transcendentals (v_exp_f32 / v_log_f32 / v_rcp_f32).
IONIC_DEV double f_exp(double x) { return exp(x); }
IONIC_DEV double f_expm1(double x) { return expm1(x); }
IONIC_DEV double f_log(double x) { return log(x); }
IONIC_DEV double f_sqrt(double x) { return sqrt(x); }
IONIC_DEV double f_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
IONIC_DEV float f_exp(float x) { return __expf(x); }
IONIC_DEV float f_expm1(float x) { return expm1f(x); }
IONIC_DEV float f_log(float x) { return __logf(x); }
IONIC_DEV float f_sqrt(float x) { return __builtin_sqrtf(x); }
IONIC_DEV float f_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Per-lane choice between two values that are both computed.  Written as a
// call, its arguments are evaluated before it, so the optimiser is left with a
// select; a conditional expression with a longer alternative is otherwise
// emitted as a branch around that alternative, which on the GPU is a divergent
// branch.  The step kernels keep no divergent branches in their per-step work
// (see sdc_kernel.h).
template <class T>
IONIC_DEV T pick(bool c, T a, T b) {
  return c ? a : b;
}

// ---- the dual type ------------------------------------------------------------
template <class T, uint32_t M>
struct D {
  static constexpr uint32_t mask = M;
  T v;
  T g[popc(M) > 0 ? popc(M) : 1];
  template <int i>
  IONIC_DEV T& d() {
    static_assert(has(M, i), "partial outside the mask");
    return g[rank(M, i)];
  }
  template <int i>
  IONIC_DEV const T& d() const {
    static_assert(has(M, i), "partial outside the mask");
    return g[rank(M, i)];
  }
};

template <class T>
IONIC_DEV D<T, 0> cst(double c) {
  D<T, 0> r;
  r.v = T(c);
  return r;
}

template <class T, int i>
IONIC_DEV D<T, (1u << i)> seed(T x) {
  D<T, (1u << i)> r;
  r.v = x;
  r.g[0] = T(1);
  return r;
}

template <class T>
IONIC_DEV D<T, 0> plain(T x) {
  D<T, 0> r;
  r.v = x;
  return r;
}

// r = ca * a + cb * b on the union of the masks (partials only).
template <class T, uint32_t A, uint32_t B, class FA, class FB, class FAB>
IONIC_DEV void combine(D<T, A | B>& r, const D<T, A>& a, const D<T, B>& b, FA fa, FB fb, FAB fab) {
  for_bits<A | B>([&](auto I) {
    constexpr int i = I;
    if constexpr (has(A, i) && has(B, i))
      r.template d<i>() = fab(a.template d<i>(), b.template d<i>());
    else if constexpr (has(A, i))
      r.template d<i>() = fa(a.template d<i>());
    else
      r.template d<i>() = fb(b.template d<i>());
  });
}

template <class T, uint32_t A, class F>
IONIC_DEV D<T, A> map_partials(const D<T, A>& a, T value, F f) {
  D<T, A> r;
  r.v = value;
  for_bits<A>([&](auto I) {
    constexpr int i = I;
    r.template d<i>() = f(a.template d<i>());
  });
  return r;
}

// ---- arithmetic -------------------------------------------------------------------
template <class T, uint32_t A, uint32_t B>
IONIC_DEV D<T, A | B> operator+(const D<T, A>& a, const D<T, B>& b) {
  D<T, A | B> r;
  r.v = a.v + b.v;
  combine(r, a, b, [](T x) { return x; }, [](T y) { return y; }, [](T x, T y) { return x + y; });
  return r;
}

template <class T, uint32_t A, uint32_t B>
IONIC_DEV D<T, A | B> operator-(const D<T, A>& a, const D<T, B>& b) {
  D<T, A | B> r;
  r.v = a.v - b.v;
  combine(r, a, b, [](T x) { return x; }, [](T y) { return -y; }, [](T x, T y) { return x - y; });
  return r;
}

template <class T, uint32_t A>
IONIC_DEV D<T, A> operator-(const D<T, A>& a) {
  return map_partials(a, -a.v, [](T x) { return -x; });
}

template <class T, uint32_t A, uint32_t B>
IONIC_DEV D<T, A | B> operator*(const D<T, A>& a, const D<T, B>& b) {
  D<T, A | B> r;
  r.v = a.v * b.v;
  const T av = a.v, bv = b.v;
  combine(r, a, b, [&](T x) { return x * bv; }, [&](T y) { return av * y; },
          [&](T x, T y) { return x * bv + av * y; });
  return r;
}

// a / b via one reciprocal of b
template <class T, uint32_t A, uint32_t B>
IONIC_DEV D<T, A | B> operator/(const D<T, A>& a, const D<T, B>& b) {
  D<T, A | B> r;
  const T inv = f_rcp(b.v);
  const T q = a.v * inv;
  r.v = q;
  combine(r, a, b, [&](T x) { return x * inv; }, [&](T y) { return -(q * inv) * y; },
          [&](T x, T y) { return (x - q * y) * inv; });
  return r;
}

// mixed with double constants (converted to T)
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator+(const D<T, A>& a, double c) {
  D<T, A> r = a;
  r.v = a.v + T(c);
  return r;
}
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator+(double c, const D<T, A>& a) {
  return a + c;
}
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator-(const D<T, A>& a, double c) {
  D<T, A> r = a;
  r.v = a.v - T(c);
  return r;
}
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator-(double c, const D<T, A>& a) {
  return map_partials(a, T(c) - a.v, [](T x) { return -x; });
}
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator*(const D<T, A>& a, double c) {
  const T t = T(c);
  return map_partials(a, a.v * t, [&](T x) { return x * t; });
}
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator*(double c, const D<T, A>& a) {
  return a * c;
}
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator/(const D<T, A>& a, double c) {
  return a * (1.0 / c);
}
template <class T, uint32_t A>
IONIC_DEV D<T, A> operator/(double c, const D<T, A>& b) {
  const T inv = f_rcp(b.v);
  const T q = T(c) * inv;
  const T s = -q * inv;
  return map_partials(b, q, [&](T y) { return s * y; });
}

// ---- elementary functions -----------------------------------------------------------
template <class T, uint32_t A>
IONIC_DEV D<T, A> exp(const D<T, A>& a) {
  const T e = f_exp(a.v);
  return map_partials(a, e, [&](T x) { return e * x; });
}

template <class T, uint32_t A>
IONIC_DEV D<T, A> log(const D<T, A>& a) {
  const T inv = f_rcp(a.v);
  return map_partials(a, f_log(a.v), [&](T x) { return x * inv; });
}

template <class T, uint32_t A>
IONIC_DEV D<T, A> sqrt(const D<T, A>& a) {
  const T s = f_sqrt(a.v);
  const T h = T(0.5) * f_rcp(s);
  return map_partials(a, s, [&](T x) { return h * x; });
}

template <class T, uint32_t A>
IONIC_DEV D<T, A> sq(const D<T, A>& a) {
  return a * a;
}

// cond ? a : b, cond uniform over the partials (derivative of the branch taken)
template <class T, uint32_t A, uint32_t B>
IONIC_DEV D<T, A | B> select(bool cond, const D<T, A>& a, const D<T, B>& b) {
  D<T, A | B> r;
  r.v = pick(cond, a.v, b.v);
  combine(r, a, b, [&](T x) { return pick(cond, x, T(0)); },
          [&](T y) { return pick(cond, T(0), y); }, [&](T x, T y) { return pick(cond, x, y); });
  return r;
}

// x / (1 - exp(-a x)) with its removable singularity at x == 0 (limit 1/a, slope 1/2)
template <class T, uint32_t A>
IONIC_DEV D<T, A> x_over_1mexp(const D<T, A>& x, double a) {
  const bool zero = (x.v == T(0));
  const T xs = pick(zero, T(1), x.v);
  const T em = f_expm1(T(-a) * xs);  // exp(-a x) - 1
  const T den = -em;
  const T inv = f_rcp(den);
  const T val = pick(zero, T(1.0 / a), xs * inv);
  // d/dx [x / (1 - e^{-ax})] = (den - a x e^{-ax}) / den^2
  const T slope = pick(zero, T(0.5), (den - T(a) * xs * (em + T(1))) * inv * inv);
  return map_partials(x, val, [&](T g) { return slope * g; });
}

// (exp(a x) - 1) / x with its removable singularity at x == 0 (limit a, slope a^2/2)
template <class T, uint32_t A>
IONIC_DEV D<T, A> expm1_over_x(const D<T, A>& x, double a) {
  const bool zero = (x.v == T(0));
  const T xs = pick(zero, T(1), x.v);
  const T em = f_expm1(T(a) * xs);
  const T inv = f_rcp(xs);
  const T val = pick(zero, T(a), em * inv);
  // d/dx [(e^{ax} - 1)/x] = (a x e^{ax} - (e^{ax} - 1)) / x^2
  const T slope = pick(zero, T(0.5 * a * a), (T(a) * xs * (em + T(1)) - em) * inv * inv);
  return map_partials(x, val, [&](T g) { return slope * g; });
}

// u / (exp(2u) - 1) with its removable singularity at u == 0 (limit 1/2, slope -1/2)
template <class T, uint32_t A>
IONIC_DEV D<T, A> u_over_expm1_2u(const D<T, A>& u) {
  const bool zero = (u.v == T(0));
  const T us = pick(zero, T(1), u.v);
  const T em = f_expm1(T(2) * us);
  const T inv = f_rcp(em);
  const T val = pick(zero, T(0.5), us * inv);
  // d/du [u / (e^{2u} - 1)] = (em - 2u e^{2u}) / em^2
  const T slope = pick(zero, T(-0.5), (em - T(2) * us * (em + T(1))) * inv * inv);
  return map_partials(u, val, [&](T g) { return slope * g; });
}

}  // namespace ionic
