// Static sparse elimination onto the membrane potential: the local block of
// the partitioned step's global systems.
//
// With the parabolic term kept implicit (paper section 3.3.2, Algorithm 2 and
// the solver paragraph after it; section 3.3.1, equation rb_system), a stage
// or correction system of the ROS2 + SDC step is
//     (B + c L) x = b,   B = blockdiag(I - c J_cell),  L = M_L^{-1} A_i on v,
// global because L couples the v of neighbouring vertices, while every other
// state couples only within its own vertex.  Eliminating, per vertex, every
// state but v from its block leaves one equation per vertex for v,
//     S dv + c (L dv) = r,
// with S and r the Schur complement and the reduced right-hand side.  A Krylov
// method solves that system over the grid; each vertex then recovers its
// other states from dv by back substitution.  This is exact block elimination
// of the same linear system.
//
// SinkSchur eliminates like SinkElim (sparse_solve.h) -- the gating rows while
// the model emits them, then the dense core -- with the core's order changed
// so that V is the last pivot: after the forward pass a[0][0] is S and b[0]
// is r.  The fill of that order is computed at compile time.
#pragma once

#include "dual.h"

namespace ionic {

template <class Model>
struct SchurElim {
  static constexpr int N = Model::N;
  static constexpr int NC = Model::N64;  // core states [0, NC); V = 0 is eliminated last
  static constexpr int NG = N - NC;
  static constexpr uint32_t G_MASK = ((N >= 32) ? 0xFFFFFFFFu : ((1u << N) - 1u)) & ~((1u << NC) - 1u);
  // elimination position -> state: the gating states, core states 1..NC-1, then V
  static constexpr int at(int k) { return k < NG ? NC + k : (k < N - 1 ? k - NG + 1 : 0); }
  // position of core state i in the core order (0..NC-1, V last)
  static constexpr int core_pos(int i) { return i == 0 ? NC - 1 : i - 1; }

  struct Pat {
    bool p[N][N];
  };
  static constexpr Pat filled() {
    Pat P{};
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < N; ++k) P.p[i][k] = (i == k) || has(Model::ROW[i], k);
    for (int kk = 0; kk < N; ++kk) {
      const int piv = at(kk);
      for (int ii = kk + 1; ii < N; ++ii) {
        const int i = at(ii);
        if (!P.p[i][piv]) continue;
        for (int jj = kk + 1; jj < N; ++jj) {
          const int jx = at(jj);
          if (P.p[piv][jx]) P.p[i][jx] = true;
        }
      }
    }
    return P;
  }
  static constexpr Pat FILL = filled();
};

// Receives F and J rows in emission order; b_i = bfn(i, F_i).  reduce() gives
// the Schur complement onto V and the reduced right-hand side; expand() the
// full solution from the value of V.
template <class Model, class T, class BFn>
struct SinkSchur {
  using E = SchurElim<Model>;
  static constexpr int N = Model::N;
  static constexpr int NC = E::NC;

  T c;
  BFn bfn;
  T f[N];       // F at the evaluation point
  T gd[N];      // gating rows: b_g / pivot
  T gc[N][NC];  // gating rows: a_gk / pivot for core columns k
  T a[NC][NC];  // core block on the fill pattern; multipliers below the diagonal
  T b[NC];
  T inv[NC];

  IONIC_DEV SinkSchur(T cc, BFn fn) : c(cc), bfn(fn) {}

  template <int i, uint32_t M>
  IONIC_DEV T jac(const D<T, M>& x) const {
    if constexpr (has(M, i))
      return x.template d<i>();
    else
      return T(0);
  }

  template <int i, uint32_t M>
  IONIC_DEV void put(const D<T, M>& x) {
    static_assert((M & ~Model::ROW[i]) == 0, "row has an entry outside its declared pattern");
    f[i] = x.v;
    const T bi = bfn(std::integral_constant<int, i>{}, x.v);
    if constexpr (i >= NC) {
      const T iv = f_rcp(T(1) - c * jac<i>(x));
      gd[i] = bi * iv;
      for_bits<Model::ROW[i] & ~bit(i)>([&](auto K) {
        constexpr int k = K;
        gc[i][k] = -(c * jac<k>(x)) * iv;
      });
    } else {
      static_for<NC>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == i)
          a[i][k] = T(1) - c * jac<k>(x);
        else if constexpr (has(Model::ROW[i], k))
          a[i][k] = -c * jac<k>(x);
        else if constexpr (E::FILL.p[i][k])
          a[i][k] = T(0);
      });
      T bb = bi;
      for_bits<Model::ROW[i] & E::G_MASK>([&](auto G) {
        constexpr int g = G;
        const T aig = -c * jac<g>(x);
        bb -= aig * gd[g];
        for_bits<Model::ROW[g] & ~bit(g)>([&](auto K) {
          constexpr int k = K;
          a[i][k] -= aig * gc[g][k];
        });
      });
      b[i] = bb;
    }
  }

  // forward elimination of the core in the order 1..NC-1, V last
  IONIC_DEV void reduce(T& S, T& r) {
    static_for<NC - 1>([&](auto PP) {
      constexpr int p = PP + 1;
      inv[p] = f_rcp(a[p][p]);
      static_for<NC>([&](auto I) {
        constexpr int i = I;
        if constexpr (E::core_pos(i) > E::core_pos(p) && E::FILL.p[i][p]) {
          const T l = a[i][p] * inv[p];
          static_for<NC>([&](auto J) {
            constexpr int jx = J;
            if constexpr (E::core_pos(jx) > E::core_pos(p) && E::FILL.p[p][jx]) a[i][jx] -= l * a[p][jx];
          });
          b[i] -= l * b[p];
        }
      });
    });
    S = a[0][0];
    r = b[0];
  }

  // after reduce(): every state's solution from the value of V
  IONIC_DEV void expand(T dV, T (&delta)[N]) {
    delta[0] = dV;
    static_for<NC - 1>([&](auto PR) {
      constexpr int p = NC - 1 - PR;  // core positions from last-but-V down to the first
      T acc = b[p];
      static_for<NC>([&](auto J) {
        constexpr int jx = J;
        if constexpr (E::core_pos(jx) > E::core_pos(p) && E::FILL.p[p][jx]) acc -= a[p][jx] * delta[jx];
      });
      delta[p] = acc * inv[p];
    });
    static_for<N - NC>([&](auto GG) {
      constexpr int g = NC + GG;
      T acc = gd[g];
      for_bits<Model::ROW[g] & ~bit(g)>([&](auto K) {
        constexpr int k = K;
        acc -= gc[g][k] * delta[k];
      });
      delta[g] = acc;
    });
  }
};

}  // namespace ionic
