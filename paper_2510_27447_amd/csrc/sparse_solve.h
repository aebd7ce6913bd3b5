// Static sparse elimination of the local Newton / SDC system (I - dtau J) x = b.
//
// With the diffusion term fixed the paper's block-Jacobi BiCGSTAB (section
// 3.3.2, solver paragraph after Algorithm 2) is exact in one step: the system
// is block diagonal with one small block per vertex.  Each block is solved
// here directly, by Gaussian elimination whose every operation is decided at
// compile time from the model's Jacobian pattern (CTSM).  The states stored in
// fp32 under the mixed layout -- the gates, and for TT06 also fCass and Rbar --
// form the set G: each of their rows touches only itself and "core" states
// (LR91 {V, Cai}; TT06 {V, Cai, CaSR, CaSS, Nai, Ki}).  G rows are eliminated
// first; their pivots are 1 + dtau / tau, so no pivoting is needed, and they
// produce fill only inside the core.  The dense core is then eliminated
// without pivoting (diagonally dominant at the step sizes used).
//
// SinkElim performs the elimination while the model emits its rows: a G row
// leaves its right-hand side and its core coefficients divided by the pivot;
// a core row, when it arrives, folds every G column it touches into its core
// entries at once.  The Jacobian is therefore never held whole, only the G
// coefficients and the core block.  The model must emit all G rows before the
// core rows.
#pragma once

#include "dual.h"

namespace ionic {

template <class Model>
struct Elim {
  static constexpr int N = Model::N;
  static constexpr int NC = Model::N64;  // core states: [0, NC)
  static constexpr int NG = N - NC;      // rows eliminated first: [NC, N)
  static constexpr uint32_t G_MASK = ((N >= 32) ? 0xFFFFFFFFu : ((1u << N) - 1u)) & ~((1u << NC) - 1u);
  // elimination position -> state index
  static constexpr int at(int k) { return k < NG ? NC + k : k - NG; }

  static constexpr bool g_rows_touch_core_only() {
    for (int g = NC; g < N; ++g)
      if ((Model::ROW[g] & G_MASK) & ~(1u << g)) return false;
    return true;
  }
  static_assert(g_rows_touch_core_only(),
                "every row eliminated first may depend only on itself and core states");

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

// Receives the rows of F and J (value and partials) in emission order and
// solves (I - dtau J) delta = b with b_i = bfn(i, F_i).
template <class Model, class T, class BFn, bool Keep = false>
struct SinkElim {
  using E = Elim<Model>;
  static constexpr int N = Model::N;
  static constexpr int NC = E::NC;

  T dtau;
  BFn bfn;
  T f[N];          // F at the evaluation point
  T gd[N];         // G rows: b_g / pivot
  T gc[N][NC];     // G rows: a_gk / pivot for core columns k
  T a[NC][NC];     // core block (on the fill pattern); multipliers below the diagonal
  T b[NC];
  T ginv[N];       // Keep: G rows' 1 / pivot
  T ag[NC][N];     // Keep: core rows' G-column entries -dtau J_ig
  T pinv[NC];      // Keep: core 1 / pivot

  IONIC_DEV SinkElim(T dt, BFn fn) : dtau(dt), bfn(fn) {}

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
      const T inv = f_rcp(T(1) - dtau * jac<i>(x));
      if constexpr (Keep) ginv[i] = inv;
      gd[i] = bi * inv;
      for_bits<Model::ROW[i] & ~bit(i)>([&](auto K) {
        constexpr int k = K;
        gc[i][k] = -(dtau * jac<k>(x)) * inv;
      });
    } else {
      // core entries of row i, fill positions cleared
      static_for<NC>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == i)
          a[i][k] = T(1) - dtau * jac<k>(x);
        else if constexpr (has(Model::ROW[i], k))
          a[i][k] = -dtau * jac<k>(x);
        else if constexpr (E::FILL.p[i][k])
          a[i][k] = T(0);
      });
      T bb = bi;
      for_bits<Model::ROW[i] & E::G_MASK>([&](auto G) {
        constexpr int g = G;
        const T aig = -dtau * jac<g>(x);
        if constexpr (Keep) ag[i][g] = aig;
        bb -= aig * gd[g];
        for_bits<Model::ROW[g] & ~bit(g)>([&](auto K) {
          constexpr int k = K;
          a[i][k] -= aig * gc[g][k];
        });
      });
      b[i] = bb;
    }
  }

  // After all rows: eliminate the core, back-substitute, recover the G states.
  IONIC_DEV void solve(T (&delta)[N]) {
    T inv[NC];
    static_for<NC>([&](auto P) {
      constexpr int p = P;
      inv[p] = f_rcp(a[p][p]);
      static_for<NC>([&](auto I) {
        constexpr int i = I;
        if constexpr (i > p && E::FILL.p[i][p]) {
          const T l = a[i][p] * inv[p];
          if constexpr (Keep) a[i][p] = l;
          static_for<NC>([&](auto J) {
            constexpr int jx = J;
            if constexpr (jx > p && E::FILL.p[p][jx]) a[i][jx] -= l * a[p][jx];
          });
          b[i] -= l * b[p];
        }
      });
    });
    static_for<NC>([&](auto PR) {
      constexpr int p = NC - 1 - PR;
      T acc = b[p];
      static_for<NC>([&](auto J) {
        constexpr int jx = J;
        if constexpr (jx > p && E::FILL.p[p][jx]) acc -= a[p][jx] * delta[jx];
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
    if constexpr (Keep) static_for<NC>([&](auto P) { pinv[P] = inv[P]; });
  }

  // After solve(): the solution of the same system for another right-hand side.
  IONIC_DEV void resolve(const T (&rhs)[N], T (&delta)[N]) {
    static_assert(Keep, "resolve needs the factorisation kept");
    static_for<N - NC>([&](auto GG) {
      constexpr int g = NC + GG;
      gd[g] = rhs[g] * ginv[g];
    });
    T c[NC];
    static_for<NC>([&](auto I) {
      constexpr int i = I;
      T bb = rhs[i];
      for_bits<Model::ROW[i] & E::G_MASK>([&](auto G) {
        constexpr int g = G;
        bb -= ag[i][g] * gd[g];
      });
      c[i] = bb;
    });
    static_for<NC>([&](auto P) {
      constexpr int p = P;
      static_for<NC>([&](auto I) {
        constexpr int i = I;
        if constexpr (i > p && E::FILL.p[i][p]) c[i] -= a[i][p] * c[p];
      });
    });
    static_for<NC>([&](auto PR) {
      constexpr int p = NC - 1 - PR;
      T acc = c[p];
      static_for<NC>([&](auto J) {
        constexpr int jx = J;
        if constexpr (jx > p && E::FILL.p[p][jx]) acc -= a[p][jx] * delta[jx];
      });
      delta[p] = acc * pinv[p];
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

// ---- the core block alone --------------------------------------------------------
// The Rush-Larsen predictor holds the gating states and solves only for the
// core (states [0, NC)): (I - dtau J_cc) delta_c = b_c.  Its pattern is the
// core block of the model's rows with the fill of eliminating it in order.
template <class Model>
struct CoreElim {
  static constexpr int NC = Model::N64;
  struct Pat {
    bool p[NC][NC];
  };
  static constexpr Pat filled() {
    Pat P{};
    for (int i = 0; i < NC; ++i)
      for (int k = 0; k < NC; ++k) P.p[i][k] = (i == k) || has(Model::ROW[i], k);
    for (int p = 0; p < NC; ++p)
      for (int i = p + 1; i < NC; ++i) {
        if (!P.p[i][p]) continue;
        for (int j = p + 1; j < NC; ++j)
          if (P.p[p][j]) P.p[i][j] = true;
      }
    return P;
  }
  static constexpr Pat FILL = filled();
};

// Receives the rows of an evaluation seeded on the core states only and keeps
// the core rows: b_i = bfn(i, F_i) and the core block of I - dtau J.  The rows
// of the gating states are not used, so their arithmetic is dead code.
template <class Model, class T, class BFn>
struct SinkCore {
  using E = CoreElim<Model>;
  static constexpr int NC = E::NC;

  T dtau;
  BFn bfn;
  T a[NC][NC];
  T b[NC];

  IONIC_DEV SinkCore(T dt, BFn fn) : dtau(dt), bfn(fn) {}

  template <int i, uint32_t M>
  IONIC_DEV void put(const D<T, M>& x) {
    static_assert((M & ~Model::ROW[i]) == 0, "row has an entry outside its declared pattern");
    if constexpr (i < NC) {
      b[i] = bfn(std::integral_constant<int, i>{}, x.v);
      static_for<NC>([&](auto K) {
        constexpr int k = K;
        if constexpr (k == i) {
          if constexpr (has(M, k))
            a[i][k] = T(1) - dtau * x.template d<k>();
          else
            a[i][k] = T(1);
        } else if constexpr (has(M, k)) {
          a[i][k] = -dtau * x.template d<k>();
        } else if constexpr (E::FILL.p[i][k]) {
          a[i][k] = T(0);
        }
      });
    }
  }

  IONIC_DEV void solve(T (&delta)[NC]) {
    T inv[NC];
    static_for<NC>([&](auto P) {
      constexpr int p = P;
      inv[p] = f_rcp(a[p][p]);
      static_for<NC>([&](auto I) {
        constexpr int i = I;
        if constexpr (i > p && E::FILL.p[i][p]) {
          const T l = a[i][p] * inv[p];
          static_for<NC>([&](auto J) {
            constexpr int jx = J;
            if constexpr (jx > p && E::FILL.p[p][jx]) a[i][jx] -= l * a[p][jx];
          });
          b[i] -= l * b[p];
        }
      });
    });
    static_for<NC>([&](auto PR) {
      constexpr int p = NC - 1 - PR;
      T acc = b[p];
      static_for<NC>([&](auto J) {
        constexpr int jx = J;
        if constexpr (jx > p && E::FILL.p[p][jx]) acc -= a[p][jx] * delta[jx];
      });
      delta[p] = acc * inv[p];
    });
  }
};

}  // namespace ionic
