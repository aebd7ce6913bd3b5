// Static sparse elimination of the local Newton / SDC system (I - dtau J) x = b.
//
// With the diffusion term fixed the paper's block-Jacobi BiCGSTAB (section
// 3.3.2, solver paragraph after Algorithm 2) is exact in one step: the system
// is block diagonal with one small block per vertex.  Each block is solved
// here directly, by Gaussian elimination whose every operation is decided at
// compile time from the model's Jacobian pattern (CTSM): the gate rows, which
// touch only V and themselves (TT06 also fCass and Rbar), are eliminated first
// and produce no new nonzeros outside the V column; the dense core left over
// (LR91: {V, Cai}; TT06: {V, Cai, CaSR, CaSS, Nai, Ki}) is eliminated without
// pivoting.  Pivots are 1 + dtau / tau_gate for the gates, so no pivoting is
// needed there; the core is diagonally dominant for the step sizes used.
// Symbolic fill-in is computed by a constexpr function, so the unrolled code
// touches structural nonzeros only.
#pragma once

#include "dual.h"

namespace ionic {

template <class Model>
struct Elim {
  static constexpr int N = Model::N;
  static constexpr int NG = N - Model::N64;  // rows eliminated first
  // elimination position -> state index
  static constexpr int at(int k) { return k < NG ? Model::N64 + k : k - NG; }

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

  static constexpr int nnz_filled() {
    int c = 0;
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < N; ++k) c += FILL.p[i][k] ? 1 : 0;
    return c;
  }
};

// Zero the fill-in positions (in FILL but outside the declared rows), which the
// Jacobian writer never touches.
template <class Model, class T>
IONIC_DEV void zero_fill(T (&a)[Model::N][Model::N]) {
  using E = Elim<Model>;
  static_for<Model::N>([&](auto I) {
    static_for<Model::N>([&](auto K) {
      constexpr int i = I, k = K;
      if constexpr (E::FILL.p[i][k] && i != k && !has(Model::ROW[i], k)) a[i][k] = T(0);
    });
  });
}

// Solve a x = b in place (x returned in b).  Only entries of Elim<Model>::FILL are
// read; the declared pattern plus the diagonal must have been written and the
// fill-in positions cleared with zero_fill.
template <class Model, class T>
IONIC_DEV void sparse_solve(T (&a)[Model::N][Model::N], T (&b)[Model::N]) {
  using E = Elim<Model>;
  constexpr int N = Model::N;
  T inv[N];
  static_for<N>([&](auto K) {
    constexpr int p = E::at(K);
    inv[p] = f_rcp(a[p][p]);
    static_for<N>([&](auto II) {
      if constexpr (II > K) {
        constexpr int i = E::at(II);
        if constexpr (E::FILL.p[i][p]) {
          const T l = a[i][p] * inv[p];
          static_for<N>([&](auto JJ) {
            if constexpr (JJ > K) {
              constexpr int jx = E::at(JJ);
              if constexpr (E::FILL.p[p][jx]) a[i][jx] -= l * a[p][jx];
            }
          });
          b[i] -= l * b[p];
        }
      }
    });
  });
  static_for<N>([&](auto KR) {
    constexpr int K = N - 1 - KR;
    constexpr int p = E::at(K);
    T acc = b[p];
    static_for<N>([&](auto JJ) {
      if constexpr (JJ > K) {
        constexpr int jx = E::at(JJ);
        if constexpr (E::FILL.p[p][jx]) acc -= a[p][jx] * b[jx];
      }
    });
    b[p] = acc * inv[p];
  });
}

}  // namespace ionic
