// Fused reaction + SDC kernel (paper section 3.3.2, equations genODE,
// picard_form, residual, sdc_ode, sdc), one vertex per lane.
//
// Per time step and vertex, entirely in registers:
//   predictor   X_0 = X_n; on each Gauss-Lobatto sub-interval m either
//               (Newton) backward Euler Y - X_m - dtau_m F(Y) = 0 by local
//               Newton with the exact sparse Jacobian; the lane stops when
//               max_i |delta_i| / max(|Y_i|, scale_i) <= tol (>= 1 iteration,
//               <= maxit); the wave runs until its last lane stops; or
//               (ROS2) one step of the two-stage Rosenbrock method of
//               section 3.3.1 (equation rb_system, gamma = 1 + 1/sqrt(2)):
//               one F+J evaluation and elimination at X_m, one F evaluation at
//               X_m + k_1/gamma and a second solve with the kept
//               factorisation; the embedded solution X_m + k_1/gamma gives the
//               scaled error estimate used for step-size control; or
//               (Rush-Larsen) exponential steps g + dtau F_g phi(dtau J_gg)
//               for the gating states at frozen X_m (one evaluation seeded
//               on the gating states), then backward Euler on the core by
//               local Newton with the gates held, each iteration an
//               evaluation seeded on the core only and a dense core solve;
//   corrections K times: F at every node, quadrature Q_m = sum_j S_mj dt F_j,
//               then node by node r = X^{k+1}_m - X^k_{m+1} + Q_m and
//               (I - dtau_m J(X^k_{m+1})) delta = r, X^{k+1}_{m+1} += delta
//               (the linearised correction of equation sdc, generalised from
//               the trapezoid to M nodes);
//   X_{n+1} = X_{M-1}.
// The time loop runs inside the kernel, so HBM sees one read and one write of
// the state per launch.  The stimulus is constant over a step and applied iff
// t_on <= t0 + (n + 1/2) dt < t_off.
//
// Precision policies: Fp64 evaluates F, J and the solve in double.  Mixed
// evaluates them in float and keeps the first N64 states (V and the
// intracellular concentrations), the residuals and the quadrature in double;
// the other states are stored and updated in float.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dual.h"
#include "sparse_solve.h"

namespace ionic {

constexpr int kMaxNodes = 5;
constexpr int kPredNewton = 0;
constexpr int kPredRos2 = 1;
constexpr int kPredRushLarsen = 2;

// ROS2 coefficients in the form of equation rb_system multiplied through by
// tau * gamma:  (I - gamma tau J) k_1 = gamma tau F(X),
//               (I - gamma tau J) k_2 = gamma tau F(X + k_1 / gamma) - 2 k_1,
//               X_new = X + 3/(2 gamma) k_1 + 1/(2 gamma) k_2,
//               X_hat = X + k_1 / gamma,  X_new - X_hat = (k_1 + k_2) / (2 gamma).
constexpr double kRosGamma = 1.70710678118654752440;  // 1 + 1/sqrt(2)
constexpr double kRosA21 = 0.58578643762690495120;    // 1/gamma = 2 - sqrt(2)
constexpr double kRosM1 = 0.87867965644035742680;     // 3/(2 gamma)
constexpr double kRosM2 = 0.29289321881345247560;     // 1/(2 gamma)
constexpr int kMaxBatch = 24;
constexpr int kBlock = 64;  // one wavefront per workgroup

// Statistics and the adaptive error maximum are reduced per wave and then
// added atomically into one of kSlots cache-line slots, slot = workgroup mod
// kSlots.  Workgroups are dealt to the XCDs round robin, so each slot is only
// touched from one XCD, and no single address takes one atomic per wave (on a
// 1e6-vertex launch that is 15,625 waves, which serialised on one address
// cost about a millisecond).  The host and the control kernel fold the slots.
constexpr int kSlots = 64;

struct alignas(128) DevStats {
  unsigned long long vertex_steps;
  unsigned long long newton_iters;
  unsigned long long newton_solves;
  unsigned long long nonconverged;
  unsigned long long nonfinite;
  unsigned int it_max;
  unsigned int pad;
};

// Largest scaled error of the lanes of one slot, as the bits of a double >= 0
// (the bit patterns of non-negative doubles order like the values).
struct alignas(128) ErrSlot {
  unsigned long long bits;
};

// Step-size control block of one adaptive run (one simulation per launch).
// The step kernel reads the pending attempt (t, tau, which buffer holds the
// state) and raises its error slot to the largest lane error; the control
// kernel then folds the slots, accepts or rejects the attempt and plans the
// next one.
struct AdaptCtl {
  double t, tau, dt_try, b;     // time, step of the pending attempt, proposed step, its breakpoint
  double t_end, dt_max, tol, dt_min, t_on, t_off;
  double err_last;
  long long accepted, rejected, attempts, max_attempts;
  int cur;                      // 0: the state is in the simulation's buffer, 1: in the work buffer
  int done, failed, hit;
};

struct SimDesc {
  void* state;             // SoA planes
  long long n;             // vertices
  long long stride;        // elements per plane
  const double* i_stim;    // amplitude per vertex or null
  const double* i_diff;    // fixed diffusion current per vertex or null
  double t0, dt, t_on, t_off;
  long long step_offset;   // steps already taken from t0
  int n_steps, n_sweeps;
  DevStats* stats;         // kSlots slots
  const int* order;        // vertex advanced by each lane slot (a permutation of [0, n)) or null
  int first_block;         // first workgroup of this simulation in the launch
  int pad;
};

template <class P>
struct LaunchArgs {
  P params;
  double S[kMaxNodes - 1][kMaxNodes];  // integration matrix on the unit interval
  double dc[kMaxNodes - 1];            // node spacing on the unit interval
  double tol;
  int maxit;
  int n_sims;
  AdaptCtl* ctl;     // adaptive run (ROS2 kernels, one simulation) or null
  ErrSlot* err;      // adaptive run: kSlots error slots
  void* state_alt;   // adaptive run: the second state buffer
  SimDesc sims[kMaxBatch];
};

struct Fp64 {
  using TE = double;
  static constexpr bool mixed = false;
};
struct Mixed {
  using TE = float;
  static constexpr bool mixed = true;
};

// ---- sinks receiving the model's rows --------------------------------------------
template <class Model, class T>
struct SinkF {
  T* f;
  template <int i, uint32_t M>
  IONIC_DEV void put(const D<T, M>& x) {
    static_assert((M & ~Model::ROW[i]) == 0, "F_i depends on a state outside its declared row");
    f[i] = x.v;
  }
};

// F of every row and the diagonal Jacobian entry of the gating rows (the
// evaluation is seeded on the gating states only)
template <class Model, class T>
struct SinkGateStep {
  T f[Model::N];
  T d[Model::N];
  template <int i, uint32_t M>
  IONIC_DEV void put(const D<T, M>& x) {
    static_assert((M & ~Model::ROW[i]) == 0, "F_i depends on a state outside its declared row");
    f[i] = x.v;
    if constexpr (i >= Model::N64) {
      if constexpr (has(M, i))
        d[i] = x.template d<i>();
      else
        d[i] = T(0);
    }
  }
};

// dense F and J (debug entry point)
template <class Model, class T>
struct SinkDense {
  T* f;
  T* J;
  template <int i, uint32_t M>
  IONIC_DEV void put(const D<T, M>& x) {
    f[i] = x.v;
    for_bits<M>([&](auto K) {
      constexpr int k = K;
      J[i * Model::N + k] = x.template d<k>();
    });
  }
};

template <class Model, class Prec>
struct Layout {
  using TE = typename Prec::TE;
  static constexpr int N = Model::N;
  static constexpr int N64 = Prec::mixed ? Model::N64 : N;  // states held in double
  static constexpr int N32 = N - N64;

  struct Node {
    double x64[N64];
    float x32[N32 > 0 ? N32 : 1];
  };
  template <int i>
  IONIC_DEV static auto& at(Node& n) {
    if constexpr (i < N64)
      return n.x64[i];
    else
      return n.x32[i - N64];
  }
  template <int i>
  IONIC_DEV static const auto& at(const Node& n) {
    if constexpr (i < N64)
      return n.x64[i];
    else
      return n.x32[i - N64];
  }

  IONIC_DEV static void load(Node& x, const void* base, long long stride, long long v) {
    const double* p64 = static_cast<const double*>(base);
    const float* p32 = reinterpret_cast<const float*>(p64 + N64 * stride);
    static_for<N>([&](auto I) {
      constexpr int i = I;
      if constexpr (i < N64)
        at<i>(x) = p64[i * stride + v];
      else
        at<i>(x) = p32[(i - N64) * stride + v];
    });
  }
  IONIC_DEV static void store(const Node& x, void* base, long long stride, long long v) {
    double* p64 = static_cast<double*>(base);
    float* p32 = reinterpret_cast<float*>(p64 + N64 * stride);
    static_for<N>([&](auto I) {
      constexpr int i = I;
      if constexpr (i < N64)
        p64[i * stride + v] = at<i>(x);
      else
        p32[(i - N64) * stride + v] = at<i>(x);
    });
  }
  IONIC_DEV static void to_eval(const Node& x, TE (&xe)[N]) {
    static_for<N>([&](auto I) {
      constexpr int i = I;
      xe[i] = TE(at<i>(x));
    });
  }
};

template <class Model, class T, class Sink, size_t... I>
IONIC_DEV void call_rhs_F(const typename Model::template Params<T>& p, T stim, T diff, Sink& s,
                          const T (&x)[Model::N], std::index_sequence<I...>) {
  Model::rhs(p, stim, diff, s, plain(x[I])...);
}
template <class Model, class T, class Sink, size_t... I>
IONIC_DEV void call_rhs_FJ(const typename Model::template Params<T>& p, T stim, T diff, Sink& s,
                           const T (&x)[Model::N], std::index_sequence<I...>) {
  Model::rhs(p, stim, diff, s, seed<T, int(I)>(x[I])...);
}

// evaluation seeded on the states in Mask only (their partials are carried,
// every other state enters as a plain value)
template <class T, int I, uint32_t Mask>
IONIC_DEV auto seed_if(T x) {
  if constexpr (has(Mask, I))
    return seed<T, I>(x);
  else
    return plain(x);
}
template <class Model, class T, uint32_t Mask, class Sink, size_t... I>
IONIC_DEV void call_rhs_masked(const typename Model::template Params<T>& p, T stim, T diff, Sink& s,
                               const T (&x)[Model::N], std::index_sequence<I...>) {
  Model::rhs(p, stim, diff, s, seed_if<T, int(I), Mask>(x[I])...);
}

template <class Model, class T>
IONIC_DEV void eval_F(const typename Model::template Params<T>& p, T stim, T diff,
                      const T (&x)[Model::N], T (&f)[Model::N]) {
  SinkF<Model, T> s{f};
  call_rhs_F<Model, T>(p, stim, diff, s, x, std::make_index_sequence<Model::N>{});
}
// F and J at x, and the solution of (I - dtau J(x)) delta = b with b_i = bfn(i, F_i),
// the elimination running while the model emits its rows.
template <class Model, class T, class BFn>
IONIC_DEV void eval_solve(const typename Model::template Params<T>& p, T stim, T diff, T dtau,
                          const T (&x)[Model::N], BFn bfn, T (&f)[Model::N], T (&delta)[Model::N]) {
  SinkElim<Model, T, BFn> s(dtau, bfn);
  call_rhs_FJ<Model, T>(p, stim, diff, s, x, std::make_index_sequence<Model::N>{});
  s.solve(delta);
  static_for<Model::N>([&](auto I) { f[I] = s.f[I]; });
}

// F and J rows held for a later solve at the same point: row i's value, then
// its partials on the pattern ROW[i] (zero where the evaluation carried none),
// one word each, in one column per lane of a [words][kBlock] array.
template <class Model>
struct JacRows {
  static constexpr int N = Model::N;
  static constexpr int off(int i) {
    int o = 0;
    for (int j = 0; j < i; ++j) o += 1 + popc(Model::ROW[j]);
    return o;
  }
  static constexpr int kWords = off(N);
};

// Keeps the rows in a JacRows column only.
template <class Model, class T>
struct SinkKeep {
  T* col;  // this lane's column: word w at col[w * kBlock]
  template <int i, uint32_t Mx>
  IONIC_DEV void put(const D<T, Mx>& x) {
    constexpr int o = JacRows<Model>::off(i);
    col[o * kBlock] = x.v;
    for_bits<Model::ROW[i]>([&](auto K) {
      constexpr int k = K;
      if constexpr (has(Mx, k))
        col[(o + 1 + rank(Model::ROW[i], k)) * kBlock] = x.template d<k>();
      else
        col[(o + 1 + rank(Model::ROW[i], k)) * kBlock] = T(0);
    });
  }
};

// Passes every row on to the inner sink and, when rec (uniform over the
// wavefront), keeps a copy in a JacRows column.
template <class Model, class T, class Inner>
struct SinkRecord {
  Inner& in;
  SinkKeep<Model, T> keep;
  bool rec;
  template <int i, uint32_t Mx>
  IONIC_DEV void put(const D<T, Mx>& x) {
    if (rec) keep.template put<i>(x);
    in.template put<i>(x);
  }
};

// eval_solve that also keeps the F and J rows in a JacRows column
template <class Model, class T, class BFn>
IONIC_DEV void eval_solve_keep(const typename Model::template Params<T>& p, T stim, T diff, T dtau,
                               const T (&x)[Model::N], BFn bfn, T (&f)[Model::N],
                               T (&delta)[Model::N], T* col, bool rec) {
  SinkElim<Model, T, BFn> s(dtau, bfn);
  SinkRecord<Model, T, SinkElim<Model, T, BFn>> r{s, {col}, rec};
  call_rhs_FJ<Model, T>(p, stim, diff, r, x, std::make_index_sequence<Model::N>{});
  s.solve(delta);
  static_for<Model::N>([&](auto I) { f[I] = s.f[I]; });
}

// The solve of eval_solve from rows kept by eval_solve_keep at the same point
// (any dtau and right-hand side): the rows are fed to the elimination again,
// rows eliminated first before the core rows, as the model emits them.
template <class Model, class T, class BFn>
IONIC_DEV void replay_solve(T dtau, BFn bfn, T (&f)[Model::N], T (&delta)[Model::N],
                            const T* col) {
  using E = Elim<Model>;
  SinkElim<Model, T, BFn> s(dtau, bfn);
  __builtin_amdgcn_sched_barrier(0);
  static_for<Model::N>([&](auto K) {
    constexpr int i = E::at(K);
    constexpr uint32_t R = Model::ROW[i];
    constexpr int o = JacRows<Model>::off(i);
    D<T, R> x;
    x.v = col[o * kBlock];
    static_for<popc(R)>([&](auto J) { x.g[J] = col[(o + 1 + J) * kBlock]; });
    s.template put<i>(x);
  });
  __builtin_amdgcn_sched_barrier(0);
  s.solve(delta);
  static_for<Model::N>([&](auto I) { f[I] = s.f[I]; });
}

IONIC_DEV unsigned long long wave_sum(unsigned long long x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
IONIC_DEV unsigned int wave_max(unsigned int x) {
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned int y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}

IONIC_DEV unsigned long long wave_max_u64(unsigned long long x) {
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}

// Register-pressure policies of the step kernel (one vertex per lane, one
// wavefront per SIMD: 512 registers per lane, beyond which it spills to
// scratch memory).
//
// lds: F(X_n) and the quadrature sums Q_m of a sweep live in LDS, one column
// per lane (lane-consecutive addresses, free of bank conflicts), instead of
// registers: 456 B per lane with 3 nodes, 608 B with 4, at most 38.9 KB per
// single-wave workgroup, so the 4 workgroups of a compute unit fit its 160 KB.
// Used by the double TT06 kernels with 3 and 4 nodes, which otherwise spill.
//
// split_evals: in a sweep, the F-only evaluations at nodes 2..M-1 and the F+J
// evaluations at the same (not yet updated) points are independent of the
// solve at node 1, and the F values they share are the same.  Left to itself
// the optimiser merges them and schedules the evaluations of several nodes
// together, which keeps two or three model evaluations' intermediates live at
// once.  With split_evals each evaluation starts from a copy of its point that
// the optimiser cannot see through and behind a scheduling barrier, so the
// evaluations run one after another (the F values are computed twice, as the
// algorithm states).  The double kernels spill 2.6x less with it at 3 nodes
// and 4.4x less at 4 nodes; the fp32 kernel with 3 nodes fits its registers
// without it and keeps the shared work.  The fp32 ROS2 kernels do not take
// it: built with it, the TT06 one with 4 nodes returned NaN for every vertex
// (the cause was not found; the same source is exact in the other kernels).

template <class Model, class Prec, int M, int Pred>
struct StepPolicy {
  static constexpr bool large = Model::N > 8;  // TT06; LR91 fits its registers either way
  static constexpr bool lds = large && !Prec::mixed && (M == 3 || M == 4);
  static constexpr bool split_evals =
      large && (!Prec::mixed || (M >= 4 && Pred != 1 /* ROS2 */));
  // wavefronts per SIMD a build for a full grid is held to: two (at most 256
  // registers per lane, what spills there is going to scratch) where measured
  // faster than one wavefront with 512 registers: LR91 with 2 and 3 nodes
  // (10-23% on 1e6 vertices), TT06 mixed with 2 nodes and the ROS2 or
  // Rush-Larsen predictor (4%, 12%); not TT06 mixed with 2 nodes and Newton (5%
  // slower), nor LR91 mixed with 4 nodes (22% slower).  A launch too small to
  // give every SIMD two wavefronts takes the one-wavefront build.
  static constexpr int waves =
      (!large && M <= 3) || (large && Prec::mixed && M == 2 && Pred != 0) ? 2 : 1;
  // reuse: the first Newton iteration on sub-interval 1 starts at X_1, the
  // node the first sweep's solve at node 1 evaluates F and J at; its rows
  // are kept in LDS (JacRows: 95 words per lane for TT06, 32 for LR91) and
  // that solve is replayed from them (with its own dtau and right-hand side)
  // instead of evaluating the model again: one evaluation per step fewer.
  // Where the evaluation at node 1 is still made (later sweeps) its rows go
  // through LDS the same way, so the solve is one code path.  Used by the
  // mixed kernels where it measured faster on 1e6 vertices: LR91 with 3
  // nodes (60.0 -> 54.5 ms for 500 steps), TT06 with 4 nodes (191 -> 187 ms
  // for 200 steps) and 5 (279 -> 213 ms for 100 steps; fewer spills).  Not
  // kept: TT06 mixed with 3 nodes (the kernel then spills, 0 -> 168 B per
  // lane, 234 -> 261 ms), LR91 mixed with 4 nodes (81 -> 86 ms), the LR91
  // double kernels (the same or slower); the TT06 double kernels' rows would
  // double the LDS a workgroup holds.
  static constexpr bool reuse =
      Pred == 0 && Prec::mixed && (large ? M >= 4 : M == 3);
};

// An opaque copy: the optimiser cannot relate the result to the argument.
template <class T, int N>
IONIC_DEV void opaque(T (&x)[N]) {
  for (int q = 0; q < N; ++q) asm volatile("" : "+v"(x[q]));
}

// W: wavefronts per SIMD the build is held to (1: up to 512 registers per
// lane; 2: up to 256)
template <class Model, class Prec, int M, int Pred, int W>
__global__ void __launch_bounds__(kBlock, W)
    sdc_kernel(const LaunchArgs<typename Model::template Params<typename Prec::TE>> args) {
  using L = Layout<Model, Prec>;
  using TE = typename Prec::TE;
  using Node = typename L::Node;
  constexpr int N = Model::N;

  // which simulation this workgroup belongs to (uniform)
  int sidx = 0;
  for (int k = 1; k < args.n_sims; ++k)
    if (int(blockIdx.x) >= args.sims[k].first_block) sidx = k;
  const SimDesc& sd = args.sims[sidx];
  const long long v = (long long)(blockIdx.x - sd.first_block) * kBlock + threadIdx.x;
  const bool active = v < sd.n;
  const long long vc = active ? v : sd.n - 1;  // tail lanes shadow the last slot
  // the vertex this lane advances (every lane reads and writes its own vertex
  // only).  Only the mixed kernels take the processing order: it made no
  // difference to the double ones, whose registers it crowded (spills)
  constexpr bool kOrdered = Prec::mixed;
  const long long vi = (kOrdered && sd.order) ? (long long)sd.order[vc] : vc;

  double t0 = sd.t0, dt = sd.dt;
  const void* src = sd.state;
  void* dst = sd.state;
  if constexpr (Pred == kPredRos2) {
    if (args.ctl) {  // adaptive attempt: time, step and buffers from the control block
      const AdaptCtl* c = args.ctl;
      if (c->done) return;
      t0 = c->t;
      dt = c->tau;
      if (c->cur)
        src = args.state_alt;
      else
        dst = args.state_alt;
    }
  }

  const auto& p = args.params;
  const TE stim_amp = sd.i_stim ? TE(sd.i_stim[vi]) : TE(0);
  const TE diff = sd.i_diff ? TE(sd.i_diff[vi]) : TE(0);
  TE dtau[M - 1];
  double Sdt[M - 1][M];
  static_for<M - 1>([&](auto m) {
    dtau[m] = TE(args.dc[m] * dt);
    static_for<M>([&](auto j) { Sdt[m][j] = args.S[m][j] * dt; });
  });
  const TE tol = TE(args.tol);

  Node X[M];
  L::load(X[0], src, sd.stride, vi);

  // F0 = F(X_n) and the quadrature sums Q(m, i) of a sweep, in registers or LDS
  using Pol = StepPolicy<Model, Prec, M, Pred>;
  __shared__ TE lds_f0[Pol::lds ? N : 1][kBlock];
  __shared__ double lds_q[Pol::lds ? (M - 1) * N : 1][kBlock];
  // F and J rows at X_1 from the predictor, for the first sweep (Pol::reuse)
  __shared__ TE lds_jac[Pol::reuse ? JacRows<Model>::kWords : 1][kBlock];
  TE* const jac_col = &lds_jac[0][threadIdx.x];
  TE reg_f0[Pol::lds ? 1 : N];
  double reg_q[Pol::lds ? 1 : (M - 1) * N];
  auto F0 = [&](int i) -> TE& {
    if constexpr (Pol::lds)
      return lds_f0[i][threadIdx.x];
    else
      return reg_f0[i];
  };
  auto Q = [&](int m, int i) -> double& {
    if constexpr (Pol::lds)
      return lds_q[m * N + i][threadIdx.x];
    else
      return reg_q[m * N + i];
  };

  unsigned long long it_total = 0;
  unsigned int it_max = 0, nonconv = 0;
  TE err_est = TE(0);  // ROS2: largest scaled embedded error of the launch

  for (int step = 0; step < sd.n_steps; ++step) {
    const double t_mid = t0 + (double(sd.step_offset + step) + 0.5) * dt;
    const TE stim = (sd.t_on <= t_mid && t_mid < sd.t_off) ? stim_amp : TE(0);
    // F0 = F(X_n), needed by the sweeps: every predictor evaluates F there first
    // and writes it before anything reads it

    if constexpr (Pred == kPredRos2) {
      // ---- predictor: one ROS2 step on each sub-interval
      static_for<M - 1>([&](auto MM) {
        constexpr int m = MM;
        TE xe[N], u1[N], u2[N], x2[N], r2[N];
        L::to_eval(X[m], xe);
        const TE gt = TE(kRosGamma) * dtau[m];
        auto b1 = [&](auto, TE fi) -> TE { return gt * fi; };
        SinkElim<Model, TE, decltype(b1), true> s(gt, b1);
        call_rhs_FJ<Model, TE>(p, stim, diff, s, xe, std::make_index_sequence<N>{});
        s.solve(u1);
        if constexpr (m == 0) static_for<N>([&](auto I) { F0(I) = s.f[I]; });
        static_for<N>([&](auto I) { x2[I] = xe[I] + TE(kRosA21) * u1[I]; });
        eval_F<Model, TE>(p, stim, diff, x2, r2);
        static_for<N>([&](auto I) { r2[I] = gt * r2[I] - TE(2) * u1[I]; });
        s.resolve(r2, u2);
        X[m + 1] = X[m];
        static_for<N>([&](auto I) {
          constexpr int i = I;
          auto& y = L::template at<i>(X[m + 1]);
          y += TE(kRosM1) * u1[i] + TE(kRosM2) * u2[i];
          const TE ay = fabs(TE(y));
          const TE sc = ay > TE(Model::SCALE[i]) ? ay : TE(Model::SCALE[i]);
          // fp32: the hardware reciprocal (1 ulp) in place of an IEEE division;
          // fp64 keeps the exact quotient
          const TE num = fabs(TE(kRosM2) * (u1[i] + u2[i]));
          TE e;
          if constexpr (sizeof(TE) == 4) e = num * f_rcp(sc); else e = num / sc;
          err_est = (e > err_est || e != e) ? e : err_est;
        });
      });
    } else if constexpr (Pred == kPredRushLarsen) {
      // ---- predictor: Rush-Larsen gating steps, then backward Euler on the core
      constexpr int NC = Model::N64;
      constexpr uint32_t CORE = (1u << NC) - 1u;
      constexpr uint32_t GATES = ((N >= 32) ? 0xFFFFFFFFu : ((1u << N) - 1u)) & ~CORE;
      static_for<M - 1>([&](auto MM) {
        constexpr int m = MM;
        Node Y = X[m];
        {
          TE xe[N];
          L::to_eval(X[m], xe);
          SinkGateStep<Model, TE> s;
          call_rhs_masked<Model, TE, GATES>(p, stim, diff, s, xe, std::make_index_sequence<N>{});
          if constexpr (m == 0) static_for<N>([&](auto I) { F0(I) = s.f[I]; });
          static_for<N - NC>([&](auto GG) {
            constexpr int g = NC + GG;
            const TE z = dtau[m] * s.d[g];
            const bool z0 = z == TE(0);
            const TE phi = pick(z0, TE(1), f_expm1(z) * f_rcp(pick(z0, TE(1), z)));
            L::template at<g>(Y) = TE(L::template at<g>(X[m])) + dtau[m] * s.f[g] * phi;
          });
        }
        int it = 0;
        bool conv = false, run = true;
        do {
          TE xe[N], delta[NC];
          L::to_eval(Y, xe);
          // core rows: b = -(Y - X_m - dtau F(Y)), formed in double
          auto bfn = [&](auto I, TE fi) -> TE {
            constexpr int i = I;
            return TE(double(L::template at<i>(X[m])) - double(L::template at<i>(Y)) +
                      double(dtau[m]) * double(fi));
          };
          SinkCore<Model, TE, decltype(bfn)> s(dtau[m], bfn);
          call_rhs_masked<Model, TE, CORE>(p, stim, diff, s, xe, std::make_index_sequence<N>{});
          s.solve(delta);
          bool now_conv = true;  // |delta_i| <= tol s_i over the core
          static_for<NC>([&](auto I) {
            constexpr int i = I;
            auto& y = L::template at<i>(Y);
            const auto yn = y + delta[i];
            y = pick(run, yn, y);
            const TE ay = fabs(TE(yn));
            const TE sc = ay > TE(Model::SCALE[i]) ? ay : TE(Model::SCALE[i]);
            now_conv &= fabs(delta[i]) <= tol * sc;
          });
          it += int(run);
          conv = (run & now_conv) | (!run & conv);
          run = run & !conv & (it < args.maxit);
        } while (__builtin_amdgcn_ballot_w64(run) != 0);
        X[m + 1] = Y;
        it_total += (unsigned long long)it;
        it_max = (unsigned int)it > it_max ? (unsigned int)it : it_max;
        nonconv += conv ? 0u : 1u;
      });
    } else {
      // ---- predictor: backward Euler by local Newton on each sub-interval.  The
      // iteration loop is uniform over the wave (it runs while any lane still
      // iterates; a lane that has stopped keeps its iterate through selects), so
      // the kernel has no divergent loop exit: at such exits gfx950 builds of
      // the double kernels placed spill code ahead of the execution-mask restore.
      static_for<M - 1>([&](auto MM) {
        constexpr int m = MM;
        Node Y = X[m];
        int it = 0, pass = 0;
        bool conv = false, run = true;
        do {
          TE xe[N], f[N], delta[N];
          L::to_eval(Y, xe);
          // b = -(Y - X_m - dtau F(Y)), formed in double
          auto bfn = [&](auto I, TE fi) -> TE {
            constexpr int i = I;
            return TE(double(L::template at<i>(X[m])) - double(L::template at<i>(Y)) +
                      double(dtau[m]) * double(fi));
          };
          if constexpr (Pol::reuse && m == 1) {
            // the first iteration evaluates at Y = X_1: its rows serve the
            // first sweep's solve at node 1 (pass is uniform over the wave)
            eval_solve_keep<Model, TE>(p, stim, diff, dtau[m], xe, bfn, f, delta, jac_col, pass == 0);
          } else {
            eval_solve<Model, TE>(p, stim, diff, dtau[m], xe, bfn, f, delta);
          }
          // the first iteration on the first sub-interval evaluates at Y = X_n:
          // its F is the F(X_n) the sweeps need (pass counts the wave's
          // iterations, so this branch is uniform)
          if constexpr (m == 0) {
            if (pass == 0) static_for<N>([&](auto I) { F0(I) = f[I]; });
          }
          ++pass;
          // every quantity below is computed on all lanes and only chosen per
          // lane, with no conditional evaluation, so no divergent branch forms
          // stop test max_i |delta_i| / s_i <= tol, written as |delta_i| <= tol s_i
          // for every i (no division)
          bool now_conv = true;
          static_for<N>([&](auto I) {
            constexpr int i = I;
            auto& y = L::template at<i>(Y);
            const auto yn = y + delta[i];
            y = pick(run, yn, y);
            const TE ay = fabs(TE(yn));
            const TE s = ay > TE(Model::SCALE[i]) ? ay : TE(Model::SCALE[i]);
            now_conv &= fabs(delta[i]) <= tol * s;
          });
          it += int(run);
          conv = (run & now_conv) | (!run & conv);
          run = run & !conv & (it < args.maxit);
        } while (__builtin_amdgcn_ballot_w64(run) != 0);
        X[m + 1] = Y;
        it_total += (unsigned long long)it;
        it_max = (unsigned int)it > it_max ? (unsigned int)it : it_max;
        nonconv += conv ? 0u : 1u;
      });
    }

    // ---- corrections
    if (sd.n_sweeps > 0) {
      for (int k = 0; k < sd.n_sweeps; ++k) {
        static_for<M - 1>([&](auto m) {
          static_for<N>([&](auto i) { Q(m, i) = Sdt[m][0] * double(F0(i)); });
        });
        // F at nodes 2..M-1 (node 1 comes with its Jacobian below)
        static_for<M - 2>([&](auto JJ) {
          constexpr int jn = JJ + 2;
          TE xe[N], fj[N];
          L::to_eval(X[jn], xe);
          if constexpr (Pol::split_evals) opaque(xe);
          eval_F<Model, TE>(p, stim, diff, xe, fj);
          static_for<M - 1>([&](auto m) {
            static_for<N>([&](auto i) { Q(m, i) += Sdt[m][jn] * double(fj[i]); });
          });
        });
        static_for<M - 1>([&](auto MM) {
          constexpr int m = MM;
          TE xe[N], f[N], delta[N];
          if constexpr (Pol::split_evals) __builtin_amdgcn_sched_barrier(0);
          L::to_eval(X[m + 1], xe);
          if constexpr (Pol::split_evals) opaque(xe);
          // r = X^{k+1}_m - X^k_{m+1} + Q_m in double, formed before the evaluation
          // (Q_m is then dead during it); at m = 0 the evaluation point is node 1,
          // whose F enters every Q_m
          double r0[N];
          static_for<N>([&](auto I) {
            constexpr int i = I;
            r0[i] = double(L::template at<i>(X[m])) - double(L::template at<i>(X[m + 1])) + Q(m, i);
          });
          auto bfn = [&](auto I, TE fi) -> TE {
            constexpr int i = I;
            double r = r0[i];
            if constexpr (m == 0) r += Sdt[0][1] * double(fi);
            return TE(r);
          };
          if constexpr (Pol::reuse && m == 0) {
            // the first sweep solves at X_1, where the predictor kept F and J;
            // a later sweep evaluates at the corrected node and keeps its rows
            // the same way (k is uniform), so the solve is one code path
            if (k > 0) {
              SinkKeep<Model, TE> sk{jac_col};
              call_rhs_FJ<Model, TE>(p, stim, diff, sk, xe, std::make_index_sequence<N>{});
            }
            replay_solve<Model, TE>(dtau[m], bfn, f, delta, jac_col);
          } else {
            eval_solve<Model, TE>(p, stim, diff, dtau[m], xe, bfn, f, delta);
          }
          if constexpr (m == 0) {
            static_for<M - 2>([&](auto MM2) {
              constexpr int mm = MM2 + 1;
              static_for<N>([&](auto i) { Q(mm, i) += Sdt[mm][1] * double(f[i]); });
            });
          }
          static_for<N>([&](auto I) {
            constexpr int i = I;
            L::template at<i>(X[m + 1]) += delta[i];
          });
        });
      }
    }
    X[0] = X[M - 1];
  }

  unsigned int nonfinite = 0;
  static_for<N>([&](auto I) {
    constexpr int i = I;
    if (!isfinite(double(L::template at<i>(X[0])))) nonfinite = 1;
  });
  if constexpr (kOrdered) {
    // the vertex index is read again for the store (a volatile read, so the
    // compiler does not keep it in registers through the whole step loop)
    const long long vs = sd.order ? (long long)*(const volatile int*)(sd.order + vc) : vc;
    if (active) L::store(X[0], dst, sd.stride, vs);
  } else {
    if (active) L::store(X[0], dst, sd.stride, v);
  }

  if constexpr (Pred == kPredRos2) {
    if (args.ctl) {  // largest lane error of the attempt; a non-finite state rejects it
      double e = double(err_est);
      if (nonfinite || !(e <= 1.0e308)) e = __builtin_inf();
      const unsigned long long bits = wave_max_u64(active ? (unsigned long long)__double_as_longlong(e) : 0ull);
      if (threadIdx.x == 0) atomicMax(&args.err[blockIdx.x % kSlots].bits, bits);
    }
  }

  // wave-level reduction of the statistics, one set of atomics per wave
  const unsigned long long a_iters = wave_sum(active ? it_total : 0ull);
  const unsigned long long a_nonconv = wave_sum(active ? nonconv : 0u);
  const unsigned long long a_nonfin = wave_sum(active ? nonfinite : 0u);
  const unsigned long long a_act = wave_sum(active ? 1ull : 0ull);
  const unsigned int a_itmax = wave_max(active ? it_max : 0u);
  if (threadIdx.x == 0 && sd.stats) {
    DevStats* st = sd.stats + blockIdx.x % kSlots;
    atomicAdd(&st->vertex_steps, a_act * (unsigned long long)sd.n_steps);
    atomicAdd(&st->newton_iters, a_iters);
    if (Pred != kPredRos2)
      atomicAdd(&st->newton_solves, a_act * (unsigned long long)sd.n_steps * (M - 1));
    atomicAdd(&st->nonconverged, a_nonconv);
    atomicAdd(&st->nonfinite, a_nonfin);
    atomicMax(&st->it_max, a_itmax);
  }
}

// ---- auxiliary kernels --------------------------------------------------------------

// FP64 SoA rows (n_states x count, row stride ld) -> precision layout at [first, first+count)
template <class Model, class Prec>
__global__ void pack_kernel(const double* __restrict__ src, long long ld, void* state,
                            long long stride, long long first, long long count) {
  using L = Layout<Model, Prec>;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  typename L::Node x;
  static_for<Model::N>([&](auto I) {
    constexpr int i = I;
    L::template at<i>(x) = src[i * ld + t];
  });
  L::store(x, state, stride, first + t);
}

// precision layout -> FP64 SoA rows
template <class Model, class Prec>
__global__ void unpack_kernel(const void* state, long long stride, long long first,
                              long long count, double* __restrict__ dst, long long ld) {
  using L = Layout<Model, Prec>;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  typename L::Node x;
  L::load(x, state, stride, first + t);
  static_for<Model::N>([&](auto I) {
    constexpr int i = I;
    dst[i * ld + t] = double(L::template at<i>(x));
  });
}

template <class Model, class Prec>
__global__ void steady_gates_kernel(const typename Model::template Params<typename Prec::TE> p,
                                    void* state, long long stride, long long n) {
  using L = Layout<Model, Prec>;
  using TE = typename Prec::TE;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  typename L::Node x;
  L::load(x, state, stride, v);
  TE xe[Model::N];
  L::to_eval(x, xe);
  Model::template steady_gates<TE>(p, xe);
  static_for<Model::N>([&](auto I) {
    constexpr int i = I;
    if constexpr (i >= Model::N64) L::template at<i>(x) = xe[i];
  });
  L::store(x, state, stride, v);
}

// Resting state of the model on one lane, written to out[0..N): with
// Model::REST_BY_NEWTON, Newton's method on F(X) = 0 (no stimulus, no
// diffusion current) from REST_GUESS with the gates at their steady state,
// each iteration a dense solve with partial pivoting, until the scaled update
// max_i |delta_i| / max(|X_i|, SCALE_i) falls below 1e-15 (at most 50
// iterations); otherwise REST_GUESS itself.
template <class Model>
__global__ void rest_state_kernel(const typename Model::template Params<double> p, double* out) {
  constexpr int N = Model::N;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double x[N];
  for (int i = 0; i < N; ++i) x[i] = Model::REST_GUESS[i];
  if constexpr (Model::REST_BY_NEWTON) {
    Model::template steady_gates<double>(p, x);
    for (int it = 0; it < 50; ++it) {
      double f[N], A[N][N + 1];
      double J[N * N];
      for (int k = 0; k < N * N; ++k) J[k] = 0.0;
      SinkDense<Model, double> s{f, J};
      call_rhs_FJ<Model, double>(p, 0.0, 0.0, s, x, std::make_index_sequence<N>{});
      for (int i = 0; i < N; ++i) {
        for (int k = 0; k < N; ++k) A[i][k] = J[i * N + k];
        A[i][N] = -f[i];
      }
      for (int c = 0; c < N; ++c) {  // elimination with partial pivoting
        int pr = c;
        for (int i = c + 1; i < N; ++i)
          if (fabs(A[i][c]) > fabs(A[pr][c])) pr = i;
        if (A[pr][c] == 0.0) break;
        for (int k = 0; k <= N; ++k) {
          const double t = A[c][k];
          A[c][k] = A[pr][k];
          A[pr][k] = t;
        }
        for (int i = c + 1; i < N; ++i) {
          const double l = A[i][c] / A[c][c];
          for (int k = c; k <= N; ++k) A[i][k] -= l * A[c][k];
        }
      }
      double delta[N], worst = 0.0;
      for (int i = N - 1; i >= 0; --i) {
        double acc = A[i][N];
        for (int k = i + 1; k < N; ++k) acc -= A[i][k] * delta[k];
        delta[i] = acc / A[i][i];
      }
      for (int i = 0; i < N; ++i) {
        x[i] += delta[i];
        const double sc = fmax(fabs(x[i]), Model::SCALE[i]);
        worst = fmax(worst, fabs(delta[i]) / sc);
      }
      if (!(worst >= 1e-15)) break;  // converged (or non-finite: stop)
    }
  }
  for (int i = 0; i < N; ++i) out[i] = x[i];
}

// Every vertex of [0, n) set to the one state x (N doubles), in the precision layout.
template <class Model, class Prec>
__global__ void broadcast_kernel(const double* __restrict__ x, void* state, long long stride,
                                 long long n) {
  using L = Layout<Model, Prec>;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  typename L::Node node;
  static_for<Model::N>([&](auto I) {
    constexpr int i = I;
    L::template at<i>(node) = x[i];
  });
  L::store(node, state, stride, v);
}

template <class Model, class Prec>
__global__ void debug_jacobian_kernel(const typename Model::template Params<typename Prec::TE> p,
                                      const void* state, long long stride, long long v,
                                      double stim, double diff, double* out /* N + N*N */) {
  using L = Layout<Model, Prec>;
  using TE = typename Prec::TE;
  constexpr int N = Model::N;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  typename L::Node x;
  L::load(x, state, stride, v);
  TE xe[N], f[N], J[N * N];
  for (int k = 0; k < N * N; ++k) J[k] = TE(0);
  L::to_eval(x, xe);
  SinkDense<Model, TE> s{f, J};
  call_rhs_FJ<Model, TE>(p, TE(stim), TE(diff), s, xe, std::make_index_sequence<N>{});
  for (int i = 0; i < N; ++i) out[i] = double(f[i]);
  for (int k = 0; k < N * N; ++k) out[N + k] = double(J[k]);
}

}  // namespace ionic
