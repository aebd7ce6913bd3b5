// The partitioned step with the parabolic term inside the implicit stages
// (paper section 3.3.2, Algorithm 2 and the solver paragraph after it;
// section 3.3.1, equation rb_system; equation sdc), on structured grids.
//
// Every ROS2 stage and the correction solve a global system
//     (B + c L) x = b,  B = blockdiag(I - c J_cell),  L = M_L^{-1} A_i on v.
// imp_block_kernel eliminates, per vertex, every state but V from its block
// (SinkSchur, schur_solve.h: the static sparse elimination with V as the last
// pivot) and leaves the reduced system S dv + c L dv = r for the field of
// V; BiCGSTAB (the paper's Krylov method) solves it over the grid with the
// diagonal of the reduced operator as preconditioner; a second pass of the
// block kernel re-evaluates F and J at the same point, repeats the same
// elimination and recovers every state from dv.  The paper applies BiCGSTAB
// with block Jacobi to the whole system; eliminating the per-vertex block
// exactly first leaves a Krylov solve over one unknown per vertex, whose
// matrix-vector product is one stencil pass (no Jacobian is stored).
//
// BiCGSTAB launch shape and reductions follow elliptic.hip: nb blocks of 256
// threads, block b owning chunk (b mod 8) nb/8 + b/8 of the nodes, dot
// products as per-block partial sums added in a fixed order by every block of
// the next launch (reproducible bit for bit, no atomics).  An iteration is five
// launches: direction, v = A p^, s, t = A s^, update; the first tests
// ||r_k|| <= rtol ||r_0|| and sets a device flag after which queued launches
// return at once.
#include "implicit_ops.h"
#include "kernel_ops.h"
#include "model_lr91.h"
#include "model_test.h"
#include "model_tt06.h"
#include "schur_solve.h"
#include "stencil.h"

namespace ionic {

namespace {

// ---- per-vertex block passes ----------------------------------------------------------

// T: the type F, J and the elimination are evaluated in (double, or float for
// handles in the mixed layout); the states, the right-hand side's base and
// every output stay double.
template <class Model, class T>
struct BlockArgs {
  typename Model::template Params<T> p;
  ImpBlock a;
};

template <class Model, class T>
__global__ void __launch_bounds__(64, 2) imp_block_kernel(const BlockArgs<Model, T> args) {
  constexpr int N = Model::N;
  const ImpBlock& a = args.a;
  const long long v = (long long)blockIdx.x * 64 + threadIdx.x;
  const bool active = v < a.n;
  const long long vi = active ? v : a.n - 1;  // tail lanes shadow the last vertex
  const long long st = a.stride;
  T x[N];
  double base[N];
  static_for<N>([&](auto I) { x[I] = T(a.X[I * st + vi]); });
  // every input is read before the evaluation, so its rows see no branch
  if (a.base)
    static_for<N>([&](auto I) { base[I] = a.base[I * st + vi]; });
  else
    static_for<N>([&](auto I) { base[I] = 0.0; });
  const T stim = T((a.stim_on && a.stim) ? a.stim[vi] : 0.0);
  const T diff = T(a.idiff ? a.idiff[vi] : 0.0);
  const double cf = a.cf;
  // the right-hand side formed in double, then taken to T
  auto bfn = [&](auto I, T fi) -> T { return T(cf * double(fi) + base[I]); };
  SinkSchur<Model, T, decltype(bfn)> s(T(a.c), bfn);
  call_rhs_FJ<Model, T>(args.p, stim, diff, s, x, std::make_index_sequence<N>{});
  T S, r;
  s.reduce(S, r);
  if (!a.expand) {
    if (active) {
      a.S[v] = double(S);
      a.r[v] = double(r);
    }
    return;
  }
  T delta[N];
  s.expand(T(a.dv[vi]), delta);
  if (active) static_for<N>([&](auto I) { a.out[I * st + v] = double(delta[I]); });
}

template <class Model, class T>
struct RhsArgs {
  typename Model::template Params<T> p;
  const double* X;
  long long n, stride;
  const double* stim;
  int stim_on;
  const double* idiff;
  double alpha, beta;
  const double* Y;
  double* out;
};

template <class Model, class T>
__global__ void __launch_bounds__(64) imp_rhs_kernel(const RhsArgs<Model, T> a) {
  constexpr int N = Model::N;
  const long long v = (long long)blockIdx.x * 64 + threadIdx.x;
  if (v >= a.n) return;
  T x[N], f[N];
  static_for<N>([&](auto I) { x[I] = T(a.X[I * a.stride + v]); });
  const T stim = T((a.stim_on && a.stim) ? a.stim[v] : 0.0);
  const T diff = T(a.idiff ? a.idiff[v] : 0.0);
  eval_F<Model, T>(a.p, stim, diff, x, f);
  static_for<N>([&](auto I) {
    const double y = a.Y ? a.Y[I * a.stride + v] : 0.0;
    a.out[I * a.stride + v] = a.alpha * double(f[I]) + a.beta * y;
  });
}

template <class Model, class T>
hipError_t block_launch(const void* params, const ImpBlock& a, hipStream_t st) {
  BlockArgs<Model, T> args;
  args.p = *static_cast<const typename Model::template Params<T>*>(params);
  args.a = a;
  hipLaunchKernelGGL((imp_block_kernel<Model, T>), dim3(unsigned((a.n + 63) / 64)), dim3(64), 0,
                     st, args);
  return hipGetLastError();
}

template <class Model, class T>
hipError_t rhs_launch(const void* params, const double* X, long long n, long long stride,
                      const double* stim, int stim_on, const double* idiff, double alpha,
                      double beta, const double* Y, double* out, hipStream_t st) {
  RhsArgs<Model, T> a;
  a.p = *static_cast<const typename Model::template Params<T>*>(params);
  a.X = X;
  a.n = n;
  a.stride = stride;
  a.stim = stim;
  a.stim_on = stim_on;
  a.idiff = idiff;
  a.alpha = alpha;
  a.beta = beta;
  a.Y = Y;
  a.out = out;
  hipLaunchKernelGGL((imp_rhs_kernel<Model, T>), dim3(unsigned((n + 63) / 64)), dim3(64), 0, st,
                     a);
  return hipGetLastError();
}

// ---- elementwise passes over state planes -------------------------------------------------

constexpr int kElemThreads = 256;
constexpr int kElemBlocks = 2048;

__global__ void __launch_bounds__(kElemThreads)
    lincomb_kernel(double* __restrict__ out, const double* __restrict__ x, double a,
                   const double* __restrict__ y, double b, const double* __restrict__ z,
                   long long elems) {
  const long long step = (long long)gridDim.x * kElemThreads;
  for (long long e = (long long)blockIdx.x * kElemThreads + threadIdx.x; e < elems; e += step) {
    double o = x[e] + a * y[e];
    if (z) o += b * z[e];
    out[e] = o;
  }
}

constexpr int kMaxStates = 32;
struct Scales {
  double s[kMaxStates];
};

__device__ __forceinline__ unsigned long long wave_max_bits(unsigned long long x) {
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}

__global__ void __launch_bounds__(kElemThreads)
    finish_kernel(const double* __restrict__ XT, const double* __restrict__ eps,
                  double* __restrict__ XK, long long n, long long stride, int n_states, Scales sc,
                  unsigned long long* change) {
  const long long step = (long long)gridDim.x * kElemThreads;
  const long long elems = (long long)n_states * stride;
  double worst = 0.0;
  for (long long e = (long long)blockIdx.x * kElemThreads + threadIdx.x; e < elems; e += step) {
    const long long i = e / stride, v = e - i * stride;
    if (v >= n) continue;
    const double xn = XT[e] + eps[e];
    const double d = fabs(xn - XK[e]) / fmax(fabs(xn), sc.s[i]);
    worst = (d > worst || d != d) ? d : worst;
    XK[e] = xn;
  }
  if (!(worst <= 1.0e308)) worst = __builtin_inf();
  const unsigned long long bits = wave_max_bits((unsigned long long)__double_as_longlong(worst));
  if ((threadIdx.x & 63) == 0) atomicMax(change, bits);
}

// ---- BiCGSTAB on the reduced system -----------------------------------------------------

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlocks = 1024;
constexpr int kXcds = 8;
constexpr int kLanesOut = 62;

__device__ __forceinline__ double wave_sum_d(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ long long chunk_id(const CgParams& c) {
  const long long b = blockIdx.x;
  return (b % kXcds) * (c.nb / kXcds) + b / kXcds;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double lds[NV][kWaves];
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = wave_sum_d(v[a]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) lds[a][threadIdx.x >> 6] = v[a];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = (lds[a][0] + lds[a][1]) + (lds[a][2] + lds[a][3]);
}

template <int NV>
__device__ __forceinline__ void put_partials(double (&v)[NV], double* const (&part)[NV],
                                             const CgParams& c) {
  block_sum(v);
  if (threadIdx.x == 0) {
    const long long L = chunk_id(c);
#pragma unroll
    for (int a = 0; a < NV; ++a) part[a][L] = v[a];
  }
}

template <int NV>
__device__ __forceinline__ void total_of(const double* const (&part)[NV], const CgParams& c,
                                         double (&s)[NV]) {
#pragma unroll
  for (int a = 0; a < NV; ++a) s[a] = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxBlocks / kThreads; ++j) {
    const long long t = threadIdx.x + (long long)j * kThreads;
    if (t < c.nb) {
#pragma unroll
      for (int a = 0; a < NV; ++a) s[a] += part[a][t];
    }
  }
  block_sum(s);
}

struct Span {
  long long first, end;
};
__device__ __forceinline__ Span my_span(const CgParams& c) {
  const long long begin = chunk_id(c) * c.chunk, end = begin + c.chunk;
  return {begin + threadIdx.x, end < c.n ? end : c.n};
}

// per-iteration scalars: rho_k, alpha_k, omega_k, r_k.r_k
__device__ __forceinline__ double* iter_sc(const BiCgWork& w, long long k) { return w.sc + 8 + 4 * k; }
__device__ __forceinline__ BiCgCtl* ctl_of(const BiCgWork& w) {
  return reinterpret_cast<BiCgCtl*>(w.sc + 4);
}

// y = S x + cst M_L^{-1} A_i x over this block's nodes (lane-shuffle stencil),
// and the block's parts of the products of y with u and of y with itself
__device__ __forceinline__ void apply_op(const CgParams& c, double inv_h2, double cst,
                                        const double* __restrict__ S, const double* __restrict__ x,
                                        double* __restrict__ y, const double* __restrict__ u,
                                        double& yu, double& yy) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long begin = chunk_id(c) * c.chunk;
  const long long end = begin + c.chunk < c.n ? begin + c.chunk : c.n;
  const auto x_of = [x](long long t) { return x[t]; };
  for (long long first = begin + wave * kLanesOut; first < end; first += kWaves * kLanesOut) {
    const long long v = first - 1 + lane;
    const long long vl = v < 0 ? 0 : (v < c.n ? v : c.n - 1);
    const Q1Coords q = q1_coords(vl, c.nx, c.ny);
    const Q1Node node(q.i, q.j, q.k, c.nx, c.ny, c.nz);
    double xv;
    const double ax = node.apply_lanes(x_of, c.si, xv);
    if (lane >= 1 && lane <= kLanesOut && v < end) {
      const double yv = S[v] * xv + cst * inv_h2 * ax / node.mass();
      y[v] = yv;
      yu += yv * u[v];
      yy += yv * yv;
    }
  }
}

// the start of a solve from the guess in w.x (zero unless warm): r = rhs - A x,
// r^ = r, p = v = 0, the inverse diagonal, and the parts of r^.r, r.r and rhs.rhs
__global__ void __launch_bounds__(kThreads)
    bicg_start_kernel(CgParams c, double inv_h2, double cst, const double* __restrict__ S,
                      const double* __restrict__ rhs, BiCgWork w, int warm) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl_of(w)->done = 0;
    ctl_of(w)->reserved = 0;
    ctl_of(w)->iters = 0;
  }
  double s[3] = {0.0, 0.0, 0.0};  // r^.r, r.r, rhs.rhs
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long begin = chunk_id(c) * c.chunk;
  const long long end = begin + c.chunk < c.n ? begin + c.chunk : c.n;
  const double* const x = w.x;
  const auto x_of = [x, warm](long long t) { return warm ? x[t] : 0.0; };
  for (long long first = begin + wave * kLanesOut; first < end; first += kWaves * kLanesOut) {
    const long long v = first - 1 + lane;
    const long long vl = v < 0 ? 0 : (v < c.n ? v : c.n - 1);
    const Q1Coords q = q1_coords(vl, c.nx, c.ny);
    const Q1Node node(q.i, q.j, q.k, c.nx, c.ny, c.nz);
    double xv;
    const double ax = node.apply_lanes(x_of, c.si, xv);
    if (lane >= 1 && lane <= kLanesOut && v < end) {
      const double m = node.mass();
      w.dinv[v] = 1.0 / (S[v] + cst * inv_h2 * node.diag(c.si) / m);
      const double b = rhs[v];
      const double r = b - (S[v] * xv + cst * inv_h2 * ax / m);
      if (!warm) w.x[v] = 0.0;
      w.r[v] = r;
      w.rh[v] = r;
      w.p[v] = 0.0;
      w.v[v] = 0.0;
      s[0] += r * r;
      s[1] += r * r;
      s[2] += b * b;
    }
  }
  double* const part[3] = {w.part[0], w.part[1], w.part[2]};
  put_partials(s, part, c);
}

// A: the test of ||r_k||, then the direction p = r + beta (p - omega v), p^ = p / D
__global__ void __launch_bounds__(kThreads) bicg_dir_kernel(CgParams c, BiCgWork w, long long k) {
  if (ctl_of(w)->done) return;
  // rho_k = r^.r_k, r_k.r_k, and at k = 0 rhs.rhs (part 2 holds it until v = A p^;
  // later it holds r^.v of the previous iteration, summed and not used)
  const double* const in[3] = {w.part[0], w.part[1], w.part[2]};
  double t[3];
  total_of(in, c, t);
  const double bb = k == 0 ? t[2] : w.sc[0];
  const double rel = bb > 0.0 ? ::sqrt(t[1] / bb) : 0.0;
  const bool stop = !(rel > c.rtol);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) w.sc[0] = t[2];
    iter_sc(w, k)[0] = t[0];
    iter_sc(w, k)[3] = t[1];
    if (stop) {
      ctl_of(w)->iters = k;
      ctl_of(w)->done = 1;
    }
  }
  if (stop) return;
  double beta = 0.0, omega = 0.0;
  if (k > 0) {
    const double* prev = iter_sc(w, k - 1);
    omega = prev[2];
    const double den = prev[0] * omega;
    beta = den != 0.0 ? (t[0] / prev[0]) * (prev[1] / omega) : 0.0;
  }
  for (long long v = my_span(c).first, e = my_span(c).end; v < e; v += kThreads) {
    const double pv = w.r[v] + beta * (w.p[v] - omega * w.v[v]);
    w.p[v] = pv;
    w.ph[v] = pv * w.dinv[v];
  }
}

// B: v = A p^ and the parts of r^.v
__global__ void __launch_bounds__(kThreads)
    bicg_mv1_kernel(CgParams c, double inv_h2, double cst, const double* __restrict__ S, BiCgWork w) {
  if (ctl_of(w)->done) return;
  double s[1] = {0.0};
  double unused = 0.0;
  apply_op(c, inv_h2, cst, S, w.ph, w.v, w.rh, s[0], unused);
  double* const part[1] = {w.part[2]};
  put_partials(s, part, c);
}

// C: alpha = rho / r^.v, s = r - alpha v, s^ = s / D
__global__ void __launch_bounds__(kThreads) bicg_s_kernel(CgParams c, BiCgWork w, long long k) {
  if (ctl_of(w)->done) return;
  const double* const in[1] = {w.part[2]};
  double t[1];
  total_of(in, c, t);
  const double rho = iter_sc(w, k)[0];
  const double alpha = t[0] != 0.0 ? rho / t[0] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) iter_sc(w, k)[1] = alpha;
  for (long long v = my_span(c).first, e = my_span(c).end; v < e; v += kThreads) {
    const double sv = w.r[v] - alpha * w.v[v];
    w.s[v] = sv;
    w.sh[v] = sv * w.dinv[v];
  }
}

// D: t = A s^ and the parts of t.s and t.t
__global__ void __launch_bounds__(kThreads)
    bicg_mv2_kernel(CgParams c, double inv_h2, double cst, const double* __restrict__ S, BiCgWork w) {
  if (ctl_of(w)->done) return;
  double s[2] = {0.0, 0.0};
  apply_op(c, inv_h2, cst, S, w.sh, w.t, w.s, s[0], s[1]);
  double* const part[2] = {w.part[3], w.part[4]};
  put_partials(s, part, c);
}

// E: omega = t.s / t.t, x += alpha p^ + omega s^, r = s - omega t, parts of r^.r and r.r
__global__ void __launch_bounds__(kThreads) bicg_upd_kernel(CgParams c, BiCgWork w, long long k) {
  if (ctl_of(w)->done) return;
  const double* const in[2] = {w.part[3], w.part[4]};
  double t[2];
  total_of(in, c, t);
  const double omega = t[1] != 0.0 ? t[0] / t[1] : 0.0;
  const double alpha = iter_sc(w, k)[1];
  if (blockIdx.x == 0 && threadIdx.x == 0) iter_sc(w, k)[2] = omega;
  double s[2] = {0.0, 0.0};
  for (long long v = my_span(c).first, e = my_span(c).end; v < e; v += kThreads) {
    w.x[v] += alpha * w.ph[v] + omega * w.sh[v];
    const double rv = w.s[v] - omega * w.t[v];
    w.r[v] = rv;
    s[0] += w.rh[v] * rv;
    s[1] += rv * rv;
  }
  double* const part[2] = {w.part[0], w.part[1]};
  put_partials(s, part, c);
}

}  // namespace

namespace {
template <class T>
hipError_t block_for(int model, const void* params, const ImpBlock& a, hipStream_t st) {
  switch (model) {
    case 1: return block_launch<LR91, T>(params, a, st);
    case 2: return block_launch<TT06, T>(params, a, st);
    case 90: return block_launch<TestLinear, T>(params, a, st);
    case 91: return block_launch<TestLogistic, T>(params, a, st);
    default: return hipErrorInvalidValue;
  }
}
template <class T>
hipError_t rhs_for(int model, const void* params, const double* X, long long n, long long stride,
                   const double* stim, int stim_on, const double* idiff, double alpha, double beta,
                   const double* Y, double* out, hipStream_t st) {
  switch (model) {
    case 1: return rhs_launch<LR91, T>(params, X, n, stride, stim, stim_on, idiff, alpha, beta, Y, out, st);
    case 2: return rhs_launch<TT06, T>(params, X, n, stride, stim, stim_on, idiff, alpha, beta, Y, out, st);
    case 90: return rhs_launch<TestLinear, T>(params, X, n, stride, stim, stim_on, idiff, alpha, beta, Y, out, st);
    case 91: return rhs_launch<TestLogistic, T>(params, X, n, stride, stim, stim_on, idiff, alpha, beta, Y, out, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t imp_block(int model, int eval_float, const void* params, const ImpBlock& a,
                     hipStream_t st) {
  return eval_float ? block_for<float>(model, params, a, st) : block_for<double>(model, params, a, st);
}

hipError_t imp_rhs(int model, int eval_float, const void* params, const double* X, long long n,
                   long long stride, const double* stim, int stim_on, const double* idiff,
                   double alpha, double beta, const double* Y, double* out, hipStream_t st) {
  return eval_float ? rhs_for<float>(model, params, X, n, stride, stim, stim_on, idiff, alpha, beta, Y, out, st)
                    : rhs_for<double>(model, params, X, n, stride, stim, stim_on, idiff, alpha, beta, Y, out, st);
}

hipError_t soa_lincomb(double* out, const double* x, double a, const double* y, double b,
                       const double* z, long long elems, hipStream_t st) {
  const long long want = (elems + kElemThreads - 1) / kElemThreads;
  const unsigned blocks = unsigned(want < kElemBlocks ? (want > 0 ? want : 1) : kElemBlocks);
  hipLaunchKernelGGL(lincomb_kernel, dim3(blocks), dim3(kElemThreads), 0, st, out, x, a, y, b, z,
                     elems);
  return hipGetLastError();
}

hipError_t imp_finish(const double* XT, const double* eps, double* XK, long long n, long long stride,
                      int n_states, const double* scale, unsigned long long* change,
                      hipStream_t st) {
  if (n_states > kMaxStates) return hipErrorInvalidValue;
  Scales sc{};
  for (int i = 0; i < n_states; ++i) sc.s[i] = scale[i];
  const long long elems = (long long)n_states * stride;
  const long long want = (elems + kElemThreads - 1) / kElemThreads;
  const unsigned blocks = unsigned(want < kElemBlocks ? (want > 0 ? want : 1) : kElemBlocks);
  hipLaunchKernelGGL(finish_kernel, dim3(blocks), dim3(kElemThreads), 0, st, XT, eps, XK, n, stride,
                     n_states, sc, change);
  return hipGetLastError();
}

hipError_t bicg_start(const CgParams& c, double h, double cst, const double* S, const double* rhs,
                      BiCgWork& w, int warm, hipStream_t st) {
  hipLaunchKernelGGL(bicg_start_kernel, dim3(unsigned(c.nb)), dim3(kThreads), 0, st, c,
                     1.0 / (h * h), cst, S, rhs, w, warm);
  return hipGetLastError();
}

hipError_t bicg_iteration(const CgParams& c, double h, double cst, const double* S, int k,
                          BiCgWork& w, hipStream_t st) {
  const double inv_h2 = 1.0 / (h * h);
  const dim3 g(unsigned(c.nb)), b(kThreads);
  hipLaunchKernelGGL(bicg_dir_kernel, g, b, 0, st, c, w, (long long)k);
  hipLaunchKernelGGL(bicg_mv1_kernel, g, b, 0, st, c, inv_h2, cst, S, w);
  hipLaunchKernelGGL(bicg_s_kernel, g, b, 0, st, c, w, (long long)k);
  hipLaunchKernelGGL(bicg_mv2_kernel, g, b, 0, st, c, inv_h2, cst, S, w);
  hipLaunchKernelGGL(bicg_upd_kernel, g, b, 0, st, c, w, (long long)k);
  return hipGetLastError();
}

}  // namespace ionic
