// Geometric multigrid preconditioner for the elliptic solve on structured
// grids: one symmetric V(1,1) cycle per application, used by the conjugate
// gradients of elliptic.hip in place of the Jacobi preconditioner.  The paper
// preconditions its elliptic Krylov solver with algebraic multigrid (section
// 3.3.2); on a structured grid the same hierarchy can be built from the
// tensor-product structure of the operator.
//
// Levels.  The Q1 operator of the fine grid is A = sum_a s_a K_a (x) M_b (x) M_c
// with 1D tridiagonal stiffness K and mass M per direction (the factors of
// stencil.h).  Each direction with more than 2 nodes is coarsened by taking
// every other node (and the last one): n -> (n + 1)/2 for odd n, n/2 + 1 for
// even n; the 1D prolongation P interpolates linearly in the index.  The
// Galerkin operator P^T A P of a tensor product is the tensor product of the
// 1D Galerkin factors P^T K P and P^T M P, again tridiagonal, so every level
// is the same kind of 27-point operator, described by 1D tables of 3 entries
// per index and direction (computed on the host, a few kB).  Coarsening stops
// at 512 nodes or fewer; that level is solved exactly: the host inverts
// A_c + alpha 1 1^T (A_c is singular, the constants being its null space;
// alpha = trace / n^2), a dense matrix of at most 2 MB, and the device applies
// it as one matrix-vector product.
//
// Cycle on level l with right-hand side b (x starts at zero):
//   pre-smoothing   x = w D^-1 b                    (one damped Jacobi sweep)
//   residual        y = b - A x
//   restriction     b_(l+1) = P^T y
//   coarse level    x_(l+1) = cycle(b_(l+1))       (coarsest: the exact inverse)
//   prolongation    x = x + P x_(l+1)
//   post-smoothing  x = x + w D^-1 (b - A x)        (one sweep, into y)
// with w = 2/3.  The smoothing before and after is the same sweep and the
// restriction is the transpose of the prolongation, so the cycle is a
// symmetric operator, as conjugate gradients require.  On level 0 the
// post-smoothing writes z and the block's part of r.z.
#include "grid_ops.h"
#include "stencil.h"

#include <algorithm>

namespace ionic {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlocks = 1024;
constexpr int kXcds = 8;
constexpr double kOmega = 2.0 / 3.0;

__device__ __forceinline__ double wave_sum_d(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ long long chunk_of(const MgLevel& g) {
  const long long b = blockIdx.x;
  return (b % kXcds) * (g.nb / kXcds) + b / kXcds;
}

struct Span {
  long long first, end;
};
__device__ __forceinline__ Span my_span(const MgLevel& g) {
  const long long begin = chunk_of(g) * g.chunk, end = begin + g.chunk;
  return {begin + threadIdx.x, end < g.n ? end : g.n};
}

// sums over the block in a fixed order, totals in every thread
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

// A node of level g: its 1D factor rows (3 entries each, zero where a
// neighbour is missing) and neighbour offsets.
struct TabNode {
  long long n0;
  long long ox[3], oy[3], oz[3];
  double Kx[3], Mx[3], Ky[3], My[3], Kz[3], Mz[3];

  __device__ __forceinline__ TabNode(long long v, const MgLevel& g) {
    const Q1Coords c = q1_coords(v, g.nx, g.ny);
    n0 = v;
    ox[0] = c.i > 0 ? -1 : 0;
    ox[1] = 0;
    ox[2] = c.i < g.nx - 1 ? 1 : 0;
    oy[0] = c.j > 0 ? -g.nx : 0;
    oy[1] = 0;
    oy[2] = c.j < g.ny - 1 ? g.nx : 0;
    oz[0] = c.k > 0 ? -g.nx * g.ny : 0;
    oz[1] = 0;
    oz[2] = c.k < g.nz - 1 ? g.nx * g.ny : 0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      Kx[t] = g.K[0][3 * c.i + t];
      Mx[t] = g.M[0][3 * c.i + t];
      Ky[t] = g.K[1][3 * c.j + t];
      My[t] = g.M[1][3 * c.j + t];
      Kz[t] = g.K[2][3 * c.k + t];
      Mz[t] = g.M[2][3 * c.k + t];
    }
  }

  __device__ __forceinline__ double diag(const double (&s)[3]) const {
    return s[0] * Kx[1] * My[1] * Mz[1] + s[1] * Mx[1] * Ky[1] * Mz[1] +
           s[2] * Mx[1] * My[1] * Kz[1];
  }

  // (A x)_node, x given by val(index); the same direction-by-direction sum as
  // Q1Node::apply_with, on differences from the node's own value
  template <class Val>
  __device__ __forceinline__ double apply_with(Val val, const double (&s)[3]) const {
    const double xc = val(n0);
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double ww = 0.0, ws = 0.0, sw = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const long long row = n0 + oz[c] + oy[b];
        double xw = 0.0, xs = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double d = val(row + ox[a]) - xc;
          xw += Mx[a] * d;
          xs += Kx[a] * d;
        }
        ww += My[b] * xw;
        ws += My[b] * xs;
        sw += Ky[b] * xw;
      }
      ax += Mz[c] * ws;
      ay += Mz[c] * sw;
      az += Kz[c] * ww;
    }
    return s[0] * ax + s[1] * ay + s[2] * az;
  }
};

// inverse diagonal of a level
__global__ void __launch_bounds__(kThreads) mg_invdiag_kernel(MgLevel g) {
  for (long long v = my_span(g).first, e = my_span(g).end; v < e; v += kThreads) {
    const TabNode node(v, g);
    const double d = node.diag(g.s);
    g.invd[v] = d > 0.0 ? 1.0 / d : 0.0;
  }
}

// pre-smoothing and residual on a coarse level: x = w D^-1 b, y = b - A x
__global__ void __launch_bounds__(kThreads)
    mg_pre_kernel(MgLevel g, const double* __restrict__ b, double* __restrict__ x,
                  double* __restrict__ y, CgCtl* ctl) {
  if (ctl->done) return;
  const double* __restrict__ invd = g.invd;
  const auto x_of = [=](long long t) { return kOmega * b[t] * invd[t]; };
  for (long long v = my_span(g).first, e = my_span(g).end; v < e; v += kThreads) {
    const TabNode node(v, g);
    const double ax = node.apply_with(x_of, g.s);
    x[v] = x_of(v);
    y[v] = b[v] - ax;
  }
}

// Level 0 (the fine grid, where nearly all the work is): the rows are the Q1
// element's (Q1Node, computed from the coordinates, no table loads), and each
// wavefront takes 62 consecutive nodes per pass with the x-neighbours from
// adjacent lanes, as in the CG's q kernel.  The trip count is the same for
// every lane of a wavefront.
constexpr int kLanesOut = 62;

struct LanePass {
  long long v;   // this lane's node (may lie outside the chunk: a neighbour)
  long long vl;  // the node it loads (v clamped to the grid)
  bool out;      // the lane produces a result for v
};
__device__ __forceinline__ LanePass lane_pass(long long first, long long end, long long n) {
  const int lane = threadIdx.x & 63;
  LanePass p;
  p.v = first - 1 + lane;
  p.vl = p.v < 0 ? 0 : (p.v < n ? p.v : n - 1);
  p.out = lane >= 1 && lane <= kLanesOut && p.v < end;
  return p;
}

// Level 0 with iter >= 0 first adds the r.r slots of the CG update (part_c),
// in the CG kernels' order, and stops the solve if ||r_iter|| meets the
// tolerance (as cg_q_kernel would one launch later), so no cycle runs after
// convergence.
__global__ void __launch_bounds__(kThreads)
    mg_pre0_kernel(MgLevel g, const double* __restrict__ b, double* __restrict__ x,
                   double* __restrict__ y, CgCtl* ctl, const double* __restrict__ rr_part,
                   long long n_parts, const double* __restrict__ bb, double rtol, double* rr_out,
                   long long iter) {
  if (ctl->done) return;
  double t[1] = {0.0};
  const long long parts = iter >= 0 ? n_parts : 0;
  for (long long j = threadIdx.x; j < parts; j += kThreads) t[0] += rr_part[j];
  block_sum(t);
  const double bbv = iter >= 0 ? *bb : 0.0;
  const double rel = bbv > 0.0 ? ::sqrt(t[0] / bbv) : 0.0;
  const bool stop = iter >= 0 && (!(rel > rtol) || ::isinf(rel));
  if (iter >= 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    *rr_out = t[0];
    if (stop) {
      ctl->iters = iter;
      ctl->done = 1;
    }
  }
  if (stop) return;
  const double* __restrict__ invd = g.invd;
  const auto x_of = [=](long long t2) { return kOmega * b[t2] * invd[t2]; };
  const long long begin = chunk_of(g) * g.chunk;
  const long long end = begin + g.chunk < g.n ? begin + g.chunk : g.n;
  for (long long first = begin + (threadIdx.x >> 6) * kLanesOut; first < end;
       first += kWaves * kLanesOut) {
    const LanePass p = lane_pass(first, end, g.n);
    const Q1Coords c = q1_coords(p.vl, g.nx, g.ny);
    const Q1Node node(c.i, c.j, c.k, g.nx, g.ny, g.nz);
    double xv;
    const double ax = node.apply_lanes(x_of, g.s, xv);
    if (p.out) {
      x[p.v] = xv;
      y[p.v] = b[p.v] - ax;
    }
  }
}

__global__ void __launch_bounds__(kThreads)
    mg_post0_kernel(MgLevel g, const double* __restrict__ b, const double* __restrict__ x,
                    double* __restrict__ out, CgCtl* ctl, double* __restrict__ rz_part) {
  if (ctl->done) return;
  double s[1] = {0.0};
  const long long begin = chunk_of(g) * g.chunk;
  const long long end = begin + g.chunk < g.n ? begin + g.chunk : g.n;
  for (long long first = begin + (threadIdx.x >> 6) * kLanesOut; first < end;
       first += kWaves * kLanesOut) {
    const LanePass p = lane_pass(first, end, g.n);
    const Q1Coords c = q1_coords(p.vl, g.nx, g.ny);
    const Q1Node node(c.i, c.j, c.k, g.nx, g.ny, g.nz);
    double xv;
    const double ax = node.apply_lanes([x](long long t2) { return x[t2]; }, g.s, xv);
    if (p.out) {
      const double z = xv + kOmega * g.invd[p.v] * (b[p.v] - ax);
      out[p.v] = z;
      s[0] += b[p.v] * z;
    }
  }
  block_sum(s);
  if (threadIdx.x == 0) rz_part[chunk_of(g)] = s[0];
}

// restriction b_c = P^T y_f: a coarse node gathers the fine nodes within one
// index of its position in each direction
struct Restrict1D {
  long long idx[3];
  double w[3];
};
__device__ __forceinline__ Restrict1D restrict_1d(long long I, long long nf, int coarsened,
                                                  const double* I0, const double* w0,
                                                  const double* w1) {
  Restrict1D r;
  const long long pos = coarsened ? (2 * I < nf - 1 ? 2 * I : nf - 1) : I;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const long long i = pos - 1 + t;
    const bool in = i >= 0 && i < nf;
    const long long ic = in ? i : pos;
    const double i0 = I0[ic];
    const double wt = (i0 == double(I)) ? w0[ic] : ((i0 + 1.0 == double(I)) ? w1[ic] : 0.0);
    r.idx[t] = ic;
    r.w[t] = in ? wt : 0.0;
  }
  return r;
}

__global__ void __launch_bounds__(kThreads)
    mg_restrict_kernel(MgLevel f, MgLevel c, const double* __restrict__ y, double* __restrict__ bc,
                       CgCtl* ctl) {
  if (ctl->done) return;
  for (long long v = my_span(c).first, e = my_span(c).end; v < e; v += kThreads) {
    const Q1Coords q = q1_coords(v, c.nx, c.ny);
    const Restrict1D rx = restrict_1d(q.i, f.nx, f.coarsened[0], f.I0[0], f.w0[0], f.w1[0]);
    const Restrict1D ry = restrict_1d(q.j, f.ny, f.coarsened[1], f.I0[1], f.w0[1], f.w1[1]);
    const Restrict1D rz = restrict_1d(q.k, f.nz, f.coarsened[2], f.I0[2], f.w0[2], f.w1[2]);
    double acc = 0.0;
#pragma unroll
    for (int tz = 0; tz < 3; ++tz) {
#pragma unroll
      for (int ty = 0; ty < 3; ++ty) {
        const double wyz = ry.w[ty] * rz.w[tz];
        const long long row = f.nx * (ry.idx[ty] + f.ny * rz.idx[tz]);
        double sx = 0.0;
#pragma unroll
        for (int tx = 0; tx < 3; ++tx) sx += rx.w[tx] * y[row + rx.idx[tx]];
        acc += wyz * sx;
      }
    }
    bc[v] = acc;
  }
}

// prolongation and correction x_f += P x_c: a fine node interpolates from the
// (up to) 2 coarse nodes around it in each direction
__global__ void __launch_bounds__(kThreads)
    mg_prolong_kernel(MgLevel f, MgLevel c, const double* __restrict__ xc, double* __restrict__ x,
                      CgCtl* ctl) {
  if (ctl->done) return;
  for (long long v = my_span(f).first, e = my_span(f).end; v < e; v += kThreads) {
    const Q1Coords q = q1_coords(v, f.nx, f.ny);
    long long ix[2], iy[2], iz[2];
    double wx[2], wy[2], wz[2];
    const long long i0 = (long long)f.I0[0][q.i], j0 = (long long)f.I0[1][q.j],
                    k0 = (long long)f.I0[2][q.k];
    ix[0] = i0;
    ix[1] = i0 + 1 < c.nx ? i0 + 1 : i0;
    iy[0] = j0;
    iy[1] = j0 + 1 < c.ny ? j0 + 1 : j0;
    iz[0] = k0;
    iz[1] = k0 + 1 < c.nz ? k0 + 1 : k0;
    wx[0] = f.w0[0][q.i];
    wx[1] = i0 + 1 < c.nx ? f.w1[0][q.i] : 0.0;
    wy[0] = f.w0[1][q.j];
    wy[1] = j0 + 1 < c.ny ? f.w1[1][q.j] : 0.0;
    wz[0] = f.w0[2][q.k];
    wz[1] = k0 + 1 < c.nz ? f.w1[2][q.k] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2)
          acc += wx[c2] * wy[b2] * wz[a] * xc[ix[c2] + c.nx * (iy[b2] + c.ny * iz[a])];
    x[v] += acc;
  }
}

// post-smoothing: out = x + w D^-1 (b - A x); on level 0 (rz_part != null)
// also the block's part of b.out (r.z) into rz_part
__global__ void __launch_bounds__(kThreads)
    mg_post_kernel(MgLevel g, const double* __restrict__ b, const double* __restrict__ x,
                   double* __restrict__ out, CgCtl* ctl, double* __restrict__ rz_part) {
  if (ctl->done) return;
  double s[1] = {0.0};
  for (long long v = my_span(g).first, e = my_span(g).end; v < e; v += kThreads) {
    const TabNode node(v, g);
    const double ax = node.apply_with([x](long long t) { return x[t]; }, g.s);
    const double z = x[v] + kOmega * g.invd[v] * (b[v] - ax);
    out[v] = z;
    s[0] += b[v] * z;
  }
  if (rz_part) {
    block_sum(s);
    if (threadIdx.x == 0) rz_part[chunk_of(g)] = s[0];
  }
}

// coarsest level: x = Ainv b with the host's dense inverse (row-major, n x n);
// one wavefront per row, the lanes stride over the columns
__global__ void __launch_bounds__(kThreads)
    mg_coarse_solve_kernel(MgLevel g, const double* __restrict__ Ainv,
                           const double* __restrict__ b, double* __restrict__ x, CgCtl* ctl) {
  if (ctl->done) return;
  const long long row = (long long)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (row >= g.n) return;  // whole wavefronts
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  for (long long col = lane; col < g.n; col += 64) acc += Ainv[row * g.n + col] * b[col];
  acc = wave_sum_d(acc);
  if (lane == 0) x[row] = acc;
}

}  // namespace

namespace {

void launch_shape(MgLevel& g) {
  const long long want = std::min<long long>(kMaxBlocks, (g.n + kThreads - 1) / kThreads);
  g.nb = (want + kXcds - 1) / kXcds * kXcds;
  g.chunk = (g.n + g.nb - 1) / g.nb;
}

}  // namespace

MgLevels mg_bind(const MgPlan& p, const double sie[3], double* region) {
  MgLevels L;
  L.count = p.levels;
  L.coarse_inverse = region + p.off_inv;
  double* tab = region;
  double* vec = region + p.table_doubles;
  for (int l = 0; l < p.levels; ++l) {
    MgLevel& g = L.lv[l];
    g.nx = p.dims[l][0];
    g.ny = p.dims[l][1];
    g.nz = p.dims[l][2];
    g.n = g.nx * g.ny * g.nz;
    launch_shape(g);
    for (int a = 0; a < 3; ++a) {
      g.s[a] = sie[a];
      g.K[a] = tab + p.off_K[l][a];
      g.M[a] = tab + p.off_M[l][a];
      const bool has_next = l + 1 < p.levels;
      g.I0[a] = has_next ? tab + p.off_P[l][a] : nullptr;
      g.w0[a] = has_next ? g.I0[a] + p.dims[l][a] : nullptr;
      g.w1[a] = has_next ? g.w0[a] + p.dims[l][a] : nullptr;
      g.coarsened[a] = has_next && p.dims[l + 1][a] != p.dims[l][a] ? 1 : 0;
    }
    const size_t n = size_t((g.n + 31) / 32 * 32);
    g.invd = vec;
    vec += n;
    if (l == 0) {
      g.x = g.y = g.b = nullptr;
    } else {
      g.x = vec;
      g.y = vec + n;
      g.b = vec + 2 * n;
      vec += 3 * n;
    }
  }
  return L;
}

hipError_t mg_setup(const MgLevels& L, hipStream_t st) {
  for (int l = 0; l < L.count; ++l)
    hipLaunchKernelGGL(mg_invdiag_kernel, dim3(unsigned(L.lv[l].nb)), dim3(kThreads), 0, st,
                       L.lv[l]);
  return hipGetLastError();
}

hipError_t mg_apply(const MgLevels& L, const double* r, double* z, double* xtmp, double* ytmp,
                    CgCtl* ctl, double* rz_part, const double* rr_part, long long n_parts,
                    const double* bb, double rtol, double* rr_out, long long iter,
                    hipStream_t st) {
  const dim3 blk(kThreads);
  // down: level l smooths its right-hand side b_l into x_l, restricts the residual
  for (int l = 0; l + 1 < L.count; ++l) {
    const MgLevel& g = L.lv[l];
    const double* b = l == 0 ? r : g.b;
    double* x = l == 0 ? xtmp : g.x;
    double* y = l == 0 ? ytmp : g.y;
    if (l == 0)
      hipLaunchKernelGGL(mg_pre0_kernel, dim3(unsigned(g.nb)), blk, 0, st, g, b, x, y, ctl,
                         rr_part, n_parts, bb, rtol, rr_out, iter);
    else
      hipLaunchKernelGGL(mg_pre_kernel, dim3(unsigned(g.nb)), blk, 0, st, g, b, x, y, ctl);
    hipLaunchKernelGGL(mg_restrict_kernel, dim3(unsigned(L.lv[l + 1].nb)), blk, 0, st, g,
                       L.lv[l + 1], (const double*)y, L.lv[l + 1].b, ctl);
  }
  const MgLevel& c = L.lv[L.count - 1];
  hipLaunchKernelGGL(mg_coarse_solve_kernel, dim3(unsigned((c.n + kWaves - 1) / kWaves)), blk, 0,
                     st, c, (const double*)L.coarse_inverse, (const double*)c.b, c.x, ctl);
  // up: prolongate the coarse result, then post-smooth into y, the residual's
  // buffer, no longer needed (level 0: into z)
  const double* coarse_result = c.x;
  for (int l = L.count - 2; l >= 0; --l) {
    const MgLevel& g = L.lv[l];
    const double* b = l == 0 ? r : g.b;
    double* x = l == 0 ? xtmp : g.x;
    double* out = l == 0 ? z : g.y;
    hipLaunchKernelGGL(mg_prolong_kernel, dim3(unsigned(g.nb)), blk, 0, st, g, L.lv[l + 1],
                       coarse_result, x, ctl);
    if (l == 0)
      hipLaunchKernelGGL(mg_post0_kernel, dim3(unsigned(g.nb)), blk, 0, st, g, b,
                         (const double*)x, out, ctl, rz_part);
    else
      hipLaunchKernelGGL(mg_post_kernel, dim3(unsigned(g.nb)), blk, 0, st, g, b,
                         (const double*)x, out, ctl, (double*)nullptr);
    coarse_result = out;
  }
  return hipGetLastError();
}

}  // namespace ionic
