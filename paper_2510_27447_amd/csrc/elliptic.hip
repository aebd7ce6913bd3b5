// The elliptic equation of the partitioned strategy and the parabolic current
// that uses its solution (paper section 3.1, equations semi-elliptic and
// semi-parabolic; section 3.3.2, Algorithm 2, first box: solve for u with v
// fixed), on a structured grid with diagonal conductivity tensors:
//
//   A_ie u = -A_i v,    A_i: sigma_i,  A_ie: sigma_i + sigma_e,
//   I_diff = -M_L^{-1} A_i (v + u).
//
// A_ie is symmetric positive semi-definite with the constants as null space
// (Neumann boundaries) and -A_i v sums to zero, so conjugate gradients
// converge on it; the lumped-mass mean of u is then set to zero.  The paper
// solves this system with BiCGSTAB and algebraic multigrid; here it is
// conjugate gradients, preconditioned by the geometric multigrid cycle of
// multigrid.hip (or by Jacobi on grids too small for a hierarchy).
//
// Launch shape: nb blocks of 256 threads (nb a multiple of 8, at most 1024);
// block L owns the nodes [L chunk, (L + 1) chunk), its threads stride through
// them.  Blocks are dispatched to the 8 XCDs in turn (block b to XCD b mod 8),
// so block b takes the chunk L = (b mod 8) nb/8 + b/8: each XCD works on one
// contiguous eighth of the grid, and the stencil's neighbours (one x-row or
// one xy-plane away) mostly sit in the same XCD's L2.
//
// Dot products are reduced in a fixed order and without any synchronisation
// between blocks: each block sums its threads (wavefront butterfly, then its 4
// wavefronts in order) into its own slot, and every block of the next launch
// that needs the total adds the nb slots itself, in the same fixed order, so
// all blocks get the same bits and a solve is reproducible bit for bit.  The
// kernels that consume a total also record it (block 0) in the scalars of
// iteration k (rz[k], pq[k], rr[k]).
//
// An iteration is two launches, cg_q_kernel (direction and q = A_ie p) and
// cg_update_kernel (u, r; z with Jacobi), then the multigrid cycle for z.
// The first launch of iteration k (the cycle's, with multigrid) adds the r.r
// slots of iteration k-1 and tests ||r_k|| <= rtol ||b||: done is set there,
// after which every queued launch returns at once; the host only reads the
// flag between batches of launches.
#include "grid_ops.h"
#include "stencil.h"

namespace ionic {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlocks = 1024;
constexpr int kXcds = 8;

__device__ __forceinline__ double wave_sum_d(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// chunk owned by this block (see the launch shape above)
__device__ __forceinline__ long long chunk_id(const CgParams& c) {
  const long long b = blockIdx.x;
  return (b % kXcds) * (c.nb / kXcds) + b / kXcds;
}

// Sum of each of NV per-thread values over the block, fixed order; the totals
// in every thread.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double lds[NV][kWaves];
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = wave_sum_d(v[a]);
  __syncthreads();  // a previous call's readers are done with lds
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) lds[a][threadIdx.x >> 6] = v[a];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = (lds[a][0] + lds[a][1]) + (lds[a][2] + lds[a][3]);
}

// this block's sums into slot chunk_id of part[a]
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

// totals of the nb slots of each part[a] (written by an earlier launch), the
// same fixed order in every block; the totals in every thread
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

// convergence after iteration k from r.r and b.b (the host's test)
__device__ __forceinline__ bool converged(const CgParams& c, double rr, double bb) {
  const double rel = bb > 0.0 ? ::sqrt(rr / bb) : 0.0;
  return !(rel > c.rtol) || ::isinf(rel);
}

// this thread's first node and the end of the block's chunk; the thread takes
// every kThreads-th node from first
struct Nodes {
  long long first, end;
};
__device__ __forceinline__ Nodes my_nodes(const CgParams& c) {
  const long long begin = chunk_id(c) * c.chunk, end = begin + c.chunk;
  return {begin + threadIdx.x, end < c.n ? end : c.n};
}

// Wavefront passes over consecutive nodes for the lane-shuffle stencil
// (Q1Node::apply_lanes): each pass covers 62 nodes (lanes 1..62; lanes 0 and
// 63 hold the nodes on either side).  The trip count is the same for every
// lane of a wavefront.
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

// r = b - A_ie U with b = -A_i V; with the Jacobi preconditioner also z = r /
// diag (the multigrid cycle forms z otherwise); block parts of b.b (part_a),
// r.z (part_b, Jacobi only) and r.r (part_c)
__global__ void __launch_bounds__(kThreads)
    cg_start_kernel(const double* __restrict__ V, const double* __restrict__ U, CgParams c,
                    CgWork w, int jacobi) {
  // a new solve: clear the previous solve's stop flag before any launch that
  // tests it (no kernel of this launch reads it)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    w.ctl()->done = 0;
    w.ctl()->iters = 0;
  }
  double s[3] = {0.0, 0.0, 0.0};  // b.b, r.z, r.r
  const long long begin = chunk_id(c) * c.chunk;
  const long long end = begin + c.chunk < c.n ? begin + c.chunk : c.n;
  const auto v_of = [V](long long t) { return V[t]; };
  const auto u_of = [U](long long t) { return U[t]; };
  for (long long first = begin + (threadIdx.x >> 6) * kLanesOut; first < end;
       first += kWaves * kLanesOut) {
    const LanePass lp = lane_pass(first, end, c.n);
    const Q1Coords x = q1_coords(lp.vl, c.nx, c.ny);
    const Q1Node node(x.i, x.j, x.k, c.nx, c.ny, c.nz);
    double own;
    const double b = -node.apply_lanes(v_of, c.si, own);
    const double rn = b - node.apply_lanes(u_of, c.sie, own);
    if (lp.out) {
      w.r[lp.v] = rn;
      if (jacobi) {
        const double zn = rn / node.diag(c.sie);
        w.z[lp.v] = zn;
        s[1] += rn * zn;
      }
      s[0] += b * b;
      s[2] += rn * rn;
    }
  }
  if (jacobi) {
    double* const part[3] = {w.part_a, w.part_b, w.part_c};
    put_partials(s, part, c);
  } else {
    double t[2] = {s[0], s[2]};
    double* const part[2] = {w.part_a, w.part_c};
    put_partials(t, part, c);
  }
}

// one block: the scalars of the start and the test before the first iteration
__global__ void __launch_bounds__(kThreads) cg_start_sums_kernel(CgParams c, CgWork w) {
  const double* const part[3] = {w.part_a, w.part_b, w.part_c};
  double s[3];  // b.b, r.z, r.r
  total_of(part, c, s);
  if (threadIdx.x == 0) {
    *w.bb() = s[0];
    *w.rz(0) = s[1];
    *w.rr(0) = s[2];
    CgCtl* ctl = w.ctl();
    ctl->done = converged(c, s[2], s[0]) ? 1 : 0;
    ctl->reserved = 0;
    ctl->iters = 0;
  }
}

// Iteration k, first launch: the direction p_k = z_k + beta_k p_(k-1) and
// q = A_ie p_k, with the block's part of p_k.q.  For k > 0 the block first adds
// the slots of r.z and r.r left by iteration k-1 (beta_k = r_k.z_k /
// r_(k-1).z_(k-1)) and stops the solve if ||r_k|| meets the tolerance.  p_k is
// formed where it is used: the stencil reads z and p_(k-1) (two buffers, p_k
// goes to the other one), so no separate direction pass is needed.  Each
// wavefront takes 62 consecutive nodes per pass (lanes 1..62; lanes 0 and 63
// hold the nodes on either side) so the x-neighbours come from adjacent lanes
// (Q1Node::apply_lanes): 9 rows per node instead of 27 values.
__global__ void __launch_bounds__(kThreads) cg_q_kernel(CgParams c, CgWork w, long long k) {
  if (w.ctl()->done) return;
  double beta = 0.0;
  if (k > 0) {
    const double* const in[2] = {w.part_b, w.part_c};
    double t[2];  // r_k.z_k, r_k.r_k
    total_of(in, c, t);
    const bool stop = converged(c, t[1], *w.bb());
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *w.rz(k) = t[0];
      *w.rr(k) = t[1];
      if (stop) {
        w.ctl()->iters = k;
        w.ctl()->done = 1;
      }
    }
    if (stop) return;
    const double rz = *w.rz(k - 1);
    beta = rz != 0.0 ? t[0] / rz : 0.0;
  }
  const double* __restrict__ z = w.z;
  const double* __restrict__ p_old = w.p_k(k - 1);
  double* __restrict__ p_new = w.p_k(k);
  // p_0 = z_0 (p_old holds no direction yet: not read into the value)
  const bool no_prev = k == 0;
  const auto p_of = [=](long long t) { return no_prev ? z[t] : z[t] + beta * p_old[t]; };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long begin = chunk_id(c) * c.chunk;
  const long long end = begin + c.chunk < c.n ? begin + c.chunk : c.n;
  double s[1] = {0.0};  // p.q
  // the trip count is the same for every lane of a wavefront
  for (long long first = begin + wave * kLanesOut; first < end; first += kWaves * kLanesOut) {
    const long long v = first - 1 + lane;
    const long long vl = v < 0 ? 0 : (v < c.n ? v : c.n - 1);  // the node this lane loads
    const Q1Coords x = q1_coords(vl, c.nx, c.ny);
    const Q1Node node(x.i, x.j, x.k, c.nx, c.ny, c.nz);
    double pn;
    const double qn = node.apply_lanes(p_of, c.sie, pn);
    if (lane >= 1 && lane <= kLanesOut && v < end) {
      p_new[v] = pn;
      w.q[v] = qn;
      s[0] += pn * qn;
    }
  }
  double* const part[1] = {w.part_a};
  put_partials(s, part, c);
}

// u += alpha p, r -= alpha q and the block's part of r.r (part_c); with the
// Jacobi preconditioner also z = r / diag and the part of r.z (part_b)
__global__ void __launch_bounds__(kThreads)
    cg_update_kernel(CgParams c, CgWork w, long long k, double* __restrict__ U, int jacobi) {
  if (w.ctl()->done) return;
  const double* const in[1] = {w.part_a};
  double pq[1];
  total_of(in, c, pq);
  if (blockIdx.x == 0 && threadIdx.x == 0) *w.pq(k) = pq[0];
  const double alpha = pq[0] != 0.0 ? *w.rz(k) / pq[0] : 0.0;
  const double* __restrict__ p = w.p_k(k);
  double s[2] = {0.0, 0.0};  // r.z, r.r
  for (long long v = my_nodes(c).first, e = my_nodes(c).end; v < e; v += kThreads) {
    U[v] += alpha * p[v];
    const double rn = w.r[v] - alpha * w.q[v];
    w.r[v] = rn;
    s[1] += rn * rn;
    if (jacobi) {
      const Q1Coords x = q1_coords(v, c.nx, c.ny);
      const Q1Node node(x.i, x.j, x.k, c.nx, c.ny, c.nz);
      const double zn = rn / node.diag(c.sie);
      w.z[v] = zn;
      s[0] += rn * zn;
    }
  }
  if (jacobi) {
    double* const part[2] = {w.part_b, w.part_c};
    put_partials(s, part, c);
  } else {
    double t[1] = {s[1]};
    double* const part[1] = {w.part_c};
    put_partials(t, part, c);
  }
}

// one block, after the last iteration launch k_end when the solve has not
// stopped: the scalars and the test after iteration k_end
__global__ void __launch_bounds__(kThreads) cg_end_sums_kernel(CgParams c, CgWork w,
                                                               long long k_end) {
  if (w.ctl()->done) return;
  const double* const in[2] = {w.part_b, w.part_c};
  double t[2];
  total_of(in, c, t);
  if (threadIdx.x == 0) {
    *w.rz(k_end) = t[0];
    *w.rr(k_end) = t[1];
    if (converged(c, t[1], *w.bb())) {
      w.ctl()->iters = k_end;
      w.ctl()->done = 1;
    }
  }
}

__global__ void __launch_bounds__(kThreads)
    mean_parts_kernel(const double* __restrict__ U, CgParams c, CgWork w) {
  double s[2] = {0.0, 0.0};  // sum m u, sum m
  for (long long v = my_nodes(c).first, e = my_nodes(c).end; v < e; v += kThreads) {
    const Q1Coords x = q1_coords(v, c.nx, c.ny);
    const Q1Node node(x.i, x.j, x.k, c.nx, c.ny, c.nz);
    const double m = node.mass();
    s[0] += m * U[v];
    s[1] += m;
  }
  double* const part[2] = {w.part_a, w.part_b};
  put_partials(s, part, c);
}

__global__ void __launch_bounds__(kThreads)
    sub_mean_kernel(CgParams c, CgWork w, double* __restrict__ U) {
  const double* const in[2] = {w.part_a, w.part_b};
  double t[2];
  total_of(in, c, t);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    w.mean_sums()[0] = t[0];
    w.mean_sums()[1] = t[1];
  }
  const double mean = t[0] / t[1];
  for (long long v = my_nodes(c).first, e = my_nodes(c).end; v < e; v += kThreads)
    U[v] -= mean;
}

__global__ void __launch_bounds__(kThreads)
    extrapolate_kernel(CgParams c, double* __restrict__ U, double* __restrict__ u_prev,
                       double* __restrict__ u_prev2, int order) {
  for (long long v = my_nodes(c).first, e = my_nodes(c).end; v < e; v += kThreads) {
    const double u = U[v], u1 = order > 0 ? u_prev[v] : u;
    if (order == 1) U[v] = 2.0 * u - u1;
    if (order == 2) U[v] = 3.0 * (u - u1) + u_prev2[v];
    u_prev2[v] = u1;
    u_prev[v] = u;
  }
}

__global__ void __launch_bounds__(kThreads)
    bidomain_current_kernel(const double* __restrict__ V, const double* __restrict__ U, CgParams c,
                            double inv_h2, double* __restrict__ out) {
  // A_i (v + u) in one pass over the sum (applied to differences, as every row)
  const long long begin = chunk_id(c) * c.chunk;
  const long long end = begin + c.chunk < c.n ? begin + c.chunk : c.n;
  const auto vu_of = [V, U](long long t) { return V[t] + U[t]; };
  for (long long first = begin + (threadIdx.x >> 6) * kLanesOut; first < end;
       first += kWaves * kLanesOut) {
    const LanePass lp = lane_pass(first, end, c.n);
    const Q1Coords x = q1_coords(lp.vl, c.nx, c.ny);
    const Q1Node node(x.i, x.j, x.k, c.nx, c.ny, c.nz);
    double own;
    const double a = node.apply_lanes(vu_of, c.si, own);
    if (lp.out) out[lp.v] = -inv_h2 * a / node.mass();
  }
}

}  // namespace

CgParams cg_params(long long nx, long long ny, long long nz) {
  CgParams c{};
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.n = nx * ny * nz;
  const long long want = std::min<long long>(kMaxBlocks, (c.n + kThreads - 1) / kThreads);
  c.nb = (want + kXcds - 1) / kXcds * kXcds;
  c.chunk = (c.n + c.nb - 1) / c.nb;
  return c;
}

hipError_t cg_start(const CgParams& c, const double* V, const double* U, CgWork& w, bool jacobi,
                    hipStream_t st) {
  hipLaunchKernelGGL(cg_start_kernel, dim3(unsigned(c.nb)), dim3(kThreads), 0, st, V, U, c, w,
                     jacobi ? 1 : 0);
  return hipGetLastError();
}

hipError_t cg_start_sums(const CgParams& c, CgWork& w, hipStream_t st) {
  hipLaunchKernelGGL(cg_start_sums_kernel, dim3(1), dim3(kThreads), 0, st, c, w);
  return hipGetLastError();
}

hipError_t cg_iteration(const CgParams& c, int k, double* U, CgWork& w, bool jacobi,
                        hipStream_t st) {
  const dim3 g(unsigned(c.nb)), b(kThreads);
  hipLaunchKernelGGL(cg_q_kernel, g, b, 0, st, c, w, (long long)k);
  hipLaunchKernelGGL(cg_update_kernel, g, b, 0, st, c, w, (long long)k, U, jacobi ? 1 : 0);
  return hipGetLastError();
}

hipError_t cg_end(const CgParams& c, int k_end, CgWork& w, hipStream_t st) {
  if (k_end > 0)
    hipLaunchKernelGGL(cg_end_sums_kernel, dim3(1), dim3(kThreads), 0, st, c, w, (long long)k_end);
  return hipGetLastError();
}

hipError_t cg_remove_mean(const CgParams& c, double* U, CgWork& w, hipStream_t st) {
  const dim3 g(unsigned(c.nb)), b(kThreads);
  hipLaunchKernelGGL(mean_parts_kernel, g, b, 0, st, U, c, w);
  hipLaunchKernelGGL(sub_mean_kernel, g, b, 0, st, c, w, U);
  return hipGetLastError();
}

hipError_t cg_extrapolate(const CgParams& c, double* U, CgWork& w, int order, hipStream_t st) {
  hipLaunchKernelGGL(extrapolate_kernel, dim3(unsigned(c.nb)), dim3(kThreads), 0, st, c, U,
                     w.u_prev, w.u_prev2, order);
  return hipGetLastError();
}

hipError_t bidomain_current(const CgParams& c, const double* V, const double* U, double h,
                            double* out, hipStream_t st) {
  hipLaunchKernelGGL(bidomain_current_kernel, dim3(unsigned(c.nb)), dim3(kThreads), 0, st, V, U,
                     c, 1.0 / (h * h), out);
  return hipGetLastError();
}

}  // namespace ionic
