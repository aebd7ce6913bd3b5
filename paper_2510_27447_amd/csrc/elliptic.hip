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
// conjugate gradients with the Jacobi preconditioner, warm-started from the
// previous step's u.
//
// Every kernel runs one thread per node on a 3D launch (64 threads along x).
// Dot products are reduced deterministically: each block writes one partial
// sum (a fixed butterfly over its wavefront), and reduce_kernel sums the
// partials in a fixed order, so a solve gives the same bits every time.  The
// scalars of iteration k live at their own addresses (rz[k], pq[k], rr[k]),
// so no kernel writes a scalar that another block of the same launch reads.
#include "kernel_ops.h"
#include "stencil.h"

namespace ionic {

namespace {

constexpr int kBlk = 64;
constexpr int kRedBlock = 256;

__device__ __forceinline__ double wave_sum_d(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

struct Launch3 {
  long long nx, ny, nz;
  __device__ __forceinline__ long long block_id() const {
    const long long gx = (nx + kBlk - 1) / kBlk;
    return blockIdx.x + gx * ((long long)blockIdx.y + ny * (long long)blockIdx.z);
  }
};

__device__ __forceinline__ void put_partial(double a, double* part, long long bid) {
  const double s = wave_sum_d(a);
  if (threadIdx.x == 0) part[bid] = s;
}

__global__ void __launch_bounds__(kBlk)
    cg_start_kernel(const double* __restrict__ V, const double* __restrict__ U, CgParams c,
                    double* __restrict__ r, double* __restrict__ z, double* __restrict__ p,
                    double* __restrict__ part_a, double* __restrict__ part_b,
                    double* __restrict__ part_c) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  const bool on = i < c.nx;
  double rz = 0.0, bb = 0.0, rr = 0.0;
  if (on) {
    const Q1Node node(i, blockIdx.y, blockIdx.z, c.nx, c.ny, c.nz);
    const long long n = node.index();
    const double b = -node.apply(V, c.si);
    const double rn = b - node.apply(U, c.sie);
    const double zn = rn / node.diag(c.sie);
    r[n] = rn;
    z[n] = zn;
    p[n] = zn;
    rz = rn * zn;
    bb = b * b;
    rr = rn * rn;
  }
  const long long bid = Launch3{c.nx, c.ny, c.nz}.block_id();
  put_partial(rz, part_a, bid);
  put_partial(bb, part_b, bid);
  put_partial(rr, part_c, bid);
}

__global__ void __launch_bounds__(kBlk)
    cg_q_kernel(const double* __restrict__ p, CgParams c, double* __restrict__ q,
                double* __restrict__ part_a) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  double pq = 0.0;
  if (i < c.nx) {
    const Q1Node node(i, blockIdx.y, blockIdx.z, c.nx, c.ny, c.nz);
    const long long n = node.index();
    const double qn = node.apply(p, c.sie);
    q[n] = qn;
    pq = p[n] * qn;
  }
  put_partial(pq, part_a, Launch3{c.nx, c.ny, c.nz}.block_id());
}

__global__ void __launch_bounds__(kBlk)
    cg_update_kernel(CgParams c, const double* __restrict__ rz_k, const double* __restrict__ pq_k,
                     double* __restrict__ U, double* __restrict__ r, double* __restrict__ z,
                     const double* __restrict__ p, const double* __restrict__ q,
                     double* __restrict__ part_a, double* __restrict__ part_b) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  const double pq = *pq_k;
  const double alpha = pq != 0.0 ? *rz_k / pq : 0.0;
  double rz = 0.0, rr = 0.0;
  if (i < c.nx) {
    const Q1Node node(i, blockIdx.y, blockIdx.z, c.nx, c.ny, c.nz);
    const long long n = node.index();
    U[n] += alpha * p[n];
    const double rn = r[n] - alpha * q[n];
    const double zn = rn / node.diag(c.sie);
    r[n] = rn;
    z[n] = zn;
    rz = rn * zn;
    rr = rn * rn;
  }
  const long long bid = Launch3{c.nx, c.ny, c.nz}.block_id();
  put_partial(rz, part_a, bid);
  put_partial(rr, part_b, bid);
}

__global__ void __launch_bounds__(kBlk)
    cg_dir_kernel(CgParams c, const double* __restrict__ rz_k, const double* __restrict__ rz_k1,
                  const double* __restrict__ z, double* __restrict__ p) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  if (i >= c.nx) return;
  const double rz = *rz_k;
  const double beta = rz != 0.0 ? *rz_k1 / rz : 0.0;
  const long long n = i + c.nx * ((long long)blockIdx.y + c.ny * (long long)blockIdx.z);
  p[n] = z[n] + beta * p[n];
}

__global__ void __launch_bounds__(kBlk)
    mean_parts_kernel(const double* __restrict__ U, CgParams c, double* __restrict__ part_a,
                      double* __restrict__ part_b) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  double mu = 0.0, m = 0.0;
  if (i < c.nx) {
    const Q1Node node(i, blockIdx.y, blockIdx.z, c.nx, c.ny, c.nz);
    m = node.mass();
    mu = m * U[node.index()];
  }
  const long long bid = Launch3{c.nx, c.ny, c.nz}.block_id();
  put_partial(mu, part_a, bid);
  put_partial(m, part_b, bid);
}

__global__ void __launch_bounds__(kBlk)
    sub_mean_kernel(CgParams c, const double* __restrict__ sums, double* __restrict__ U) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  if (i >= c.nx) return;
  const double mean = sums[0] / sums[1];
  U[i + c.nx * ((long long)blockIdx.y + c.ny * (long long)blockIdx.z)] -= mean;
}

__global__ void __launch_bounds__(kBlk)
    bidomain_current_kernel(const double* __restrict__ V, const double* __restrict__ U, CgParams c,
                            double inv_h2, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  if (i >= c.nx) return;
  const Q1Node node(i, blockIdx.y, blockIdx.z, c.nx, c.ny, c.nz);
  out[node.index()] = -inv_h2 * (node.apply(V, c.si) + node.apply(U, c.si)) / node.mass();
}

// one block: out_a = sum of a[0..n), out_b = sum of b[0..n) (b may be null),
// in a fixed order (thread t takes t, t + 256, ...; then a tree in LDS)
__global__ void __launch_bounds__(kRedBlock)
    reduce_kernel(const double* __restrict__ a, const double* __restrict__ b, long long n,
                  double* __restrict__ out_a, double* __restrict__ out_b) {
  __shared__ double sa[kRedBlock], sb[kRedBlock];
  double x = 0.0, y = 0.0;
  for (long long t = threadIdx.x; t < n; t += kRedBlock) {
    x += a[t];
    if (b) y += b[t];
  }
  sa[threadIdx.x] = x;
  sb[threadIdx.x] = y;
  __syncthreads();
  for (int w = kRedBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out_a = sa[0];
    if (b) *out_b = sb[0];
  }
}

dim3 grid3(const CgParams& c) {
  return dim3(unsigned((c.nx + kBlk - 1) / kBlk), unsigned(c.ny), unsigned(c.nz));
}

}  // namespace

long long cg_blocks(long long nx, long long ny, long long nz) {
  return (nx + kBlk - 1) / kBlk * ny * nz;
}

hipError_t cg_start(const CgParams& c, const double* V, const double* U, CgWork& w,
                    hipStream_t st) {
  hipLaunchKernelGGL(cg_start_kernel, grid3(c), dim3(kBlk), 0, st, V, U, c, w.r, w.z, w.p,
                     w.part_a, w.part_b, w.part_c);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedBlock), 0, st, w.part_a, w.part_b,
                     w.n_parts, w.rz(0), w.bb());
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedBlock), 0, st, w.part_c,
                     (const double*)nullptr, w.n_parts, w.rr(0), (double*)nullptr);
  return hipGetLastError();
}

hipError_t cg_iteration(const CgParams& c, int k, double* U, CgWork& w, hipStream_t st) {
  hipLaunchKernelGGL(cg_q_kernel, grid3(c), dim3(kBlk), 0, st, w.p, c, w.q, w.part_a);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedBlock), 0, st, w.part_a,
                     (const double*)nullptr, w.n_parts, w.pq(k), (double*)nullptr);
  hipLaunchKernelGGL(cg_update_kernel, grid3(c), dim3(kBlk), 0, st, c, w.rz(k), w.pq(k), U, w.r,
                     w.z, w.p, w.q, w.part_a, w.part_b);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedBlock), 0, st, w.part_a, w.part_b,
                     w.n_parts, w.rz(k + 1), w.rr(k + 1));
  hipLaunchKernelGGL(cg_dir_kernel, grid3(c), dim3(kBlk), 0, st, c, w.rz(k), w.rz(k + 1), w.z,
                     w.p);
  return hipGetLastError();
}

hipError_t cg_remove_mean(const CgParams& c, double* U, CgWork& w, hipStream_t st) {
  hipLaunchKernelGGL(mean_parts_kernel, grid3(c), dim3(kBlk), 0, st, U, c, w.part_a, w.part_b);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedBlock), 0, st, w.part_a, w.part_b,
                     w.n_parts, w.mean_sums(), w.mean_sums() + 1);
  hipLaunchKernelGGL(sub_mean_kernel, grid3(c), dim3(kBlk), 0, st, c, w.mean_sums(), U);
  return hipGetLastError();
}

hipError_t bidomain_current(const CgParams& c, const double* V, const double* U, double h,
                            double* out, hipStream_t st) {
  hipLaunchKernelGGL(bidomain_current_kernel, grid3(c), dim3(kBlk), 0, st, V, U, c,
                     1.0 / (h * h), out);
  return hipGetLastError();
}

}  // namespace ionic
