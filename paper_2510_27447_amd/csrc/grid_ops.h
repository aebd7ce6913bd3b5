// Kernels on structured grids of nodes: the diffusion current (diffusion.hip)
// and the elliptic solve of the partitioned step with its current
// (elliptic.hip).  Host-side launchers; the step kernels do not use these.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace ionic {

// Diffusion current on a structured grid (diffusion.hip).
hipError_t diffusion_launch(const double* V, long long nx, long long ny, long long nz, double h,
                            double sigma, double* out, hipStream_t st);

// Elliptic equation A_ie u = -A_i v by Jacobi-preconditioned conjugate
// gradients and the current -M_L^{-1} A_i (v + u) (elliptic.hip).  Grids have
// fewer than 2^31 nodes.
struct CgParams {
  long long nx, ny, nz;
  long long n;      // nx ny nz
  long long nb;     // blocks of every launch (a multiple of 8), one partial sum each
  long long chunk;  // consecutive nodes per block
  double si[3];     // sigma_i per direction
  double sie[3];    // sigma_i + sigma_e per direction
  double rtol;      // stop when ||r|| <= rtol ||b||
};
CgParams cg_params(long long nx, long long ny, long long nz);

// Device-side control of one solve: the first iteration count k with
// ||r_k|| <= rtol ||b|| (done = 1 from then on; every later iteration launch
// returns at once).
struct CgCtl {
  int done;
  int reserved;
  long long iters;
};

// Work vectors and scalars of one solve, carved from one device buffer.
// Scalars: [0] b.b, [1], [2] the lumped-mass sums of the mean, [3..4] CgCtl,
// then from index 8 the triple (r.z, p.q, r.r) of every iteration k.
struct CgWork {
  double *r, *z, *q;                 // n each
  double* p[2];                      // n each: p_k is p[k & 1]
  double* u_prev;                    // n: the previous step's u (time loops)
  double *part_a, *part_b, *part_c;  // one partial sum per block each
  double* sc;
  __host__ __device__ double* p_k(long long k) const { return p[k & 1]; }
  __host__ __device__ double* bb() { return sc; }
  __host__ __device__ double* mean_sums() { return sc + 1; }
  __host__ __device__ CgCtl* ctl() { return reinterpret_cast<CgCtl*>(sc + 3); }
  __host__ __device__ double* rz(long long k) { return sc + 8 + 3 * k; }
  __host__ __device__ double* pq(long long k) { return sc + 8 + 3 * k + 1; }
  __host__ __device__ double* rr(long long k) { return sc + 8 + 3 * k + 2; }
  static size_t bytes(long long n, long long n_parts, int max_iter) {
    return sizeof(double) * size_t(6 * n + 3 * n_parts + 8 + 3 * (max_iter + 2));
  }
};
static_assert(sizeof(CgCtl) == 2 * sizeof(double), "CgCtl occupies scalars 3 and 4");
// r, z, p from the guess U and the field V; r.z, b.b, r.r; done if already converged
hipError_t cg_start(const CgParams& c, const double* V, const double* U, CgWork& w,
                    hipStream_t st);
// iteration k (k = 0, 1, ...): no work once done; the test of ||r_k|| runs at
// the start of iteration k
hipError_t cg_iteration(const CgParams& c, int k, double* U, CgWork& w, hipStream_t st);
// after the last iteration launch (k_end launched iterations): the scalars and
// the test of ||r_(k_end)|| if the solve has not stopped
hipError_t cg_end(const CgParams& c, int k_end, CgWork& w, hipStream_t st);
hipError_t cg_remove_mean(const CgParams& c, double* U, CgWork& w, hipStream_t st);
// initial guess of a time loop's next solve: with first, u_prev = U (the guess
// stays U); otherwise U = 2 U - u_prev and u_prev = the old U (linear
// extrapolation from the last two solutions)
hipError_t cg_extrapolate(const CgParams& c, double* U, CgWork& w, bool first, hipStream_t st);
hipError_t bidomain_current(const CgParams& c, const double* V, const double* U, double h,
                            double* out, hipStream_t st);

}  // namespace ionic
