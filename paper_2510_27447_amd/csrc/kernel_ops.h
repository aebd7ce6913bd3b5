// Type-erased launch table of one cell model: the host library dispatches on
// (model, precision, node count) at run time through these entries; each
// model's kernels are instantiated in a translation unit of their own.
#pragma once

#include <hip/hip_runtime.h>

#include "sdc_kernel.h"

namespace ionic {

struct LaunchCommon {
  double S[kMaxNodes - 1][kMaxNodes];
  double dc[kMaxNodes - 1];
  double tol;
  int maxit;
  int n_sims;
  AdaptCtl* ctl;
  ErrSlot* err;
  void* state_alt;
  SimDesc sims[kMaxBatch];
};

using SdcLaunch = hipError_t (*)(int M, const void* params, const LaunchCommon& c, int blocks,
                                 hipStream_t st);

struct ModelOps {
  int n_states;
  int n_fp64;  // leading planes in double under the mixed layout
  int n_params;
  const char* const* param_names;
  const double* param_defaults;  // n_params (+ trailing fixed entries)
  int n_raw;                     // length of the raw parameter vector
  const char* const* state_names;
  size_t params_bytes[2];        // sizeof(Params<double>), sizeof(Params<float>)
  void (*derive)(const double* raw, void* p64, void* p32);
  // fused step kernels, [precision policy: double, mixed][predictor: Newton, ROS2, Rush-Larsen]
  SdcLaunch sdc[2][3];
  hipError_t (*pack)(int prec, const double* src, long long ld, void* state, long long stride,
                     long long first, long long count, hipStream_t st);
  hipError_t (*unpack)(int prec, const void* state, long long stride, long long first,
                       long long count, double* dst, long long ld, hipStream_t st);
  hipError_t (*steady)(int prec, const void* params, void* state, long long stride, long long n,
                       hipStream_t st);
  hipError_t (*debug_jac)(int prec, const void* params, const void* state, long long stride,
                          long long v, double stim, double diff, double* out, hipStream_t st);
};

// The step kernels of the cell models live in translation units of their own
// (one per model, precision policy and predictor) so they compile in
// parallel.
hipError_t tt06_sdc_fp64_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_fp64_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_mixed_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_mixed_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_fp64_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_fp64_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_mixed_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_mixed_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_fp64_rl(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_mixed_rl(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_fp64_rl(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_mixed_rl(int, const void*, const LaunchCommon&, int, hipStream_t);

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
    return sizeof(double) * size_t(5 * n + 3 * n_parts + 8 + 3 * (max_iter + 2));
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
hipError_t bidomain_current(const CgParams& c, const double* V, const double* U, double h,
                            double* out, hipStream_t st);

// Adaptive step control (control.hip).
hipError_t adapt_init(AdaptCtl* c, ErrSlot* err, double t0, double t_end, double dt_init,
                      double dt_max, double tol, double dt_min, double t_on, double t_off,
                      long long max_attempts, hipStream_t st);
hipError_t adapt_control(AdaptCtl* c, ErrSlot* err, double* history, long long history_len,
                         hipStream_t st);

extern const ModelOps kOpsLR91;
extern const ModelOps kOpsTT06;
extern const ModelOps kOpsTestLinear;
extern const ModelOps kOpsTestLogistic;

}  // namespace ionic
