// Kernels on structured grids of nodes: the diffusion current (diffusion.hip)
// and the elliptic solve of the partitioned step with its current
// (elliptic.hip).  Host-side launchers; the step kernels do not use these.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

namespace ionic {

// Diffusion current on a structured grid (diffusion.hip).
hipError_t diffusion_launch(const double* V, long long nx, long long ny, long long nz, double h,
                            double sigma, double* out, hipStream_t st);

// Elliptic equation A_ie u = -A_i v by preconditioned conjugate gradients
// and the current -M_L^{-1} A_i (v + u) (elliptic.hip).  Grids have fewer
// than 2^31 nodes.
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
  double* u_prev;                    // n: u of the previous step (time loops)
  double* u_prev2;                   // n: u of the step before it
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
    return sizeof(double) * size_t(7 * n + 3 * n_parts + 8 + 3 * (max_iter + 2));
  }
};
static_assert(sizeof(CgCtl) == 2 * sizeof(double), "CgCtl occupies scalars 3 and 4");
// r (and with jacobi z) from the guess U and the field V, and the block parts
// of b.b, r.z (jacobi) and r.r; cg_start_sums then forms the scalars of
// iteration 0 (with the multigrid preconditioner after z and its r.z parts
// come from mg_apply) and tests convergence
hipError_t cg_start(const CgParams& c, const double* V, const double* U, CgWork& w, bool jacobi,
                    hipStream_t st);
hipError_t cg_start_sums(const CgParams& c, CgWork& w, hipStream_t st);
// iteration k (k = 0, 1, ...): no work once done; the test of ||r_k|| runs at
// the start of iteration k; without jacobi, z and its r.z parts must come from
// mg_apply after each iteration
hipError_t cg_iteration(const CgParams& c, int k, double* U, CgWork& w, bool jacobi,
                        hipStream_t st);
// after the last iteration launch (k_end launched iterations): the scalars and
// the test of ||r_(k_end)|| if the solve has not stopped
hipError_t cg_end(const CgParams& c, int k_end, CgWork& w, hipStream_t st);
hipError_t cg_remove_mean(const CgParams& c, double* U, CgWork& w, hipStream_t st);
// Geometric multigrid preconditioner (multigrid.hip): one symmetric V(1,1)
// cycle on the tensor-product hierarchy of the grid.
constexpr int kMgMaxLevels = 16;
struct MgLevel {
  long long nx, ny, nz, n;
  long long nb, chunk;       // launch shape, as CgParams
  double s[3];               // sigma_i + sigma_e per direction
  const double* K[3];        // 1D stiffness rows, 3 per index (offsets -1, 0, +1)
  const double* M[3];        // 1D mass rows
  const double* I0[3];       // prolongation from the next level: fine index i
  const double* w0[3];       //   takes w0 x_c[I0] + w1 x_c[I0 + 1]
  const double* w1[3];
  int coarsened[3];          // the next level halves this direction
  double *invd, *x, *y, *b;  // n each (x, y, b on levels >= 1 only)
};
struct MgLevels {
  int count;
  MgLevel lv[kMgMaxLevels];
  const double* coarse_inverse;  // dense inverse of the coarsest level (row-major)
};
struct MgPlan {
  int levels;
  bool usable;  // at least two levels and a coarsest level of at most 512 nodes
  long long dims[kMgMaxLevels][3];
  size_t off_K[kMgMaxLevels][3], off_M[kMgMaxLevels][3], off_P[kMgMaxLevels][3];
  size_t off_inv;  // the coarsest level's dense inverse
  size_t table_doubles, vector_doubles;
};
MgPlan mg_plan(long long nx, long long ny, long long nz);
size_t mg_doubles(const MgPlan& p);  // device doubles of tables and vectors (0 if unusable)
std::vector<double> mg_tables(const MgPlan& p);
// fills the coarsest inverse of tables for the conductivities s
void mg_coarse_inverse(const MgPlan& p, const double s[3], std::vector<double>& tables);
MgLevels mg_bind(const MgPlan& p, const double sie[3], double* region);
hipError_t mg_setup(const MgLevels& L, hipStream_t st);
// z = cycle(r), and the block parts of r.z into rz_part (the CG's layout);
// xtmp, ytmp: n doubles each, free for the call.  With iter >= 0 the first
// launch first tests ||r_iter|| from the r.r parts (rr_part, n_parts) and
// stops the solve (ctl) if it meets rtol, recording r.r at rr_out.
hipError_t mg_apply(const MgLevels& L, const double* r, double* z, double* xtmp, double* ytmp,
                    CgCtl* ctl, double* rz_part, const double* rr_part, long long n_parts,
                    const double* bb, double rtol, double* rr_out, long long iter,
                    hipStream_t st);

// initial guess of a time loop's next solve from the last solutions (U holds
// the last one): order 0 keeps U, order 1 takes 2 U - u_prev (linear), order 2
// 3 U - 3 u_prev + u_prev2 (quadratic extrapolation); u_prev2 and u_prev then
// move one step on (u_prev = the old U)
hipError_t cg_extrapolate(const CgParams& c, double* U, CgWork& w, int order, hipStream_t st);
hipError_t bidomain_current(const CgParams& c, const double* V, const double* U, double h,
                            double* out, hipStream_t st);

}  // namespace ionic
