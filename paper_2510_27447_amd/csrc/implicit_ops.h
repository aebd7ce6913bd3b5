// Host launchers of the partitioned step with the parabolic term implicit
// (implicit.hip): the per-vertex block kernels of the ROS2 stages and the
// correction, elementwise kernels on state planes, and BiCGSTAB on the
// reduced system of the membrane potential.
#pragma once

#include <hip/hip_runtime.h>

#include "grid_ops.h"

namespace ionic {

// One per-vertex pass over the states X (fp64 planes, stride elements each):
// evaluate F and J (the cell model, stimulus amplitude stim when stim_on, the
// parabolic current idiff, which may be null), take the block B = I - c J and
// the right-hand side b = cf F(X) + base (base: planes, or null for 0), then
// either (expand = 0) write the Schur complement onto V and the reduced
// right-hand side to S, r (n doubles each), or (expand = 1) read the V part of
// the solution from dv and write the full solution to out (planes).
struct ImpBlock {
  const double* X;
  long long n, stride;
  const double* stim;
  int stim_on;
  const double* idiff;
  double c;
  double cf;
  const double* base;
  int expand;
  double* S;
  double* r;
  const double* dv;
  double* out;
};
// eval_float: F, J and the elimination in float (params: the model's float
// parameters), else in double (its double parameters); inputs and outputs are
// double either way.
hipError_t imp_block(int model, int eval_float, const void* params, const ImpBlock& a,
                     hipStream_t st);

// out = alpha F(X) + beta Y (planes; Y may be null when beta = 0), F evaluated
// as imp_block's
hipError_t imp_rhs(int model, int eval_float, const void* params, const double* X, long long n,
                   long long stride, const double* stim, int stim_on, const double* idiff,
                   double alpha, double beta, const double* Y, double* out, hipStream_t st);

// out = x + a y + b z over n_states planes of stride elements (z may be null)
hipError_t soa_lincomb(double* out, const double* x, double a, const double* y, double b,
                       const double* z, long long elems, hipStream_t st);

// X_next = XT + eps; the largest |X_next - XK| / max(|X_next|, scale_i) over
// the vertices and states into *change (bits of a non-negative double, raised
// with atomicMax; the caller clears it); then XK = X_next.
hipError_t imp_finish(const double* XT, const double* eps, double* XK, long long n, long long stride,
                      int n_states, const double* scale_dev, unsigned long long* change,
                      hipStream_t st);

// BiCGSTAB for (S + c M_L^{-1} A_i) x = r on the grid (A_i the Q1 stiffness of
// sigma_i, M_L the lumped mass), preconditioned by its diagonal.  Work: the
// BiCgWork vectors; the solve runs until ||r_k|| <= rtol ||r_0|| or max_iter.
struct BiCgWork {
  double* x;                                        // n: the solution (and the guess when warm)
  double *r, *rh, *p, *ph, *v, *s, *sh, *t, *dinv;  // n each
  double* part[5];                                      // nb each: r^.r, r.r, r^.v, t.s, t.t
  double* sc;  // scalars: [0] b.b, [1] rho, [2] alpha, [3] omega, [4..5] ctl, then r.r per iteration
  static size_t bytes(long long n, long long nb, int max_iter) {
    return sizeof(double) * size_t(10 * n + 5 * nb + 8 + 4 * (max_iter + 2));
  }
};
// the start of a solve; with warm != 0 from the guess already in w.x, else from zero
hipError_t bicg_start(const CgParams& c, double h, double cst, const double* S, const double* rhs,
                      BiCgWork& w, int warm, hipStream_t st);
// iteration k: no work once the device has found convergence
hipError_t bicg_iteration(const CgParams& c, double h, double cst, const double* S, int k,
                          BiCgWork& w, hipStream_t st);
// state of the solve: done flag and the iteration count at which ||r|| met rtol
struct BiCgCtl {
  int done;
  int reserved;
  long long iters;
};

}  // namespace ionic
