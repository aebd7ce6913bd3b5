// Diffusion current of the parabolic equation on a structured grid (paper
// section 3.1, equation semi-parabolic; Q1 elements, lumped mass), as the
// per-step input of the reaction stage:
//
//   I_diff = -sigma * M_L^{-1} A v,
//
// A the unit-conductivity stiffness matrix, M_L the lumped mass, homogeneous
// Neumann boundaries (natural).  The rows of A come from stencil.h.  One
// thread per node on a 1D launch (no idle lanes at the ends of x-rows); V is
// the first state plane (double in every precision layout), read through the
// L1/L2 caches for the neighbours.  The kernel moves 16 bytes per node from HBM
// (V once, I_diff once).  Grids have fewer than 2^31 nodes.
#include "grid_ops.h"
#include "stencil.h"

namespace ionic {

namespace {

constexpr int kDiffBlock = 256;

__global__ void __launch_bounds__(kDiffBlock)
    diffusion_kernel(const double* __restrict__ V, long long n, long long nx, long long ny,
                     long long nz, double sigma, double inv_h2, double* __restrict__ out) {
  const long long v = (long long)blockIdx.x * kDiffBlock + threadIdx.x;
  if (v >= n) return;
  const Q1Coords x = q1_coords(v, nx, ny);
  const Q1Node node(x.i, x.j, x.k, nx, ny, nz);
  const double s[3] = {sigma, sigma, sigma};
  out[v] = -inv_h2 * node.apply(V, s) / node.mass();
}

}  // namespace

hipError_t diffusion_launch(const double* V, long long nx, long long ny, long long nz, double h,
                            double sigma, double* out, hipStream_t st) {
  const long long n = nx * ny * nz;
  if (n >= (1ll << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(diffusion_kernel, dim3(unsigned((n + kDiffBlock - 1) / kDiffBlock)),
                     dim3(kDiffBlock), 0, st, V, n, nx, ny, nz, sigma, 1.0 / (h * h), out);
  return hipGetLastError();
}

}  // namespace ionic
