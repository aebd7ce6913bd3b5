// Diffusion current of the parabolic equation on a structured grid (paper
// section 3.1, equation semi-parabolic; Q1 elements, lumped mass), as the
// per-step input of the reaction stage:
//
//   I_diff = -sigma * M_L^{-1} A v,
//
// A the unit-conductivity stiffness matrix, M_L the lumped mass, homogeneous
// Neumann boundaries (natural).  The rows of A come from stencil.h.  One
// thread per node; V is the first state plane (double in every precision
// layout), read through the L1/L2 caches for the neighbours.  The kernel moves
// 16 bytes per node from HBM (V once, I_diff once) and keeps index arithmetic
// cheap: a 3D launch, no division.
#include "kernel_ops.h"
#include "stencil.h"

namespace ionic {

namespace {

constexpr int kDiffBlock = 64;

// Grid: x across the threads of a block row (blockIdx.x), y and z one block
// row each (blockIdx.y, blockIdx.z).
__global__ void __launch_bounds__(kDiffBlock)
    diffusion_kernel(const double* __restrict__ V, long long nx, long long ny, long long nz,
                     double sigma, double inv_h2, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * kDiffBlock + threadIdx.x;
  if (i >= nx) return;
  const Q1Node node(i, blockIdx.y, blockIdx.z, nx, ny, nz);
  const double s[3] = {sigma, sigma, sigma};
  out[node.index()] = -inv_h2 * node.apply(V, s) / node.mass();
}

}  // namespace

hipError_t diffusion_launch(const double* V, long long nx, long long ny, long long nz, double h,
                            double sigma, double* out, hipStream_t st) {
  if (ny > 65535 || nz > 65535) return hipErrorInvalidValue;  // grid y/z extent
  const long long gx = (nx + kDiffBlock - 1) / kDiffBlock;
  hipLaunchKernelGGL(diffusion_kernel, dim3(unsigned(gx), unsigned(ny), unsigned(nz)),
                     dim3(kDiffBlock), 0, st, V, nx, ny, nz, sigma, 1.0 / (h * h), out);
  return hipGetLastError();
}

}  // namespace ionic
