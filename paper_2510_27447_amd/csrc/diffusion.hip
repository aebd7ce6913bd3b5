// Diffusion current of the parabolic equation on a structured grid (paper
// section 3.1, equation semi-parabolic; Q1 elements, lumped mass), as the
// per-step input of the reaction stage:
//
//   I_diff = -sigma * M_L^{-1} A v,
//
// A the unit-conductivity stiffness matrix, M_L the lumped mass, homogeneous
// Neumann boundaries (natural).  The rows of A come from stencil.h.  One
// wavefront per 62 consecutive nodes on a 1D launch; V is the first state
// plane (double in every precision layout), read through the L1/L2 caches for
// the neighbours.  The kernel moves 16 bytes per node from HBM
// (V once, I_diff once).  Grids have fewer than 2^31 nodes.
#include "grid_ops.h"
#include "stencil.h"

namespace ionic {

namespace {

constexpr int kDiffBlock = 256;
constexpr int kLanesOut = 62;  // nodes per wavefront pass
constexpr int kNodesPerBlock = (kDiffBlock / 64) * kLanesOut;

// Each wavefront takes 62 consecutive nodes (lanes 1..62; lanes 0 and 63 hold
// the nodes on either side): every lane loads its own column of the 9 rows and
// takes the x-neighbours from the adjacent lanes (Q1Node::apply_lanes).
__global__ void __launch_bounds__(kDiffBlock)
    diffusion_kernel(const double* __restrict__ V, long long n, long long nx, long long ny,
                     long long nz, double sigma, double inv_h2, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const long long v =
      (long long)blockIdx.x * kNodesPerBlock + (threadIdx.x >> 6) * kLanesOut - 1 + lane;
  const long long vl = v < 0 ? 0 : (v < n ? v : n - 1);  // the node this lane loads
  const Q1Coords x = q1_coords(vl, nx, ny);
  const Q1Node node(x.i, x.j, x.k, nx, ny, nz);
  const double s[3] = {sigma, sigma, sigma};
  double own;
  const double a = node.apply_lanes([V](long long t) { return V[t]; }, s, own);
  if (lane >= 1 && lane <= kLanesOut && v < n) out[v] = -inv_h2 * a / node.mass();
}

}  // namespace

hipError_t diffusion_launch(const double* V, long long nx, long long ny, long long nz, double h,
                            double sigma, double* out, hipStream_t st) {
  const long long n = nx * ny * nz;
  if (n >= (1ll << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(diffusion_kernel, dim3(unsigned((n + kNodesPerBlock - 1) / kNodesPerBlock)),
                     dim3(kDiffBlock), 0, st, V, n, nx, ny, nz, sigma, 1.0 / (h * h), out);
  return hipGetLastError();
}

}  // namespace ionic
