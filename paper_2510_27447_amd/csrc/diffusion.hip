// Diffusion current of the parabolic equation on a structured grid (paper
// section 3.1, equation semi-parabolic; Q1 elements, lumped mass), as the
// per-step input of the reaction stage:
//
//   I_diff = -sigma * M_L^{-1} A v,
//
// A the unit-conductivity stiffness matrix, M_L the lumped mass, homogeneous
// Neumann boundaries (natural).  On a uniform grid of node spacing h the
// assembled row of node p couples it to the nodes p + o, o in {-1,0,1}^d, and
// the Q1 element is a tensor product of 1D linear elements, so every entry
// follows from the 1D element stiffness (1, -1)/h and mass (1/3, 1/6) h.
// Along a grid direction j a node has c_j in {1, 2} adjacent elements; for
// offset o_j the direction contributes
//   stiffness factor S_j = c_j (o_j == 0) or -1 (o_j != 0),
//   mass factor      W_j = c_j / 3 (o_j == 0) or 1/6 (o_j != 0),
// the entry is h^(d-2) * sum_k S_k prod_{j != k} W_j, and the lumped mass is
// h^d prod_j c_j / 2.  Directions with a single node drop out (d counts the
// others).  One thread per node; V is the first state plane (double in every
// precision layout), read through the L1/L2 caches for the neighbours.  The
// kernel moves 16 bytes per node from HBM (V once, I_diff once) and is bound
// by memory, so it keeps index arithmetic cheap: a 3D launch, no division.
#include "kernel_ops.h"

namespace ionic {

namespace {

constexpr int kDiffBlock = 64;

// Per direction: the number of adjacent elements c of the node and, for the
// three offsets -1, 0, +1, the stiffness factor S and mass factor W.  A
// direction with a single node has c = 0 and is skipped.
struct Dir {
  int c;
  double S[3], W[3];
};

__device__ __forceinline__ Dir direction(long long i, long long n) {
  Dir d;
  d.c = n > 1 ? int(i > 0) + int(i < n - 1) : 0;
  d.S[0] = d.S[2] = -1.0;
  d.W[0] = d.W[2] = 1.0 / 6.0;
  d.S[1] = double(d.c);
  d.W[1] = d.c / 3.0;
  return d;
}

// Grid: x across the threads of a block row (blockIdx.x), y and z one block
// row each (blockIdx.y, blockIdx.z), so no index division is needed.
__global__ void __launch_bounds__(kDiffBlock)
    diffusion_kernel(const double* __restrict__ V, long long nx, long long ny, long long nz,
                     double scale /* sigma / h^2 */, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * kDiffBlock + threadIdx.x;
  if (i >= nx) return;
  const long long j = blockIdx.y, k = blockIdx.z;
  const long long p = i + nx * (j + ny * k);
  const Dir dx = direction(i, nx), dy = direction(j, ny), dz = direction(k, nz);
  const bool ax = nx > 1, ay = ny > 1, az = nz > 1;
  double mass = 1.0;
  if (ax) mass *= 0.5 * dx.c;
  if (ay) mass *= 0.5 * dy.c;
  if (az) mass *= 0.5 * dz.c;
  double acc = 0.0;
  for (int oz = -1; oz <= 1; ++oz) {
    if ((!az && oz != 0) || k + oz < 0 || k + oz >= nz) continue;
    for (int oy = -1; oy <= 1; ++oy) {
      if ((!ay && oy != 0) || j + oy < 0 || j + oy >= ny) continue;
      const double* row = V + nx * ((j + oy) + ny * (k + oz));
      for (int ox = -1; ox <= 1; ++ox) {
        if ((!ax && ox != 0) || i + ox < 0 || i + ox >= nx) continue;
        // sum over directions a of S_a times the W of the other directions
        const double Wx = ax ? dx.W[ox + 1] : 1.0, Wy = ay ? dy.W[oy + 1] : 1.0,
                     Wz = az ? dz.W[oz + 1] : 1.0;
        double coef = 0.0;
        if (ax) coef += dx.S[ox + 1] * Wy * Wz;
        if (ay) coef += dy.S[oy + 1] * Wx * Wz;
        if (az) coef += dz.S[oz + 1] * Wx * Wy;
        acc += coef * row[i + ox];
      }
    }
  }
  out[p] = -scale * acc / mass;
}

}  // namespace

hipError_t diffusion_launch(const double* V, long long nx, long long ny, long long nz, double h,
                            double sigma, double* out, hipStream_t st) {
  if (ny > 65535 || nz > 65535) return hipErrorInvalidValue;  // grid y/z extent
  const long long gx = (nx + kDiffBlock - 1) / kDiffBlock;
  hipLaunchKernelGGL(diffusion_kernel, dim3(unsigned(gx), unsigned(ny), unsigned(nz)),
                     dim3(kDiffBlock), 0, st, V, nx, ny, nz, sigma / (h * h), out);
  return hipGetLastError();
}

}  // namespace ionic
