// Rows of the Q1 stiffness matrix on a uniform structured grid of nodes (paper
// section 3.1: multilinear elements on quadrilaterals / hexahedra), for a
// diagonal conductivity tensor s = (s_x, s_y, s_z).
//
// The Q1 element is a tensor product of 1D linear elements, so every entry
// follows from the 1D element stiffness (1, -1)/h and mass (1/3, 1/6) h.
// Along a grid direction a node has c in {1, 2} adjacent elements; for an
// offset o the direction contributes the stiffness factor S = c (o == 0) or
// -1 (o != 0) and the mass factor W = c/3 (o == 0) or 1/6 (o != 0).  The entry
// for offset (o_x, o_y, o_z) is h^(d-2) sum_a s_a S_a prod_{b != a} W_b, and
// the lumped mass of the node is h^d prod_a c_a / 2, where d counts the
// directions with more than one node (the others drop out).  Everything here
// omits the common factor h^(d-2) of the entries and h^d of the mass.
#pragma once

#include <hip/hip_runtime.h>

namespace ionic {

struct Q1Dir {
  bool on;       // the direction has more than one node
  int c;         // adjacent elements along it
  double S[3], W[3];
};

__device__ __forceinline__ Q1Dir q1_dir(long long i, long long n) {
  Q1Dir d;
  d.on = n > 1;
  d.c = d.on ? int(i > 0) + int(i < n - 1) : 0;
  d.S[0] = d.S[2] = -1.0;
  d.W[0] = d.W[2] = 1.0 / 6.0;
  d.S[1] = double(d.c);
  d.W[1] = d.c / 3.0;
  return d;
}

// node (i, j, k) of an nx x ny x nz grid, vertex index i + nx (j + ny k)
struct Q1Node {
  long long i, j, k, nx, ny, nz;
  Q1Dir dx, dy, dz;
  __device__ __forceinline__ Q1Node(long long i_, long long j_, long long k_, long long nx_,
                                    long long ny_, long long nz_)
      : i(i_), j(j_), k(k_), nx(nx_), ny(ny_), nz(nz_), dx(q1_dir(i_, nx_)), dy(q1_dir(j_, ny_)),
        dz(q1_dir(k_, nz_)) {}

  __device__ __forceinline__ long long index() const { return i + nx * (j + ny * k); }

  // lumped mass / h^d
  __device__ __forceinline__ double mass() const {
    double m = 1.0;
    if (dx.on) m *= 0.5 * dx.c;
    if (dy.on) m *= 0.5 * dy.c;
    if (dz.on) m *= 0.5 * dz.c;
    return m;
  }

  __device__ __forceinline__ double coef(int ox, int oy, int oz, const double (&s)[3]) const {
    const double Wx = dx.on ? dx.W[ox + 1] : 1.0, Wy = dy.on ? dy.W[oy + 1] : 1.0,
                 Wz = dz.on ? dz.W[oz + 1] : 1.0;
    double c = 0.0;
    if (dx.on) c += s[0] * dx.S[ox + 1] * Wy * Wz;
    if (dy.on) c += s[1] * dy.S[oy + 1] * Wx * Wz;
    if (dz.on) c += s[2] * dz.S[oz + 1] * Wx * Wy;
    return c;
  }

  // diagonal entry / h^(d-2)
  __device__ __forceinline__ double diag(const double (&s)[3]) const { return coef(0, 0, 0, s); }

  // (A_s x)_node / h^(d-2).  Every row sums to zero (constants are in the null
  // space), so the row is applied to differences from the node's own value,
  // sum_{o != 0} a_o (x_{node+o} - x_node): a field with a large common offset
  // (V near -85 mV) loses nothing to cancellation, and a constant field gives
  // exactly zero.  The entries a_o of a pair of nodes are the same products in
  // both rows, so the operator stays exactly symmetric.
  __device__ __forceinline__ double apply(const double* __restrict__ x,
                                          const double (&s)[3]) const {
    const double xc = x[index()];
    double acc = 0.0;
    for (int oz = -1; oz <= 1; ++oz) {
      if ((!dz.on && oz != 0) || k + oz < 0 || k + oz >= nz) continue;
      for (int oy = -1; oy <= 1; ++oy) {
        if ((!dy.on && oy != 0) || j + oy < 0 || j + oy >= ny) continue;
        const double* row = x + nx * ((j + oy) + ny * (k + oz));
        for (int ox = -1; ox <= 1; ++ox) {
          if ((!dx.on && ox != 0) || i + ox < 0 || i + ox >= nx) continue;
          if (ox == 0 && oy == 0 && oz == 0) continue;
          acc += coef(ox, oy, oz, s) * (row[i + ox] - xc);
        }
      }
    }
    return acc;
  }
};

}  // namespace ionic
