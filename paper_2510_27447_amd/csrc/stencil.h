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
//
// A missing neighbour (a boundary node, or a direction with one node) gets
// S = W = 0 for its offset and its load is redirected to an existing node, so
// the row is evaluated without branches; a direction with one node has
// W = (0, 1, 0) and S = 0.
#pragma once

#include <hip/hip_runtime.h>

namespace ionic {

struct Q1Dir {
  double S[3], W[3];  // factors of the offsets -1, 0, +1
  double m;           // lumped-mass factor c/2 (1 for a direction with one node)
  long long lo, hi;   // index offsets of the -1 / +1 neighbours (0 where missing)
};

__device__ __forceinline__ Q1Dir q1_dir(long long i, long long n, long long stride) {
  Q1Dir d;
  const bool on = n > 1, has_lo = on && i > 0, has_hi = on && i < n - 1;
  const double c = double(int(has_lo) + int(has_hi));
  d.S[0] = has_lo ? -1.0 : 0.0;
  d.S[1] = c;
  d.S[2] = has_hi ? -1.0 : 0.0;
  d.W[0] = has_lo ? 1.0 / 6.0 : 0.0;
  d.W[1] = on ? c / 3.0 : 1.0;
  d.W[2] = has_hi ? 1.0 / 6.0 : 0.0;
  d.m = on ? 0.5 * c : 1.0;
  d.lo = has_lo ? -stride : 0;
  d.hi = has_hi ? stride : 0;
  return d;
}

// node (i, j, k) of an nx x ny x nz grid, vertex index i + nx (j + ny k)
struct Q1Node {
  long long n0;
  Q1Dir dx, dy, dz;
  __device__ __forceinline__ Q1Node(long long i, long long j, long long k, long long nx,
                                    long long ny, long long nz)
      : n0(i + nx * (j + ny * k)), dx(q1_dir(i, nx, 1)), dy(q1_dir(j, ny, nx)),
        dz(q1_dir(k, nz, nx * ny)) {}

  __device__ __forceinline__ long long index() const { return n0; }

  // lumped mass / h^d
  __device__ __forceinline__ double mass() const { return dx.m * dy.m * dz.m; }

  // diagonal entry / h^(d-2)
  __device__ __forceinline__ double diag(const double (&s)[3]) const {
    return s[0] * dx.S[1] * dy.W[1] * dz.W[1] + s[1] * dx.W[1] * dy.S[1] * dz.W[1] +
           s[2] * dx.W[1] * dy.W[1] * dz.S[1];
  }

  // (A_s x)_node / h^(d-2), x given by val(index).  Every row sums to zero
  // (constants are in the null space), so the row is applied to differences
  // from the node's own value, sum_o a_o (x_{node+o} - x_node): a field with a
  // large common offset (V near -85 mV) loses nothing to cancellation, and a
  // constant field gives exactly zero.  The 27 entries are products of one
  // factor per direction, so the sum is taken direction by direction: along x
  // within each of the 9 rows, then along y, then along z (about 120 flops
  // instead of forming 26 entries).
  template <class Val>
  __device__ __forceinline__ double apply_with(Val val, const double (&s)[3]) const {
    const double xc = val(n0);
    const long long ox[3] = {dx.lo, 0, dx.hi}, oy[3] = {dy.lo, 0, dy.hi},
                    oz[3] = {dz.lo, 0, dz.hi};
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double ww = 0.0, ws = 0.0, sw = 0.0;  // sum_y W_y (sum_x W_x d), W_y (S_x d), S_y (W_x d)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const long long row = n0 + oz[c] + oy[b];
        double xw = 0.0, xs = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double d = val(row + ox[a]) - xc;
          xw += dx.W[a] * d;
          xs += dx.S[a] * d;
        }
        ww += dy.W[b] * xw;
        ws += dy.W[b] * xs;
        sw += dy.S[b] * xw;
      }
      ax += dz.W[c] * ws;
      ay += dz.W[c] * sw;
      az += dz.S[c] * ww;
    }
    return s[0] * ax + s[1] * ay + s[2] * az;
  }

  __device__ __forceinline__ double apply(const double* __restrict__ x,
                                          const double (&s)[3]) const {
    return apply_with([x](long long t) { return x[t]; }, s);
  }

  // The same row when the lanes of the wavefront hold consecutive nodes: each
  // lane loads only its own column of the 9 rows (offsets in y and z), and the
  // -1 / +1 neighbours along x come from the previous / next lane.  Where a
  // node has an x-neighbour it is the adjacent node of the same x-row, so the
  // adjacent lane used the same y and z offsets; where it has none, the weight
  // is zero.  Every lane of the wavefront must call this together; lanes 0 and
  // 63 only supply values (their own results lack a neighbour).  x is given by
  // val(index); xc receives this lane's own value.
  template <class Val>
  __device__ __forceinline__ double apply_lanes(Val val, const double (&s)[3], double& xc) const {
    xc = val(n0);
    const long long oy[3] = {dy.lo, 0, dy.hi}, oz[3] = {dz.lo, 0, dz.hi};
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double ww = 0.0, ws = 0.0, sw = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double xm = val(n0 + oz[c] + oy[b]);
        const double d[3] = {__shfl_up(xm, 1, 64) - xc, xm - xc, __shfl_down(xm, 1, 64) - xc};
        double xw = 0.0, xs = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          xw += dx.W[a] * d[a];
          xs += dx.S[a] * d[a];
        }
        ww += dy.W[b] * xw;
        ws += dy.W[b] * xs;
        sw += dy.S[b] * xw;
      }
      ax += dz.W[c] * ws;
      ay += dz.W[c] * sw;
      az += dz.S[c] * ww;
    }
    return s[0] * ax + s[1] * ay + s[2] * az;
  }
};

// (i, j, k) of vertex v of an nx x ny x nz grid with fewer than 2^31 nodes
// (32-bit division)
struct Q1Coords {
  long long i, j, k;
};
__device__ __forceinline__ Q1Coords q1_coords(long long v, long long nx, long long ny) {
  const unsigned int uv = unsigned(v), unx = unsigned(nx), uny = unsigned(ny);
  const unsigned int jk = uv / unx;
  return {(long long)(uv - jk * unx), (long long)(jk % uny), (long long)(jk / uny)};
}

}  // namespace ionic
