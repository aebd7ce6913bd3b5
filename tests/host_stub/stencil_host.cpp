// The library's Q1 stencil header built as plain host C++ (test only): every
// node's row applied to a field, its diagonal and its lumped mass.
#include <hip/hip_runtime.h>
// wavefront shuffles: declared for the lane-shuffle variant of the row, which
// this host build does not call
double __shfl_up(double, unsigned int, int);
double __shfl_down(double, unsigned int, int);
#include "stencil.h"

extern "C" int q1_rows(const double* x, long long nx, long long ny, long long nz,
                       const double* sigma, double* out, double* diag, double* mass) {
  const double s[3] = {sigma[0], sigma[1], sigma[2]};
  const long long n = nx * ny * nz;
  for (long long v = 0; v < n; ++v) {
    const ionic::Q1Coords c = ionic::q1_coords(v, nx, ny);
    const ionic::Q1Node node(c.i, c.j, c.k, nx, ny, nz);
    if (node.index() != v) return 1;
    out[v] = node.apply(x, s);
    diag[v] = node.diag(s);
    mass[v] = node.mass();
  }
  return 0;
}
