// Host side of the multigrid preconditioner of multigrid.hip: the level
// hierarchy of a structured grid, the 1D tables of every level (the Q1
// element's stiffness and mass rows, the linear prolongation, the Galerkin
// products) and the dense inverse of the coarsest level.  Plain C++ (no device
// code), so the tests build it on the host as well.
#include <algorithm>
#include <cmath>

#include "grid_ops.h"

namespace ionic {

namespace {

constexpr long long kMaxCoarsest = 512;

long long coarse_extent(long long n) {
  if (n <= 2) return n;
  return n % 2 ? (n + 1) / 2 : n / 2 + 1;
}

}  // namespace

MgPlan mg_plan(long long nx, long long ny, long long nz) {
  MgPlan p;
  long long d[3] = {nx, ny, nz};
  p.levels = 0;
  for (;;) {
    for (int a = 0; a < 3; ++a) p.dims[p.levels][a] = d[a];
    ++p.levels;
    const long long n = d[0] * d[1] * d[2];
    long long c[3];
    bool any = false;
    for (int a = 0; a < 3; ++a) {
      c[a] = coarse_extent(d[a]);
      any = any || c[a] != d[a];
    }
    if (n <= kMaxCoarsest || !any || p.levels == kMgMaxLevels) break;
    for (int a = 0; a < 3; ++a) d[a] = c[a];
  }
  // the coarsest level is inverted densely: at most 512 nodes (a 2 MB inverse)
  const long long* last = p.dims[p.levels - 1];
  p.usable = p.levels >= 2 && last[0] * last[1] * last[2] <= kMaxCoarsest;
  // table layout: per level, per direction K and M (3 each per index), then
  // (levels but the coarsest) I0, w0, w1 per index
  size_t off = 0;
  for (int l = 0; l < p.levels; ++l)
    for (int a = 0; a < 3; ++a) {
      p.off_K[l][a] = off;
      off += 3 * size_t(p.dims[l][a]);
      p.off_M[l][a] = off;
      off += 3 * size_t(p.dims[l][a]);
      if (l + 1 < p.levels) {
        p.off_P[l][a] = off;
        off += 3 * size_t(p.dims[l][a]);
      }
    }
  const long long nc = last[0] * last[1] * last[2];
  p.off_inv = off;
  off += size_t(nc * nc);
  p.table_doubles = (off + 31) / 32 * 32;
  // vectors: invd on every level; x, y, b on the coarse levels
  size_t vec = 0;
  for (int l = 0; l < p.levels; ++l) {
    const size_t n = size_t(p.dims[l][0] * p.dims[l][1] * p.dims[l][2]);
    vec += (l == 0 ? 1 : 4) * ((n + 31) / 32 * 32);
  }
  p.vector_doubles = vec;
  return p;
}

size_t mg_doubles(const MgPlan& p) { return p.usable ? p.table_doubles + p.vector_doubles : 0; }

// 1D factor rows of the fine level (the Q1 element) and the Galerkin products
// P^T T P of the coarser ones; the prolongation of each coarsened direction.
std::vector<double> mg_tables(const MgPlan& p) {
  std::vector<double> t(p.table_doubles, 0.0);
  for (int a = 0; a < 3; ++a) {
    const long long n = p.dims[0][a];
    double* K = &t[p.off_K[0][a]];
    double* M = &t[p.off_M[0][a]];
    for (long long i = 0; i < n; ++i) {
      if (n == 1) {
        M[3 * i + 1] = 1.0;
        continue;
      }
      const bool lo = i > 0, hi = i < n - 1;
      const double c = double(int(lo) + int(hi));
      K[3 * i + 0] = lo ? -1.0 : 0.0;
      K[3 * i + 1] = c;
      K[3 * i + 2] = hi ? -1.0 : 0.0;
      M[3 * i + 0] = lo ? 1.0 / 6.0 : 0.0;
      M[3 * i + 1] = c / 3.0;
      M[3 * i + 2] = hi ? 1.0 / 6.0 : 0.0;
    }
  }
  for (int l = 0; l + 1 < p.levels; ++l)
    for (int a = 0; a < 3; ++a) {
      const long long nf = p.dims[l][a], nc = p.dims[l + 1][a];
      double* I0 = &t[p.off_P[l][a]];
      double* w0 = I0 + nf;
      double* w1 = w0 + nf;
      const bool coarsened = nc != nf;
      for (long long i = 0; i < nf; ++i) {
        if (!coarsened) {
          I0[i] = double(i);
          w0[i] = 1.0;
          w1[i] = 0.0;
          continue;
        }
        // coarse node I sits at fine index min(2I, nf - 1)
        long long I = std::min(i / 2, nc - 1);
        if (I == nc - 1 && I > 0 && i < nf - 1) I = nc - 2;
        const long long pa = std::min(2 * I, nf - 1);
        const long long pb = I + 1 < nc ? std::min(2 * (I + 1), nf - 1) : pa;
        I0[i] = double(I);
        if (pb == pa) {
          w0[i] = 1.0;
          w1[i] = 0.0;
        } else {
          w0[i] = double(pb - i) / double(pb - pa);
          w1[i] = 1.0 - w0[i];
        }
      }
      // Galerkin products of both tridiagonal factors
      for (int which = 0; which < 2; ++which) {
        const double* T = &t[which == 0 ? p.off_K[l][a] : p.off_M[l][a]];
        double* C = &t[which == 0 ? p.off_K[l + 1][a] : p.off_M[l + 1][a]];
        for (long long i = 0; i < nf; ++i)
          for (int o = -1; o <= 1; ++o) {
            const long long j = i + o;
            if (j < 0 || j >= nf) continue;
            const double tij = T[3 * i + o + 1];
            if (tij == 0.0) continue;
            for (int u = 0; u < 2; ++u) {
              const long long I = (long long)I0[i] + u;
              const double pI = u == 0 ? w0[i] : w1[i];
              if (pI == 0.0 || I >= nc) continue;
              for (int v2 = 0; v2 < 2; ++v2) {
                const long long J = (long long)I0[j] + v2;
                const double pJ = v2 == 0 ? w0[j] : w1[j];
                if (pJ == 0.0 || J >= nc || J - I < -1 || J - I > 1) continue;
                C[3 * I + (J - I) + 1] += pI * tij * pJ;
              }
            }
          }
      }
    }
  return t;
}

// The coarsest matrix A_c = sum_a s_a K_a (x) M_b (x) M_c from its 1D rows,
// plus alpha 1 1^T, inverted by Cholesky (it is symmetric positive definite:
// A_c is semi-definite with the constants as null space, which alpha 1 1^T
// covers); the inverse goes to the table's off_inv block.
void mg_coarse_inverse(const MgPlan& p, const double s[3], std::vector<double>& t) {
  const int L = p.levels - 1;
  const long long nx = p.dims[L][0], ny = p.dims[L][1], nz = p.dims[L][2];
  const long long n = nx * ny * nz;
  const double* K[3] = {&t[p.off_K[L][0]], &t[p.off_K[L][1]], &t[p.off_K[L][2]]};
  const double* M[3] = {&t[p.off_M[L][0]], &t[p.off_M[L][1]], &t[p.off_M[L][2]]};
  std::vector<double> A(size_t(n * n), 0.0);
  for (long long k = 0; k < nz; ++k)
    for (long long j = 0; j < ny; ++j)
      for (long long i = 0; i < nx; ++i) {
        const long long v = i + nx * (j + ny * k);
        for (int oz = -1; oz <= 1; ++oz)
          for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
              const long long i2 = i + ox, j2 = j + oy, k2 = k + oz;
              if (i2 < 0 || i2 >= nx || j2 < 0 || j2 >= ny || k2 < 0 || k2 >= nz) continue;
              const double kx = K[0][3 * i + ox + 1], mx = M[0][3 * i + ox + 1];
              const double ky = K[1][3 * j + oy + 1], my = M[1][3 * j + oy + 1];
              const double kz = K[2][3 * k + oz + 1], mz = M[2][3 * k + oz + 1];
              A[size_t(v * n + (i2 + nx * (j2 + ny * k2)))] =
                  s[0] * kx * my * mz + s[1] * mx * ky * mz + s[2] * mx * my * kz;
            }
      }
  double trace = 0.0;
  for (long long v = 0; v < n; ++v) trace += A[size_t(v * n + v)];
  const double alpha = trace > 0.0 ? trace / double(n * n) : 1.0;
  for (auto& a : A) a += alpha;
  // Cholesky A = L L^T in the lower triangle
  for (long long j = 0; j < n; ++j) {
    double d = A[size_t(j * n + j)];
    for (long long q = 0; q < j; ++q) d -= A[size_t(j * n + q)] * A[size_t(j * n + q)];
    d = std::sqrt(std::max(d, 1e-300));
    A[size_t(j * n + j)] = d;
    for (long long i = j + 1; i < n; ++i) {
      double e = A[size_t(i * n + j)];
      for (long long q = 0; q < j; ++q) e -= A[size_t(i * n + q)] * A[size_t(j * n + q)];
      A[size_t(i * n + j)] = e / d;
    }
  }
  // inverse column by column: L y = e_c, L^T x = y
  double* inv = &t[p.off_inv];
  std::vector<double> y(static_cast<size_t>(n));
  for (long long c = 0; c < n; ++c) {
    for (long long i = 0; i < n; ++i) {
      double e = i == c ? 1.0 : 0.0;
      for (long long q = 0; q < i; ++q) e -= A[size_t(i * n + q)] * y[size_t(q)];
      y[size_t(i)] = e / A[size_t(i * n + i)];
    }
    for (long long i = n - 1; i >= 0; --i) {
      double e = y[size_t(i)];
      for (long long q = i + 1; q < n; ++q) e -= A[size_t(q * n + i)] * inv[size_t(q * n + c)];
      inv[size_t(i * n + c)] = e / A[size_t(i * n + i)];
    }
  }
}

}  // namespace ionic
