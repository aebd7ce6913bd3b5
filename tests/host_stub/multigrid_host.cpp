// The library's multigrid planning (multigrid_plan.cpp) behind a C interface
// for the CPU tests: the level extents, and the tables of every level with
// the offsets of each block.
#include <cstring>

#include "grid_ops.h"

extern "C" int mg_host_plan(long long nx, long long ny, long long nz, long long* dims,
                            int* usable, long long* table_doubles) {
  const ionic::MgPlan p = ionic::mg_plan(nx, ny, nz);
  for (int l = 0; l < p.levels; ++l)
    for (int a = 0; a < 3; ++a) dims[3 * l + a] = p.dims[l][a];
  *usable = p.usable ? 1 : 0;
  *table_doubles = (long long)p.table_doubles;
  return p.levels;
}

// offsets: per level and direction K, M, P (P: -1 on the coarsest), then the
// coarsest inverse's offset last
extern "C" int mg_host_tables(long long nx, long long ny, long long nz, const double* s,
                              double* out, long long cap, long long* offsets) {
  const ionic::MgPlan p = ionic::mg_plan(nx, ny, nz);
  if ((long long)p.table_doubles > cap) return -1;
  std::vector<double> t = ionic::mg_tables(p);
  if (p.usable) ionic::mg_coarse_inverse(p, s, t);
  std::memcpy(out, t.data(), t.size() * sizeof(double));
  long long* o = offsets;
  for (int l = 0; l < p.levels; ++l)
    for (int a = 0; a < 3; ++a) {
      *o++ = (long long)p.off_K[l][a];
      *o++ = (long long)p.off_M[l][a];
      *o++ = l + 1 < p.levels ? (long long)p.off_P[l][a] : -1;
    }
  *o = (long long)p.off_inv;
  return p.levels;
}
