// Double-precision LR91 step kernel, in a translation unit of its own built at
// -O1, for the same reason as kernels_tt06_fp64.hip: an -O3 build of it
// returned non-finite states on gfx950 while -O1 and host builds are exact.
#include "kernel_ops_impl.h"
#include "model_lr91.h"

namespace ionic {
hipError_t lr91_sdc64(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<LR91>::sdc64(M, params, c, blocks, st);
}
}  // namespace ionic
