// Double-precision TT06 step kernel, in a translation unit of its own: the
// build compiles it at -O1.  At -O3 the register allocator's handling of this
// kernel (over 256 VGPRs plus AGPRs at one wave per SIMD) corrupted state
// carried across the time-step loop on gfx950, while -O1 code is exact.
#include "kernel_ops_impl.h"
#include "model_tt06.h"

namespace ionic {
hipError_t tt06_sdc64(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<TT06>::sdc64(M, params, c, blocks, st);
}
}  // namespace ionic
