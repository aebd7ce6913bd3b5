// Mixed-precision LR91 step kernels (Rush-Larsen predictor), in a translation unit
// of their own so the model kernels compile in parallel.
#include "kernel_ops_impl.h"
#include "model_lr91.h"

namespace ionic {
hipError_t lr91_sdc_mixed_rl(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<LR91>::sdc<Mixed, kPredRushLarsen>(M, params, c, blocks, st);
}
}  // namespace ionic
