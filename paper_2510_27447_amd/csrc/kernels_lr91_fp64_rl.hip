// Double-precision LR91 step kernels (Rush-Larsen predictor), in a translation unit
// of their own so the model kernels compile in parallel; guarded by the
// build's codegen check like the other double kernels.
#include "kernel_ops_impl.h"
#include "model_lr91.h"

namespace ionic {
hipError_t lr91_sdc_fp64_rl(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<LR91>::sdc<Fp64, kPredRushLarsen>(M, params, c, blocks, st);
}
}  // namespace ionic
