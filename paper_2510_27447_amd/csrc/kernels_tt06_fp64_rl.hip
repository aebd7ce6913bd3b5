// Double-precision TT06 step kernels (Rush-Larsen predictor), in a translation unit
// of their own so the model kernels compile in parallel; guarded by the
// build's codegen check like the other double kernels.
#include "kernel_ops_impl.h"
#include "model_tt06.h"

namespace ionic {
hipError_t tt06_sdc_fp64_rl(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<TT06>::sdc<Fp64, kPredRushLarsen>(M, params, c, blocks, st);
}
}  // namespace ionic
