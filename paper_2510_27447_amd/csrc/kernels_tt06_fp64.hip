// Double-precision TT06 step kernels (Newton predictor), in a translation unit
// of their own so the model kernels compile in parallel.  These kernels need
// all 512 vector registers and still spill; the build's codegen check guards
// them against spill code placed ahead of an execution-mask restore.
#include "kernel_ops_impl.h"
#include "model_tt06.h"

namespace ionic {
hipError_t tt06_sdc_fp64_newton(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<TT06>::sdc<Fp64, kPredNewton>(M, params, c, blocks, st);
}
}  // namespace ionic
