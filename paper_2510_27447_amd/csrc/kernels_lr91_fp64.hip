// Double-precision LR91 step kernels (Newton predictor), in a translation
// unit of their own built at -O1, for the same reason as the TT06 ones: an -O3
// build of the Newton variant returned non-finite states on gfx950 while -O1
// and host builds are exact.
#include "kernel_ops_impl.h"
#include "model_lr91.h"

namespace ionic {
hipError_t lr91_sdc_fp64_newton(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<LR91>::sdc<Fp64, kPredNewton>(M, params, c, blocks, st);
}
}  // namespace ionic
