// Double-precision TT06 step kernels (Newton predictor), in a translation
// unit of their own: the build compiles it at -O1.  At -O3 the Newton variant
// of this kernel (over 256 VGPRs plus AGPRs and scratch at one wave per SIMD)
// returned corrupted state on gfx950 while the same source at -O1, and on the
// host, matches the reference to 1e-15; the other double kernels follow suit.
#include "kernel_ops_impl.h"
#include "model_tt06.h"

namespace ionic {
hipError_t tt06_sdc_fp64_newton(int M, const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
  return OpsImpl<TT06>::sdc<Fp64, kPredNewton>(M, params, c, blocks, st);
}
}  // namespace ionic
