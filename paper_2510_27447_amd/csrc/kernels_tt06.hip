// TT06 (epicardial) launch table and auxiliary kernels; the step kernels are
// instantiated in kernels_tt06_{fp64,mixed}[_ros2|_rl].hip.
#include "kernel_ops_impl.h"
#include "model_tt06.h"

namespace ionic {
static const char* const kNamesTT06[] = {"V",   "Cai", "CaSR", "CaSS", "Nai", "Ki", "m",
                                         "h",   "j",   "xr1",  "xr2",  "xs",  "r",  "s",
                                         "d",   "f",   "f2",   "fCass", "Rbar"};
static ModelOps make_tt06() {
  ModelOps o = OpsImpl<TT06>::make<false>(kNamesTT06);
  o.sdc[0][kPredNewton] = &tt06_sdc_fp64_newton;
  o.sdc[0][kPredRos2] = &tt06_sdc_fp64_ros2;
  o.sdc[1][kPredNewton] = &tt06_sdc_mixed_newton;
  o.sdc[1][kPredRos2] = &tt06_sdc_mixed_ros2;
  o.sdc[0][kPredRushLarsen] = &tt06_sdc_fp64_rl;
  o.sdc[1][kPredRushLarsen] = &tt06_sdc_mixed_rl;
  return o;
}
const ModelOps kOpsTT06 = make_tt06();
}  // namespace ionic
