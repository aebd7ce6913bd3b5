// LR91 launch table and auxiliary kernels; the step kernels are instantiated
// in kernels_lr91_{fp64,mixed}[_ros2|_rl].hip.
#include "kernel_ops_impl.h"
#include "model_lr91.h"

namespace ionic {
static const char* const kNamesLR91[] = {"V", "Cai", "m", "h", "j", "d", "f", "X"};
static ModelOps make_lr91() {
  ModelOps o = OpsImpl<LR91>::make<false>(kNamesLR91);
  o.sdc[0][kPredNewton] = &lr91_sdc_fp64_newton;
  o.sdc[0][kPredRos2] = &lr91_sdc_fp64_ros2;
  o.sdc[1][kPredNewton] = &lr91_sdc_mixed_newton;
  o.sdc[1][kPredRos2] = &lr91_sdc_mixed_ros2;
  o.sdc[0][kPredRushLarsen] = &lr91_sdc_fp64_rl;
  o.sdc[1][kPredRushLarsen] = &lr91_sdc_mixed_rl;
  return o;
}
const ModelOps kOpsLR91 = make_lr91();
}  // namespace ionic
