// LR91 instantiations of the reaction + SDC kernels.
#include "kernel_ops_impl.h"
#include "model_lr91.h"

namespace ionic {
static const char* const kNamesLR91[] = {"V", "Cai", "m", "h", "j", "d", "f", "X"};
static ModelOps make_lr91() {
  ModelOps o = OpsImpl<LR91>::make<false>(kNamesLR91);
  o.sdc64 = &lr91_sdc64;  // instantiated in kernels_lr91_fp64.hip
  return o;
}
const ModelOps kOpsLR91 = make_lr91();
}  // namespace ionic
