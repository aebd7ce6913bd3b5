// LR91 instantiations of the reaction + SDC kernels.
#include "kernel_ops_impl.h"
#include "model_lr91.h"

namespace ionic {
static const char* const kNamesLR91[] = {"V", "Cai", "m", "h", "j", "d", "f", "X"};
const ModelOps kOpsLR91 = OpsImpl<LR91>::make(kNamesLR91);
}  // namespace ionic
