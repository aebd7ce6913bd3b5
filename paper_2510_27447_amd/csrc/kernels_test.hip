// Instantiations for the scalar test problems.
#include "kernel_ops_impl.h"
#include "model_test.h"

namespace ionic {
static const char* const kNamesY[] = {"y"};
const ModelOps kOpsTestLinear = OpsImpl<TestLinear>::make(kNamesY);
const ModelOps kOpsTestLogistic = OpsImpl<TestLogistic>::make(kNamesY);
}  // namespace ionic
