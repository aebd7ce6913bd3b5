// TT06 (epicardial) instantiations of the reaction + SDC kernels.
#include "kernel_ops_impl.h"
#include "model_tt06.h"

namespace ionic {
static const char* const kNamesTT06[] = {"V",   "Cai", "CaSR", "CaSS", "Nai", "Ki", "m",
                                         "h",   "j",   "xr1",  "xr2",  "xs",  "r",  "s",
                                         "d",   "f",   "f2",   "fCass", "Rbar"};
static ModelOps make_tt06() {
  ModelOps o = OpsImpl<TT06>::make<false>(kNamesTT06);
  o.sdc64 = &tt06_sdc64;  // instantiated in kernels_tt06_fp64.hip
  return o;
}
const ModelOps kOpsTT06 = make_tt06();
}  // namespace ionic
