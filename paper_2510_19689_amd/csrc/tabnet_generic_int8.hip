// INT8 generic entries of the forward: kernels compiled for larger feature and
// hidden tiles that serve the models between the exact shape families (tabnet_kernel.hip,
// TABNET_GENERIC_SET).  A translation unit of its own so that the build compiles them
// beside the main kernels.
#define TABNET_GENERIC_TU
#include "tabnet_kernel.hip"

namespace tabnet {
extern const KernelEntry kGenericInt8[];
extern const int kGenericInt8Count;
const KernelEntry kGenericInt8[] = {TABNET_GENERIC_SET(3)};
const int kGenericInt8Count = (int)(sizeof(kGenericInt8) / sizeof(kGenericInt8[0]));
}  // namespace tabnet
