// FP8-weight (E4M3 weights, BF16 inputs) generic entries of the forward: kernels compiled for larger feature and
// hidden tiles that serve the models between the exact shape families (tabnet_kernel.hip,
// TABNET_GENERIC_SET).  A translation unit of its own so that the build compiles them
// beside the main kernels.
#define TABNET_GENERIC_TU
#include "tabnet_kernel.hip"

namespace tabnet {
extern const KernelEntry kGenericFp8w[];
extern const int kGenericFp8wCount;
const KernelEntry kGenericFp8w[] = {TABNET_GENERIC_SET(9)};
const int kGenericFp8wCount = (int)(sizeof(kGenericFp8w) / sizeof(kGenericFp8w[0]));
}  // namespace tabnet
