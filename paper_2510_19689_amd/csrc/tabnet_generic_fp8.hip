// FP8 (E4M3 on both GEMM operands) generic entries of the forward: kernels compiled for larger
// feature and hidden tiles that serve the models between the exact shape families
// (tabnet_kernel.hip, TABNET_GENERIC_SET).  A translation unit of its own so that the
// build compiles them beside the main kernels.
#define TABNET_GENERIC_TU
#include "tabnet_kernel.hip"

namespace tabnet {
extern const KernelEntry kGenericFp8[];
extern const int kGenericFp8Count;
const KernelEntry kGenericFp8[] = {TABNET_GENERIC_SET(2)};
const int kGenericFp8Count = (int)(sizeof(kGenericFp8) / sizeof(kGenericFp8[0]));
}  // namespace tabnet
