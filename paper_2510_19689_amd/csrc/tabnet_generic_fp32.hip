// FP32 generic entries of the forward: kernels compiled for larger feature and hidden
// tiles that serve the models between the exact shape families (tabnet_kernel.hip, TABNET_GENERIC_SET).  A translation unit of its own so that
// the build compiles them beside the main kernels.
#define TABNET_GENERIC_TU
#include "tabnet_kernel.hip"

namespace tabnet {
extern const KernelEntry kGenericFp32[];
extern const int kGenericFp32Count;
const KernelEntry kGenericFp32[] = {TABNET_GENERIC_SET(0)};
const int kGenericFp32Count =
    (int)(sizeof(kGenericFp32) / sizeof(kGenericFp32[0]));
}  // namespace tabnet
