// BF16 generic entries of the forward: kernels compiled for larger feature and hidden
// tiles that serve the models between the exact shape families (tabnet_kernel.hip, TABNET_GENERIC_SET).  A translation unit of its own so that
// the build compiles them beside the main kernels.
#define TABNET_GENERIC_TU
#include "tabnet_kernel.hip"

namespace tabnet {
extern const KernelEntry kGenericBf16[];
extern const int kGenericBf16Count;
const KernelEntry kGenericBf16[] = {TABNET_GENERIC_SET(1)};
const int kGenericBf16Count =
    (int)(sizeof(kGenericBf16) / sizeof(kGenericBf16[0]));
}  // namespace tabnet
