// BF16 raw-row twins of the generic register-resident entries (the embedding gathered
// in the kernel, masks per raw column; tabnet_kernel.hip, TABNET_GENERIC_RAW_SET).  A
// translation unit of its own so that the build compiles them beside the main kernels.
#define TABNET_GENERIC_TU
#include "tabnet_kernel.hip"

namespace tabnet {
extern const KernelEntry kGenericBf16Raw[];
extern const int kGenericBf16RawCount;
const KernelEntry kGenericBf16Raw[] = {TABNET_GENERIC_RAW_SET(1)};
const int kGenericBf16RawCount = (int)(sizeof(kGenericBf16Raw) / sizeof(kGenericBf16Raw[0]));
}  // namespace tabnet
