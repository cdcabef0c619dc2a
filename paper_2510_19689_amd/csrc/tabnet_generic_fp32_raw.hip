// FP32 raw-row twins of the generic register-resident entries (the embedding gathered
// in the kernel, masks per raw column; tabnet_kernel.hip, TABNET_GENERIC_RAW_SET).  A
// translation unit of its own so that the build compiles them beside the main kernels.
#define TABNET_GENERIC_TU
#include "tabnet_kernel.hip"

namespace tabnet {
extern const KernelEntry kGenericFp32Raw[];
extern const int kGenericFp32RawCount;
const KernelEntry kGenericFp32Raw[] = {TABNET_GENERIC_RAW_SET(0)};
const int kGenericFp32RawCount = (int)(sizeof(kGenericFp32Raw) / sizeof(kGenericFp32Raw[0]));
}  // namespace tabnet
