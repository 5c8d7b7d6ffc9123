// On-chip decoder kernels of one register budget: at least 3 waves per SIMD.
#include "onchip_kernel.h"

namespace ldpc {
namespace onchip {
const KernelFn kKernelsW3[2][kNumVariants] = {LDPC_ONCHIP_ROW(3, false), LDPC_ONCHIP_ROW(3, true)};
} // namespace onchip
} // namespace ldpc
