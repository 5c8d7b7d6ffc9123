// On-chip decoder kernels of one register budget: at least 4 waves per SIMD.
#include "onchip_kernel.h"

namespace ldpc {
namespace onchip {
const KernelFn kKernelsW4[2][kNumVariants] = {LDPC_ONCHIP_ROW(4, false), LDPC_ONCHIP_ROW(4, true)};
} // namespace onchip
} // namespace ldpc
