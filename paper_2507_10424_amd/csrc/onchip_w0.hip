// On-chip decoder kernels of one register budget: the compiler's.
#include "onchip_kernel.h"

namespace ldpc {
namespace onchip {
const KernelFn kKernelsW0[2][kNumVariants] = {LDPC_ONCHIP_ROW(0, false), LDPC_ONCHIP_ROW(0, true)};
} // namespace onchip
} // namespace ldpc
