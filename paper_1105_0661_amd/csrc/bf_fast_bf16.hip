// bf_fast_bf16.hip -- fast contraction kernels with BF16 operands.
#include "bf_fast_impl.h"

namespace lbf {
hipError_t launch_fast_bf16(const BlockDesc& d, hipStream_t st) { return launch_fast_h<CT_BF16>(d, st); }
}  // namespace lbf
