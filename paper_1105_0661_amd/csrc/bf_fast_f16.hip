// bf_fast_f16.hip -- fast contraction kernels with FP16 operands.
#include "bf_fast_impl.h"

namespace lbf {
hipError_t launch_fast_f16(const BlockDesc& d, hipStream_t st) { return launch_fast_h<CT_F16>(d, st); }
}  // namespace lbf
