// bf_fast_f32.hip -- fast contraction kernels with FP32 operands.
#include "bf_fast_impl.h"

namespace lbf {
hipError_t launch_fast_f32(const BlockDesc& d, hipStream_t st) {
    int nbg;
    const int n = block_items_fast_f32(d, &nbg);
    if (d.xtype == XT_CI8) return launch_f32_xt<XT_CI8>(d, nbg, n, st);
    if (d.xtype == XT_CI16) return launch_f32_xt<XT_CI16>(d, nbg, n, st);
    return launch_f32_xt<XT_CF32>(d, nbg, n, st);
}
}  // namespace lbf
