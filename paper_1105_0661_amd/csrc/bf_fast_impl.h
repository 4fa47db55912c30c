// bf_fast_impl.h -- kernels and launchers of the fast contraction workers,
// instantiated per operand type in bf_fast_f32.hip / _f16.hip / _bf16.hip.
#pragma once
#include "bf_common.h"
#include "bf_workers.h"

namespace lbf {

// 8 waves, two per SIMD; LDS: the three weight planes of 128 beams
template <int XT, int PR, int TI>
__global__ __launch_bounds__(kThreadsH) void bf_f32_fast_kernel(BlockDesc d, int nbg, int nitems) {
    __shared__ __attribute__((aligned(16))) float pl[3 * kPlaneWords];
    item_f32_fast<XT, PR, TI>(d, xcd_remap(blockIdx.x, nitems), nbg, pl);
}

// 8 waves, two per SIMD; LDS: NS streams x 2 buffers of one A tile (and the
// incoherent beam's partial sums in the INC form)
template <int XT, int CT, int PR, int TI, int NK, int NS, bool INC>
__global__ __launch_bounds__(kThreadsH) void bf_h_fast_kernel(BlockDesc d, int nbg, int nitems) {
    __shared__ __attribute__((aligned(16))) uint32_t at[NS * 2 * kATileWords + (INC ? kIncLdsFloats : 0)];
    item_h_fast<XT, CT, PR, TI, NK, NS, INC>(d, xcd_remap(blockIdx.x, nitems), nbg, at);
}

// launch one instantiation; PR/TI/NK chosen from the block by the callers
template <int XT, int PR, int TI>
inline hipError_t launch_f32_k(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    hipLaunchKernelGGL((bf_f32_fast_kernel<XT, PR, TI>), dim3(n), dim3(kThreadsH), 0, st, d, nbg, n);
    return hipGetLastError();
}

template <int XT, int PR>
inline hipError_t launch_f32_pr(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    if (PR == PR_VOLT) return launch_f32_k<XT, PR, 1>(d, nbg, n, st);
    switch (d.t_int) {
        case 1: return launch_f32_k<XT, PR, 1>(d, nbg, n, st);
        case 2: return launch_f32_k<XT, PR, 2>(d, nbg, n, st);
        case 4: return launch_f32_k<XT, PR, 4>(d, nbg, n, st);
        case 8: return launch_f32_k<XT, PR, 8>(d, nbg, n, st);
        default: return launch_f32_k<XT, PR, 16>(d, nbg, n, st);
    }
}

template <int XT>
inline hipError_t launch_f32_xt(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    if (d.product == PR_VOLT) return launch_f32_pr<XT, PR_VOLT>(d, nbg, n, st);
    if (d.product == PR_I) return launch_f32_pr<XT, PR_I>(d, nbg, n, st);
    return launch_f32_pr<XT, PR_IQUV>(d, nbg, n, st);
}

template <int XT, int CT, int PR, int TI, int NS, bool INC>
inline void launch_h_nsi(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    const dim3 g(n), b(kThreadsH);
    switch (fast_h_ksteps(d.S)) {
        case 4: hipLaunchKernelGGL((bf_h_fast_kernel<XT, CT, PR, TI, 4, NS, INC>), g, b, 0, st, d, nbg, n); break;
        case 5: hipLaunchKernelGGL((bf_h_fast_kernel<XT, CT, PR, TI, 5, NS, INC>), g, b, 0, st, d, nbg, n); break;
        case 6: hipLaunchKernelGGL((bf_h_fast_kernel<XT, CT, PR, TI, 6, NS, INC>), g, b, 0, st, d, nbg, n); break;
        case 7: hipLaunchKernelGGL((bf_h_fast_kernel<XT, CT, PR, TI, 7, NS, INC>), g, b, 0, st, d, nbg, n); break;
        default: hipLaunchKernelGGL((bf_h_fast_kernel<XT, CT, PR, TI, 8, NS, INC>), g, b, 0, st, d, nbg, n); break;
    }
}

// the INC form (incoherent beam beside the Stokes products) only for Stokes
// with several sample streams (fuses_incoherent)
template <int XT, int CT, int PR, int TI, int NS>
inline void launch_h_ns(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    if constexpr (PR != PR_VOLT && NS >= 2) {
        if (d.inc != nullptr) {
            launch_h_nsi<XT, CT, PR, TI, NS, true>(d, nbg, n, st);
            return;
        }
    }
    launch_h_nsi<XT, CT, PR, TI, NS, false>(d, nbg, n, st);
}

template <int XT, int CT, int PR, int TI>
inline hipError_t launch_h_k(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    if constexpr (XT == XT_CF32) {
        launch_h_ns<XT, CT, PR, TI, 1>(d, nbg, n, st);      // complex f32: one stream (fast_h_streams)
    } else {
        const int ns = fast_h_streams(d);
        if (ns == 1) launch_h_ns<XT, CT, PR, TI, 1>(d, nbg, n, st);
        else if (ns == 2) launch_h_ns<XT, CT, PR, TI, 2>(d, nbg, n, st);
        else launch_h_ns<XT, CT, PR, TI, 4>(d, nbg, n, st);
    }
    return hipGetLastError();
}

template <int XT, int CT, int PR>
inline hipError_t launch_h_pr(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    if (PR == PR_VOLT) return launch_h_k<XT, CT, PR, 1>(d, nbg, n, st);
    switch (d.t_int) {
        case 1: return launch_h_k<XT, CT, PR, 1>(d, nbg, n, st);
        case 2: return launch_h_k<XT, CT, PR, 2>(d, nbg, n, st);
        case 4: return launch_h_k<XT, CT, PR, 4>(d, nbg, n, st);
        case 8: return launch_h_k<XT, CT, PR, 8>(d, nbg, n, st);
        default: return launch_h_k<XT, CT, PR, 16>(d, nbg, n, st);
    }
}

template <int XT, int CT>
inline hipError_t launch_h_xt(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    if (d.product == PR_VOLT) return launch_h_pr<XT, CT, PR_VOLT>(d, nbg, n, st);
    if (d.product == PR_I) return launch_h_pr<XT, CT, PR_I>(d, nbg, n, st);
    return launch_h_pr<XT, CT, PR_IQUV>(d, nbg, n, st);
}

template <int CT>
inline hipError_t launch_fast_h(const BlockDesc& d, hipStream_t st) {
    BlockDesc part[2];
    const int np = split_fast_h(d, part);
    for (int p = 0; p < np; ++p) {
        int nbg;
        const int n = block_items_fast_h(part[p], &nbg);
        const hipError_t e = d.xtype == XT_CI8    ? launch_h_xt<XT_CI8, CT>(part[p], nbg, n, st)
                             : d.xtype == XT_CI16 ? launch_h_xt<XT_CI16, CT>(part[p], nbg, n, st)
                                                  : launch_h_xt<XT_CF32, CT>(part[p], nbg, n, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lbf
