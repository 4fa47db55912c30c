// superstation.hip -- superstation beam forming (Section 4.2 of Mol &
// Romein: a simplified beam former that combines several stations as if
// they were one):
//   out[g][c][t][p] = sum over the members s of group g of w[c][s] x[s][c][t][p]
// in member order, FP32, with unit weights when none are given.  The output
// has the station-sample layout, so superstations feed the beam former like
// stations.
//
// One thread per (group, channel, sample), both polarisations, or per group
// of P = 16 / sample bytes samples read as one 16-byte vector when T is a
// multiple of P: consecutive threads take consecutive samples of one
// (member, channel) row, so every member's loads are coalesced; the group
// table travels in the kernel arguments.  Roofline: HBM (each member sample read once, each superstation
// sample written once).
#include "lbf_device.h"
#include "lbf_launch.h"

namespace lbf {

constexpr int kSsThreads = 256;

template <int XT>
__global__ __launch_bounds__(kSsThreads) void superstation_kernel(const void* __restrict__ x,
                                                                  const float* __restrict__ w, int S, int C, int T,
                                                                  int nchunk, SsGroups gr, floatx4* __restrict__ out) {
    const long wg = blockIdx.x;
    const long gc = wg / nchunk;                            // g C + c
    const int t = (int)(wg - gc * nchunk) * kSsThreads + threadIdx.x;
    if (t >= T) return;                                     // no barrier in this kernel
    const int g = (int)(gc / C), c = (int)(gc - (long)g * C);
    float xr = 0.f, xi = 0.f, yr = 0.f, yi = 0.f;
    for (int m = gr.off[g]; m < gr.off[g + 1]; ++m) {
        const int s = gr.mem[m];
        const floatx4 v = Sample<XT>::load(x, ((size_t)s * C + c) * T + t);
        float wr = 1.f, wi = 0.f;
        if (w) {
            wr = w[2 * ((size_t)c * S + s)];
            wi = w[2 * ((size_t)c * S + s) + 1];
        }
        xr += wr * v[0] - wi * v[1];
        xi += wr * v[1] + wi * v[0];
        yr += wr * v[2] - wi * v[3];
        yi += wr * v[3] + wi * v[2];
    }
    floatx4 o;
    o[0] = xr;
    o[1] = xi;
    o[2] = yr;
    o[3] = yi;
    __builtin_nontemporal_store(o, out + ((size_t)g * C + c) * T + t);
}

// The same with P = 16 / sample bytes consecutive samples per thread, read as
// one 16-byte vector per member (T a multiple of P, so every row starts on a
// 16-byte boundary)
template <int XT>
__global__ __launch_bounds__(kSsThreads) void superstation_vec_kernel(const void* __restrict__ x,
                                                                      const float* __restrict__ w, int S, int C, int T,
                                                                      int nchunk, SsGroups gr,
                                                                      floatx4* __restrict__ out) {
    constexpr int P = 16 / Sample<XT>::bytes;
    const long wg = blockIdx.x;
    const long gc = wg / nchunk;                            // g C + c
    const int t0 = ((int)(wg - gc * nchunk) * kSsThreads + threadIdx.x) * P;
    if (t0 >= T) return;                                    // no barrier in this kernel
    const int g = (int)(gc / C), c = (int)(gc - (long)g * C);
    float acc[P][4];
#pragma unroll
    for (int h = 0; h < P; ++h) acc[h][0] = acc[h][1] = acc[h][2] = acc[h][3] = 0.f;
    for (int m = gr.off[g]; m < gr.off[g + 1]; ++m) {
        const int s = gr.mem[m];
        const intx4 q = __builtin_nontemporal_load(reinterpret_cast<const intx4*>(
            static_cast<const char*>(x) + (((size_t)s * C + c) * T + t0) * Sample<XT>::bytes));
        float f[P][4];
        if constexpr (XT == XT_CI8) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                f[h][0] = (float)((q[h] << 24) >> 24);
                f[h][1] = (float)((q[h] << 16) >> 24);
                f[h][2] = (float)((q[h] << 8) >> 24);
                f[h][3] = (float)(q[h] >> 24);
            }
        } else if constexpr (XT == XT_CI16) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                f[h][0] = (float)((q[2 * h] << 16) >> 16);
                f[h][1] = (float)(q[2 * h] >> 16);
                f[h][2] = (float)((q[2 * h + 1] << 16) >> 16);
                f[h][3] = (float)(q[2 * h + 1] >> 16);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) f[0][k] = __int_as_float(q[k]);
        }
        float wr = 1.f, wi = 0.f;
        if (w) {
            wr = w[2 * ((size_t)c * S + s)];
            wi = w[2 * ((size_t)c * S + s) + 1];
        }
#pragma unroll
        for (int h = 0; h < P; ++h) {
            acc[h][0] += wr * f[h][0] - wi * f[h][1];
            acc[h][1] += wr * f[h][1] + wi * f[h][0];
            acc[h][2] += wr * f[h][2] - wi * f[h][3];
            acc[h][3] += wr * f[h][3] + wi * f[h][2];
        }
    }
#pragma unroll
    for (int h = 0; h < P; ++h) {
        floatx4 o;
        o[0] = acc[h][0];
        o[1] = acc[h][1];
        o[2] = acc[h][2];
        o[3] = acc[h][3];
        __builtin_nontemporal_store(o, out + ((size_t)g * C + c) * T + t0 + h);
    }
}

hipError_t launch_superstation(const void* x, int xtype, int S, int C, int T, const float* w, const SsGroups& gr,
                               float* out, hipStream_t st) {
    const int P = xtype == XT_CI8 ? 4 : xtype == XT_CI16 ? 2 : 1;
    const bool vec = T % P == 0;
    const int per = kSsThreads * (vec ? P : 1);             // samples per work group
    const int nchunk = (T + per - 1) / per;
    const dim3 g((unsigned)((size_t)gr.G * C * nchunk)), b(kSsThreads);
    floatx4* o = reinterpret_cast<floatx4*>(out);
#define LBF_SS(K)                                                                                     \
    if (xtype == XT_CI8) hipLaunchKernelGGL(K<XT_CI8>, g, b, 0, st, x, w, S, C, T, nchunk, gr, o);       \
    else if (xtype == XT_CI16) hipLaunchKernelGGL(K<XT_CI16>, g, b, 0, st, x, w, S, C, T, nchunk, gr, o); \
    else hipLaunchKernelGGL(K<XT_CF32>, g, b, 0, st, x, w, S, C, T, nchunk, gr, o);
    if (vec) {
        LBF_SS(superstation_vec_kernel)
    } else {
        LBF_SS(superstation_kernel)
    }
#undef LBF_SS
    return hipGetLastError();
}

}  // namespace lbf
