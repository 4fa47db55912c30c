// superstation.hip -- superstation beam forming (Section 4.2 of Mol &
// Romein: a simplified beam former that combines several stations as if
// they were one):
//   out[g][c][t][p] = sum over the members s of group g of w[c][s] x[s][c][t][p]
// in member order, FP32, with unit weights when none are given.  The output
// has the station-sample layout, so superstations feed the beam former like
// stations.
//
// One thread per (group, channel, sample), both polarisations: consecutive
// threads take consecutive samples of one (member, channel) row, so every
// member's loads are coalesced; the group table travels in the kernel
// arguments.  Roofline: HBM (each member sample read once, each superstation
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

hipError_t launch_superstation(const void* x, int xtype, int S, int C, int T, const float* w, const SsGroups& gr,
                               float* out, hipStream_t st) {
    const int nchunk = (T + kSsThreads - 1) / kSsThreads;
    const dim3 g((unsigned)((size_t)gr.G * C * nchunk)), b(kSsThreads);
    floatx4* o = reinterpret_cast<floatx4*>(out);
    if (xtype == XT_CI8) hipLaunchKernelGGL(superstation_kernel<XT_CI8>, g, b, 0, st, x, w, S, C, T, nchunk, gr, o);
    else if (xtype == XT_CI16) hipLaunchKernelGGL(superstation_kernel<XT_CI16>, g, b, 0, st, x, w, S, C, T, nchunk, gr, o);
    else hipLaunchKernelGGL(superstation_kernel<XT_CF32>, g, b, 0, st, x, w, S, C, T, nchunk, gr, o);
    return hipGetLastError();
}

}  // namespace lbf
