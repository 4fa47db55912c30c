// fft_device.h -- complex helpers of the FFT kernels (channeliser and
// channel-level dedispersion): a complex float pair, its product, and the
// 4-point DFT with the forward sign exp(-2 pi i j k / 4).
#pragma once
#include "lbf_device.h"

namespace lbf {

typedef float cfl __attribute__((ext_vector_type(2)));   // (re, im)

__device__ __forceinline__ cfl cmul(cfl a, cfl b) {
    cfl r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

__device__ __forceinline__ cfl mk(float re, float im) {
    cfl r;
    r.x = re;
    r.y = im;
    return r;
}

// 4-point DFT, forward sign: X1 = (a0 - a2) - i (a1 - a3), X3 = (a0 - a2) + i (a1 - a3)
__device__ __forceinline__ void dft4(cfl& a0, cfl& a1, cfl& a2, cfl& a3) {
    const cfl s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3, d13 = a1 - a3;
    a0 = s02 + s13;
    a2 = s02 - s13;
    a1 = mk(d02.x + d13.y, d02.y - d13.x);
    a3 = mk(d02.x - d13.y, d02.y + d13.x);
}

// LDS position of element n of a buffer: one pad element after every 32,
// which spreads the Stockham pass writes n = (j / Ns) R Ns + j mod Ns + r Ns
// of neighbouring lanes over the banks
__device__ __forceinline__ int lds_index(int n) { return n + (n >> 5); }

}  // namespace lbf
