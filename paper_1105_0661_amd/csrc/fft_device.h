// fft_device.h -- complex helpers of the FFT kernels (channeliser and
// channel-level dedispersion): a complex float pair, its product, the 4- and
// 16-point DFTs with the forward sign exp(-2 pi i j k / n), and the padded
// LDS index.
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

// 16-point DFT, forward sign, in place: with x[4a + b], 4-point DFTs over a
// give Y_b[c]; then Y_b[c] W16^(b c); then 4-point DFTs over b give X[c + 4d]
__device__ __forceinline__ void dft16(cfl* v) {
    cfl y[4][4];                                            // y[b][c]
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        cfl a0 = v[b], a1 = v[4 + b], a2 = v[8 + b], a3 = v[12 + b];
        dft4(a0, a1, a2, a3);
        y[b][0] = a0; y[b][1] = a1; y[b][2] = a2; y[b][3] = a3;
    }
    const float c8 = 0.92387953251128674f, s8 = 0.38268343236508978f, h = 0.70710678118654752f;
    // W16^(b c) for b c = 1, 2, 3, 2, 4, 6, 3, 6, 9 (cos and sin of pi/8 and pi/4)
    y[1][1] = cmul(y[1][1], mk(c8, -s8));
    y[1][2] = cmul(y[1][2], mk(h, -h));
    y[1][3] = cmul(y[1][3], mk(s8, -c8));
    y[2][1] = cmul(y[2][1], mk(h, -h));
    y[2][2] = mk(y[2][2].y, -y[2][2].x);
    y[2][3] = cmul(y[2][3], mk(-h, -h));
    y[3][1] = cmul(y[3][1], mk(s8, -c8));
    y[3][2] = cmul(y[3][2], mk(-h, -h));
    y[3][3] = cmul(y[3][3], mk(-c8, s8));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cfl a0 = y[0][c], a1 = y[1][c], a2 = y[2][c], a3 = y[3][c];
        dft4(a0, a1, a2, a3);
        v[c] = a0; v[c + 4] = a1; v[c + 8] = a2; v[c + 12] = a3;
    }
}

// LDS position of element n of a buffer: one pad element after every 32,
// which spreads the Stockham pass writes n = (j / Ns) R Ns + j mod Ns + r Ns
// of neighbouring lanes over the banks
__device__ __forceinline__ int lds_index(int n) { return n + (n >> 5); }

}  // namespace lbf
