// channelize.hip -- the FFT that splits each subband into channels (Section
// 4.2 of Mol & Romein), with the sample-granularity part of delay
// compensation (Section 3): station s contributes the window of T_sb subband
// samples starting shift[s] samples into its row (samples outside the row
// read as zero); every station's and polarisation's window is cut into
// consecutive groups of nch samples, and the FFT of a group (forward sign,
// no window function, no scaling) gives one sample of each of the subband's
// nch channels, lowest frequency first (channel q = FFT bin (q + nch/2) mod
// nch).
//
// One work group per tile of kChTile (2048) consecutive samples of one
// (station, subband) row, both polarisations, in LDS (33 KiB with padding,
// so four groups share a compute unit):
//   1. coalesced loads of the tile's samples (the station's shifted window),
//      16-byte vectors of 1, 2 or 4 samples when the window, widened to
//      16-byte boundaries, lies inside the row (any shift), single samples
//      otherwise; converted to float;
//   2. Stockham passes over the tile's kChTile / nch spectra: radix 16
//      while four or more bits of nch remain, then radix 4, then radix 2
//      (two radix-16 passes for 256 channels); each pass reads all its
//      inputs, meets a barrier, and writes in place; the spectra come out in
//      natural order;
//   3. stores in channel order, consecutive lanes on consecutive output
//      times of one channel: out[s][sb nch + q][t][p], 16 bytes (both
//      polarisations) per lane.
// Roofline: HBM (every sample read once, every channel sample written once).
#include "fft_device.h"
#include "lbf_launch.h"

namespace lbf {

constexpr int kChThreads = 256;
constexpr int kChWords = kChTile + kChTile / 32;      // LDS words per polarisation, padded

// One radix-R (16, 4 or 2) pass of span Ns over every spectrum of the tile;
// a task is one (butterfly, polarisation).  Twiddles exp(-2 pi i k r / (R Ns)),
// k = j mod Ns: w[1] from sincospif (exact argument: R Ns is a power of two),
// the other powers as products built by squaring.
template <int R>
__device__ __forceinline__ void ch_pass(cfl* buf, int nch, int Ns) {
    constexpr int PER_POL = kChTile / R;              // butterflies per polarisation
    constexpr int TPT = 2 * PER_POL / kChThreads;     // tasks per thread
    static_assert(TPT >= 1 && 2 * PER_POL % kChThreads == 0, "whole tasks per thread");
    const int nb = nch / R;                           // butterflies per spectrum
    cfl v[TPT][R];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int task = threadIdx.x + kChThreads * u;
        const int p = task / PER_POL, g = task - p * PER_POL;
        const int m = g / nb, j = g - m * nb;
        const cfl* pb = buf + p * kChWords;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = pb[lds_index(m * nch + j + r * nb)];
        if (Ns > 1) {
            float sn, cs;
            sincospif(-2.0f * (float)(j % Ns) / (float)(R * Ns), &sn, &cs);
            cfl w[R];
            w[1] = mk(cs, sn);
            if (R >= 4) {
                w[2] = cmul(w[1], w[1]);
                w[3] = cmul(w[1], w[2]);
            }
            if (R == 16) {
                w[4] = cmul(w[2], w[2]);
                w[8] = cmul(w[4], w[4]);
                w[5] = cmul(w[1], w[4]);
                w[6] = cmul(w[2], w[4]);
                w[7] = cmul(w[3], w[4]);
#pragma unroll
                for (int r = 9; r < R; ++r) w[r] = cmul(w[r - 8], w[8]);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], w[r]);
        }
        if (R == 2) {
            const cfl a = v[u][0], b = v[u][1];
            v[u][0] = a + b;
            v[u][1] = a - b;
        } else if (R == 4) {
            dft4(v[u][0], v[u][1], v[u][2], v[u][3]);
        } else {
            dft16(v[u]);
        }
    }
    __syncthreads();                                  // every read of this pass before any write
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int task = threadIdx.x + kChThreads * u;
        const int p = task / PER_POL, g = task - p * PER_POL;
        const int m = g / nb, j = g - m * nb;
        const int d0 = m * nch + (j / Ns) * Ns * R + j % Ns;
        cfl* pb = buf + p * kChWords;
#pragma unroll
        for (int r = 0; r < R; ++r) pb[lds_index(d0 + r * Ns)] = v[u][r];
    }
    __syncthreads();                                  // the writes before the next pass reads
}

// The samples of one 16-byte vector, each as (x re, x im, y re, y im):
// 4 complex int8 samples, 2 complex int16 samples or 1 complex float sample
template <int XT>
__device__ __forceinline__ void vec_samples(const intx4 q, float (*f)[4]) {
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
}

template <int XT>
__global__ __launch_bounds__(kChThreads) void channelize_kernel(const void* __restrict__ x, int NSB, int Tin, int Tsb,
                                                                int nch, const int* __restrict__ shift, int ntile,
                                                                floatx4* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) cfl buf[2 * kChWords];
    const int M = kChTile / nch;                      // spectra per tile
    const int T2 = Tsb / nch;
    const long wg = blockIdx.x;
    const long row = wg / ntile;                      // s NSB + sb
    const int t0 = (int)(wg - row * ntile) * M;
    const int nvalid = min(M, T2 - t0) * nch;         // samples of the tile inside the window
    const int s = (int)(row / NSB), sb = (int)(row - (long)s * NSB);
    const long t_first = (long)t0 * nch + (shift ? shift[s] : 0);   // row sample of the tile's first
    constexpr int P = 16 / Sample<XT>::bytes;           // samples per 16-byte vector
    const size_t r0 = (size_t)row * Tin;
    // 16-byte vectors from the aligned sample at or before the window's first
    // one (off samples earlier) to past its last, when all of them lie inside
    // the row
    const int off = t_first >= 0 ? (int)((r0 + t_first) % P) : 0;
    const int nv = (off + nvalid + P - 1) / P;
    if (t_first >= off && t_first + nvalid <= Tin && t_first - off + (long)nv * P <= Tin) {
        // P samples per lane and load; sample h of vector iv is tile sample
        // iv P + h - off, zero past the window
        const intx4* xv =
            reinterpret_cast<const intx4*>(static_cast<const char*>(x) + (r0 + t_first - off) * Sample<XT>::bytes);
        for (int iv = threadIdx.x; iv < (kChTile + off + P - 1) / P; iv += kChThreads) {
            intx4 q = {0, 0, 0, 0};
            if (iv < nv) q = __builtin_nontemporal_load(xv + iv);
            float f[P][4];
            vec_samples<XT>(q, f);
#pragma unroll
            for (int h = 0; h < P; ++h) {
                const int i = iv * P + h - off;
                if (i < 0 || i >= kChTile) continue;
                const bool in = i < nvalid;
                buf[lds_index(i)] = mk(in ? f[h][0] : 0.f, in ? f[h][1] : 0.f);
                buf[kChWords + lds_index(i)] = mk(in ? f[h][2] : 0.f, in ? f[h][3] : 0.f);
            }
        }
    } else {
        for (int i = threadIdx.x; i < kChTile; i += kChThreads) {
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            const long t = t_first + i;
            if (i < nvalid && t >= 0 && t < Tin) v = Sample<XT>::load(x, r0 + (size_t)t);
            buf[lds_index(i)] = mk(v[0], v[1]);
            buf[kChWords + lds_index(i)] = mk(v[2], v[3]);
        }
    }
    __syncthreads();
    // radix 16 while four or more bits of nch remain, then 4, then 2
    int Ns = 1, L = __builtin_ctz(nch);
    for (; L >= 4; L -= 4, Ns *= 16) ch_pass<16>(buf, nch, Ns);
    for (; L >= 2; L -= 2, Ns *= 4) ch_pass<4>(buf, nch, Ns);
    if (L == 1) ch_pass<2>(buf, nch, Ns);
    const size_t C = (size_t)NSB * nch;
    for (int e = threadIdx.x; e < kChTile; e += kChThreads) {
        const int q = e / M, m = e - q * M;
        if (t0 + m >= T2) continue;
        const int n = m * nch + ((q + nch / 2) & (nch - 1));
        const cfl a = buf[lds_index(n)], b = buf[kChWords + lds_index(n)];
        floatx4 o;
        o[0] = a.x;
        o[1] = a.y;
        o[2] = b.x;
        o[3] = b.y;
        __builtin_nontemporal_store(o, out + ((size_t)s * C + (size_t)sb * nch + q) * T2 + t0 + m);
    }
}

hipError_t launch_channelize(const void* x, int xtype, int S, int NSB, int Tin, int Tsb, int nch, const int* shift,
                             float* out, hipStream_t st) {
    const int M = kChTile / nch;
    const int ntile = (Tsb / nch + M - 1) / M;
    const dim3 g((unsigned)((size_t)S * NSB * ntile)), b(kChThreads);
    floatx4* o = reinterpret_cast<floatx4*>(out);
    if (xtype == XT_CI8)
        hipLaunchKernelGGL(channelize_kernel<XT_CI8>, g, b, 0, st, x, NSB, Tin, Tsb, nch, shift, ntile, o);
    else if (xtype == XT_CI16)
        hipLaunchKernelGGL(channelize_kernel<XT_CI16>, g, b, 0, st, x, NSB, Tin, Tsb, nch, shift, ntile, o);
    else
        hipLaunchKernelGGL(channelize_kernel<XT_CF32>, g, b, 0, st, x, NSB, Tin, Tsb, nch, shift, ntile, o);
    return hipGetLastError();
}

}  // namespace lbf
