// aux_kernels.hip -- weights (FP64), unfused Stokes, final-order transpose and
// the incoherent beam.
#include <algorithm>

#include "lbf_device.h"
#include "lbf_launch.h"

namespace lbf {

// ---------------------------------------------------------------------------
// Weights (Section 3 and Section 4.3 of Mol & Romein): the delay of station s
// for beam b, tau = p_s . (u_b - u_ref) / c0 - delta_s (delta_s: the station's
// residual delay after a whole-sample shift, Section 3), and the phase-shift
// weight w = exp(-2 pi i frac(f tau)).  Everything up to the final rounding is FP64:
// f * tau spans many turns and only its fractional part matters.
// One thread per (b, s) and group of kWChan channels: tau once, then one
// weight per channel; threads of a block are consecutive (b, s), so each
// channel's stores are coalesced.
// ---------------------------------------------------------------------------
constexpr double kC0 = 299792458.0;
constexpr int kWChan = 32;

// cos(2 pi r) and sin(2 pi r) for |r| <= 1/2, in FP64.  Quarter-turn
// reduction r = q/4 + u (q = rint(4r), |u| <= 1/8, u exact), then the Taylor
// series of sin and cos at theta = 2 pi u (|theta| <= pi/4, so the first
// omitted terms, theta^17/17! and theta^18/18!, are below 5e-17), then the
// quadrant q mod 4 by symmetry: swap for odd q, and sign flips.  About twenty
// FP64 operations instead of a general-argument library call.
struct CisCoef {
    double s[7];   // -1/15!, 1/13!, ..., -1/3!  (Horner order)
    double c[8];   //  1/16!, -1/14!, ..., -1/2!
};

__device__ inline CisCoef cis_coef() {
    CisCoef k;
    k.s[0] = -1.0 / 1307674368000.0;
    k.s[1] = 1.0 / 6227020800.0;
    k.s[2] = -1.0 / 39916800.0;
    k.s[3] = 1.0 / 362880.0;
    k.s[4] = -1.0 / 5040.0;
    k.s[5] = 1.0 / 120.0;
    k.s[6] = -1.0 / 6.0;
    k.c[0] = 1.0 / 20922789888000.0;
    k.c[1] = -1.0 / 87178291200.0;
    k.c[2] = 1.0 / 479001600.0;
    k.c[3] = -1.0 / 3628800.0;
    k.c[4] = 1.0 / 40320.0;
    k.c[5] = -1.0 / 720.0;
    k.c[6] = 1.0 / 24.0;
    k.c[7] = -0.5;
    return k;
}

// (cos 2 pi r, -sin 2 pi r): the weight of a fractional turn r
__device__ inline void weight_of_turn(double r, const CisCoef& k, double* wr, double* wi) {
    const double q = rint(4.0 * r);
    const double u = __builtin_fma(q, -0.25, r);
    const double th = u * 6.283185307179586;
    const double t2 = th * th;
    double ps = k.s[0];
#pragma unroll
    for (int i = 1; i < 7; ++i) ps = __builtin_fma(ps, t2, k.s[i]);
    const double sn = __builtin_fma(th * t2, ps, th);
    double pc = k.c[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) pc = __builtin_fma(pc, t2, k.c[i]);
    const double cs = __builtin_fma(t2, pc, 1.0);
    // quadrant q (mod 4): (cos, sin) = (c, s), (-s, c), (-c, -s), (s, -c)
    const int quad = (int)q;
    const bool odd = (quad & 1) != 0;
    const uint64_t x = __builtin_bit_cast(uint64_t, odd ? sn : cs);
    const uint64_t y = __builtin_bit_cast(uint64_t, odd ? cs : sn);
    const uint64_t negx = (uint64_t)((quad + 1) & 2) << 62;
    const uint64_t negy = ((uint64_t)(quad & 2) << 62) ^ 0x8000000000000000ull;   // and -sin
    *wr = __builtin_bit_cast(double, x ^ negx);
    *wi = __builtin_bit_cast(double, y ^ negy);
}

template <int WT>
__global__ __launch_bounds__(256) void weights_kernel(const double* __restrict__ pos, int S,
                                                      const double* __restrict__ dir, int B, double rx, double ry,
                                                      double rz, const double* __restrict__ delay,
                                                      const double* __restrict__ freq, int C, void* w, double* tau) {
    const int bs = blockIdx.x * blockDim.x + threadIdx.x;
    if (bs >= B * S) return;
    const int b = bs / S, s = bs - b * S;
    const double dx = dir[3 * b + 0] - rx, dy = dir[3 * b + 1] - ry, dz = dir[3 * b + 2] - rz;
    const double proj = pos[3 * s + 0] * dx + pos[3 * s + 1] * dy + pos[3 * s + 2] * dz;
    const double t = proj / kC0 - (delay != nullptr ? delay[s] : 0.0);
    if (tau != nullptr && blockIdx.y == 0) tau[bs] = t;
    const int c0 = blockIdx.y * kWChan, c1 = min(C, c0 + kWChan);
    const size_t BS = (size_t)B * S;
    // the series coefficients stay in registers across the channel loop
    CisCoef k = cis_coef();
#pragma unroll
    for (int i = 0; i < 7; ++i) __asm__ volatile("" : "+v"(k.s[i]));
#pragma unroll
    for (int i = 0; i < 8; ++i) __asm__ volatile("" : "+v"(k.c[i]));
    for (int c = c0; c < c1; ++c) {
        const double m = freq[c] * t;
        const double r = m - rint(m);          // fractional turn in [-0.5, 0.5]
        double wr, wi;
        weight_of_turn(r, k, &wr, &wi);
        const size_t i = (size_t)c * BS + bs;
        if (WT == CT_F32) {
            float2 v;
            v.x = (float)wr;
            v.y = (float)wi;
            reinterpret_cast<float2*>(w)[i] = v;
        } else if (WT == CT_F16) {
            // round-to-odd to f32, then the packed hardware conversion (RNE)
            typedef _Float16 h2 __attribute__((ext_vector_type(2)));
            const h2 v = {(_Float16)f64_to_f32_round_odd(wr), (_Float16)f64_to_f32_round_odd(wi)};
            reinterpret_cast<uint32_t*>(w)[i] = __builtin_bit_cast(uint32_t, v);
        } else {
            typedef __bf16 b2 __attribute__((ext_vector_type(2)));
            const b2 v = {(__bf16)f64_to_f32_round_odd(wr), (__bf16)f64_to_f32_round_odd(wi)};
            reinterpret_cast<uint32_t*>(w)[i] = __builtin_bit_cast(uint32_t, v);
        }
    }
}

hipError_t launch_weights(const double* pos, int S, const double* dir, int B, double rx, double ry, double rz,
                          const double* delay, const double* freq, int C, int wtype, void* w, double* tau,
                          hipStream_t st) {
    const int bs = B * S;
    dim3 g((unsigned)((bs + 255) / 256), (unsigned)((C + kWChan - 1) / kWChan)), b(256);
    if (wtype == CT_F32)
        hipLaunchKernelGGL(weights_kernel<CT_F32>, g, b, 0, st, pos, S, dir, B, rx, ry, rz, delay, freq, C, w, tau);
    else if (wtype == CT_F16)
        hipLaunchKernelGGL(weights_kernel<CT_F16>, g, b, 0, st, pos, S, dir, B, rx, ry, rz, delay, freq, C, w, tau);
    else
        hipLaunchKernelGGL(weights_kernel<CT_BF16>, g, b, 0, st, pos, S, dir, B, rx, ry, rz, delay, freq, C, w, tau);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Unfused Stokes detection + integration (Section 4.5; Section 5.1):
// y [C][B][T][2] complex f32 -> s [C'][B][T'][K].  One thread per output
// (c', b, t'); any t_int | T and f_int | C.  Sum order: channel, then time.
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(256) void stokes_kernel(const floatx4* __restrict__ y, int B, int C, int T, int t_int,
                                                     int f_int, float* __restrict__ s) {
    const int T2 = T / t_int, C2 = C / f_int;
    const size_t n = (size_t)C2 * B * T2;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int t2 = (int)(i % T2);
        const size_t cb = i / T2;
        const int b = (int)(cb % B);
        const int c2 = (int)(cb / B);
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int dc = 0; dc < f_int; ++dc) {
            const int c = c2 * f_int + dc;
            const floatx4* row = y + ((size_t)c * B + b) * T + (size_t)t2 * t_int;
            for (int dt = 0; dt < t_int; ++dt) {
                const floatx4 v = row[dt];
                const float xx = v[0] * v[0] + v[1] * v[1];
                const float yy = v[2] * v[2] + v[3] * v[3];
                acc[0] += xx + yy;
                if (K == 4) {
                    acc[1] += xx - yy;
                    acc[2] += 2.0f * (v[0] * v[2] + v[1] * v[3]);
                    acc[3] += 2.0f * (v[1] * v[2] - v[0] * v[3]);
                }
            }
        }
        if (K == 4) {
            floatx4 o;
            o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3];
            reinterpret_cast<floatx4*>(s)[i] = o;
        } else {
            s[i] = acc[0];
        }
    }
}

// Power-of-two t_int: G = min(t_int, 64) consecutive lanes share an output
// (c', b, t').  Lane g reads samples t'*t_int + g + G*j (j < t_int/G) of the
// f_int channels, so a wave's loads are 64 consecutive 16-byte samples of one
// (c, b) row; the G partial sums meet in a butterfly of lane exchanges and
// lane g = 0 stores them.  Sum order: channel, then the lane's samples, then
// the butterfly.
template <int K>
__global__ __launch_bounds__(256) void stokes_wave_kernel(const floatx4* __restrict__ y, int B, int C, int T,
                                                          int t_int, int f_int, float* __restrict__ s) {
    const int T2 = T / t_int, C2 = C / f_int;
    const int G = t_int < kWave ? t_int : kWave;
    const size_t slots = (size_t)C2 * B * T2 * G;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i - threadIdx.x % kWave < slots;
         i += (size_t)gridDim.x * blockDim.x) {
        // whole waves stay in the loop together (the exchanges need every
        // lane); lanes past the end add zeros and store nothing
        const bool live = i < slots;
        const size_t o = live ? i / G : 0;
        const int g = (int)(i % G);
        const int t2 = (int)(o % T2);
        const size_t cb = o / T2;
        const int b = (int)(cb % B);
        const int c2 = (int)(cb / B);
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        if (live) {
            for (int dc = 0; dc < f_int; ++dc) {
                const floatx4* row = y + ((size_t)(c2 * f_int + dc) * B + b) * T + (size_t)t2 * t_int + g;
                for (int j = 0; j < t_int / G; ++j) {
                    const floatx4 v = row[(size_t)j * G];
                    const float xx = v[0] * v[0] + v[1] * v[1];
                    const float yy = v[2] * v[2] + v[3] * v[3];
                    acc[0] += xx + yy;
                    if (K == 4) {
                        acc[1] += xx - yy;
                        acc[2] += 2.0f * (v[0] * v[2] + v[1] * v[3]);
                        acc[3] += 2.0f * (v[1] * v[2] - v[0] * v[3]);
                    }
                }
            }
        }
        for (int m = G / 2; m >= 1; m /= 2)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += __shfl_xor(acc[k], m, kWave);
        if (live && g == 0) {
            if (K == 4) {
                floatx4 v;
                v[0] = acc[0]; v[1] = acc[1]; v[2] = acc[2]; v[3] = acc[3];
                reinterpret_cast<floatx4*>(s)[o] = v;
            } else {
                s[o] = acc[0];
            }
        }
    }
}

hipError_t launch_stokes(const float* y, int B, int C, int T, int product, int t_int, int f_int, float* s,
                         hipStream_t st) {
    const floatx4* yy = reinterpret_cast<const floatx4*>(y);
    if ((t_int & (t_int - 1)) == 0) {
        const size_t slots = (size_t)(C / f_int) * B * (T / t_int) * (t_int < kWave ? t_int : kWave);
        size_t blocks = (slots + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        if (product == PR_IQUV)
            hipLaunchKernelGGL(stokes_wave_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, yy, B, C, T, t_int,
                               f_int, s);
        else
            hipLaunchKernelGGL(stokes_wave_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, yy, B, C, T, t_int,
                               f_int, s);
        return hipGetLastError();
    }
    const size_t n = (size_t)(C / f_int) * B * (T / t_int);
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    if (product == PR_IQUV)
        hipLaunchKernelGGL(stokes_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, yy, B, C, T, t_int, f_int, s);
    else
        hipLaunchKernelGGL(stokes_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, yy, B, C, T, t_int, f_int, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final order (Section 4.6): out[b][k][t][c] = in[c][b][t][k].  Viewing the
// input as a C2 x M matrix (M = B*T2*K), 32x32 tiles go through LDS so both
// the reads (along m) and the writes (along c) are coalesced.
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(256) void transpose_kernel(const E* __restrict__ in, int C2, int B, int T2, int K,
                                                        E* __restrict__ out) {
    __shared__ E tile[32][33];
    const long M = (long)B * T2 * K;
    const long m0 = (long)blockIdx.x * 32;
    const int c0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int c = c0 + r;
        const long m = m0 + tx;
        if (c < C2 && m < M) tile[r][tx] = in[(size_t)c * M + m];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const long m = m0 + r;
        const int c = c0 + tx;
        if (c < C2 && m < M) {
            const int k = (int)(m % K);
            const long bt = m / K;
            const int t = (int)(bt % T2);
            const int b = (int)(bt / T2);
            out[(((size_t)b * K + k) * T2 + t) * C2 + c] = tile[tx][r];
        }
    }
}

// The same reorder with 16-byte accesses (Q = T2 K and C2 multiples of the
// elements per 16 bytes, both buffers 16-byte aligned): for one beam b, a
// tile of 64 channels x 64 consecutive (t, k) values moves through LDS;
// reads are 64-element runs of one channel's (t, k) values, writes 64-element
// runs of channels of one (k, t) row of the final order.
template <typename E>
__global__ __launch_bounds__(256) void reorder_final_vec_kernel(const E* __restrict__ in, int C2, int B, int T2, int K,
                                                                E* __restrict__ out) {
    constexpr int V = 16 / sizeof(E);            // elements per 16-byte access
    constexpr int LPR = 64 / V;                  // lanes per 64-element row
    constexpr int RPP = 256 / LPR;               // rows per pass
    __shared__ E tile[64][65];
    const long Q = (long)T2 * K;
    const long q0 = (long)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64, b = blockIdx.z;
    const int l = threadIdx.x % LPR, rr = threadIdx.x / LPR;
#pragma unroll
    for (int p = 0; p < 64 / RPP; ++p) {
        const int r = p * RPP + rr, c = c0 + r;
        const long q = q0 + V * l;
        if (c < C2 && q < Q) {
            const floatx4 v = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(in + ((size_t)c * B + b) * Q + q));
            const E* e = reinterpret_cast<const E*>(&v);
#pragma unroll
            for (int i = 0; i < V; ++i) tile[r][V * l + i] = e[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 64 / RPP; ++p) {
        const int r = p * RPP + rr;
        const long q = q0 + r;
        const int c = c0 + V * l;
        if (q < Q && c < C2) {
            const long t = q / K;
            const int k = (int)(q - t * K);
            floatx4 v;
            E* e = reinterpret_cast<E*>(&v);
#pragma unroll
            for (int i = 0; i < V; ++i) e[i] = tile[V * l + i][r];
            __builtin_nontemporal_store(v, reinterpret_cast<floatx4*>(out + (((size_t)b * K + k) * T2 + t) * C2 + c));
        }
    }
}

hipError_t launch_transpose(const void* in, int C2, int B, int T2, int K, int elem_bytes, void* out,
                            hipStream_t st) {
    const long Q = (long)T2 * K;
    const int V = 16 / elem_bytes;
    if (Q % V == 0 && C2 % V == 0 && B <= 65535 && (Q + 63) / 64 < (1L << 31) &&
        (((uintptr_t)in | (uintptr_t)out) & 15) == 0) {
        dim3 g((unsigned)((Q + 63) / 64), (unsigned)((C2 + 63) / 64), (unsigned)B), b(256);
        if (elem_bytes == 4)
            hipLaunchKernelGGL(reorder_final_vec_kernel<float>, g, b, 0, st, (const float*)in, C2, B, T2, K,
                               (float*)out);
        else
            hipLaunchKernelGGL(reorder_final_vec_kernel<float2>, g, b, 0, st, (const float2*)in, C2, B, T2, K,
                               (float2*)out);
        return hipGetLastError();
    }
    const long M = (long)B * T2 * K;
    dim3 g((unsigned)((M + 31) / 32), (unsigned)((C2 + 31) / 32)), b(256);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(transpose_kernel<float>, g, b, 0, st, (const float*)in, C2, B, T2, K, (float*)out);
    else
        hipLaunchKernelGGL(transpose_kernel<float2>, g, b, 0, st, (const float2*)in, C2, B, T2, K, (float2*)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Channel-major staging s[c][m][b] (rows of ldb >= B values) -> out[b][m][c]
// (Section 4.6), output rows of ldo >= C2 channels (a chunk of the channels
// goes to columns [0, C2) of rows that hold all of them).  For Stokes the staging is [c][t'][beam][k]: m = t' and the
// B index runs over (beam, k) pairs, so out[(beam k)][t'][c] is the final
// [beam][k][t'][c].  Each work group moves a
// 64-channel x 64-beam tile of one m through LDS: reads are 256-byte runs
// along b, writes 256-byte runs along c, 16 bytes per lane where the rows allow
// it (VEC: ldb and C2 multiples of 4).  With ldb a multiple of 32 every read
// run starts on a 128-byte line.  The order in which the grid walks the tiles
// (`walk`) is the one measured fastest for the row alignment: 0 m, channel
// tile, beam tile (any M); 1 channel tile, m, beam tile (128-byte-aligned
// rows); 2 beam tile, channel tile, m (other rows).  The 16-byte accesses are
// non-temporal: the staging is read once and the output not again here
// (timed alone: 0.322 against 0.338 ms for 0.8 GB of Stokes, 1.222 against
// 1.252 ms for 3 GB).
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ __launch_bounds__(256) void stage_to_beam_major_kernel(const float* __restrict__ in, int C2, int M, int B,
                                                                  int ldb, float* __restrict__ out, size_t ldo,
                                                                  int walk) {
    __shared__ float tile[64][65];
    int bt, ct;
    size_t m;
    if (walk == 0) { m = blockIdx.x; ct = blockIdx.y; bt = blockIdx.z; }
    else if (walk == 1) { ct = blockIdx.x; m = blockIdx.y; bt = blockIdx.z; }
    else { bt = blockIdx.x; ct = blockIdx.y; m = blockIdx.z; }
    const int b0 = bt * 64, c0 = ct * 64;
    const int q = threadIdx.x & 15, rr = threadIdx.x >> 4;       // 16 lanes x 4 elements per row
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int r = p * 16 + rr, c = c0 + r, b = b0 + 4 * q;
        if (c >= C2) continue;
        const float* src = in + ((size_t)c * M + m) * ldb + b;
        if (VEC && b + 3 < B) {
            const floatx4 v = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(src));
            tile[r][4 * q + 0] = v[0];
            tile[r][4 * q + 1] = v[1];
            tile[r][4 * q + 2] = v[2];
            tile[r][4 * q + 3] = v[3];
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (b + e < B) tile[r][4 * q + e] = src[e];
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int rb = p * 16 + rr, b = b0 + rb, c = c0 + 4 * q;
        if (b >= B) continue;
        float* dst = out + ((size_t)b * M + m) * ldo + c;
        if (VEC && c + 3 < C2) {
            floatx4 v;
            v[0] = tile[4 * q + 0][rb];
            v[1] = tile[4 * q + 1][rb];
            v[2] = tile[4 * q + 2][rb];
            v[3] = tile[4 * q + 3][rb];
            __builtin_nontemporal_store(v, reinterpret_cast<floatx4*>(dst));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (c + e < C2) dst[e] = tile[4 * q + e][rb];
        }
    }
}

hipError_t launch_stage_to_beam_major(const float* stage, int C2, int M, int B, int ldb, float* out, size_t ldo,
                                      hipStream_t st) {
    const unsigned nm = (unsigned)M, nc = (unsigned)((C2 + 63) / 64), nb = (unsigned)((B + 63) / 64);
    const int walk = M > 65535 || nc > 65535 ? 0 : ldb % 32 == 0 ? 1 : 2;
    const dim3 g = walk == 0 ? dim3(nm, nc, nb) : walk == 1 ? dim3(nc, nm, nb) : dim3(nb, nc, nm), b(256);
    const bool aligned = ((reinterpret_cast<uintptr_t>(stage) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (aligned && ldb % 4 == 0 && C2 % 4 == 0 && ldo % 4 == 0)
        hipLaunchKernelGGL(stage_to_beam_major_kernel<true>, g, b, 0, st, stage, C2, M, B, ldb, out, ldo, walk);
    else
        hipLaunchKernelGGL(stage_to_beam_major_kernel<false>, g, b, 0, st, stage, C2, M, B, ldb, out, ldo, walk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Channel integration out of the staging (Section 3, Section 5.1): the fast
// workers stage each channel's Stokes parameters integrated in time, and the
// sums over groups of F adjacent channels are formed here, in channel order,
// while the staging is read once.  Both kernels add the F values in the same
// order, so the two output orders hold the same bits.
// ---------------------------------------------------------------------------

// staging s[c][m][b] (rows of ldb, C2 channels, a multiple of F) ->
// out[b][m][c'] (rows of ldo), c' = c / F.  A work group moves 64 channels x
// 64 beams of one m through LDS: 256-byte reads along b (16 bytes per lane
// where the rows allow it), then 64 / F consecutive sums per beam.
template <bool VEC>
__global__ __launch_bounds__(256) void stage_sum_to_beam_major_kernel(const float* __restrict__ in, int C2, int M, int B,
                                                                      int ldb, int F, float* __restrict__ out,
                                                                      size_t ldo) {
    __shared__ float tile[64][65];
    const size_t m = blockIdx.x;
    const int c0 = blockIdx.y * 64, b0 = blockIdx.z * 64;
    const int q = threadIdx.x & 15, rr = threadIdx.x >> 4;       // 16 lanes x 4 elements per row
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int r = p * 16 + rr, c = c0 + r, b = b0 + 4 * q;
        if (c >= C2) continue;
        const float* src = in + ((size_t)c * M + m) * ldb + b;
        if (VEC && b + 3 < B) {
            const floatx4 v = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(src));
#pragma unroll
            for (int e = 0; e < 4; ++e) tile[r][4 * q + e] = v[e];
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (b + e < B) tile[r][4 * q + e] = src[e];
        }
    }
    __syncthreads();
    const int G = 64 / F;                                        // sums per beam in the tile
    for (int v = threadIdx.x; v < 64 * G; v += 256) {
        const int bl = v / G, g = v - bl * G;
        const int b = b0 + bl, c = c0 + g * F;
        if (b >= B || c >= C2) continue;                          // C2 is a multiple of F: the group is whole
        float sum = tile[g * F][bl];
        for (int j = 1; j < F; ++j) sum += tile[g * F + j][bl];
        out[((size_t)b * M + m) * ldo + c / F] = sum;
    }
}

hipError_t launch_stage_sum_to_beam_major(const float* stage, int C2, int M, int B, int ldb, int F, float* out,
                                          size_t ldo, hipStream_t st) {
    const dim3 g((unsigned)M, (unsigned)((C2 + 63) / 64), (unsigned)((B + 63) / 64)), b(256);
    const bool aligned = (reinterpret_cast<uintptr_t>(stage) & 15) == 0;
    if (aligned && ldb % 4 == 0)
        hipLaunchKernelGGL(stage_sum_to_beam_major_kernel<true>, g, b, 0, st, stage, C2, M, B, ldb, F, out, ldo);
    else
        hipLaunchKernelGGL(stage_sum_to_beam_major_kernel<false>, g, b, 0, st, stage, C2, M, B, ldb, F, out, ldo);
    return hipGetLastError();
}

// staging s[c][m][b] (rows of ldb, C2 channels) -> out[c'][m][b] (rows of B):
// one thread per 4 consecutive b (16-byte loads and stores) where the rows
// and buffers allow it, else per b.
template <bool VEC>
__global__ __launch_bounds__(256) void stage_sum_channels_kernel(const float* __restrict__ in, int C2, int M, int B,
                                                                 int ldb, int F, float* __restrict__ out) {
    const int BV = VEC ? B / 4 : B;
    const size_t n = (size_t)(C2 / F) * M * BV;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int bv = (int)(i % BV);
        const size_t cm = i / BV;
        const size_t m = cm % M;
        const size_t co = cm / M;
        const float* src = in + ((size_t)co * F * M + m) * ldb;
        float* dst = out + (co * M + m) * (size_t)B;
        if (VEC) {
            floatx4 sum = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(src + 4 * bv));
            for (int j = 1; j < F; ++j) {
                const floatx4 v = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(src + (size_t)j * M * ldb + 4 * bv));
#pragma unroll
                for (int e = 0; e < 4; ++e) sum[e] += v[e];
            }
            __builtin_nontemporal_store(sum, reinterpret_cast<floatx4*>(dst + 4 * bv));
        } else {
            float sum = src[bv];
            for (int j = 1; j < F; ++j) sum += src[(size_t)j * M * ldb + bv];
            dst[bv] = sum;
        }
    }
}

hipError_t launch_stage_sum_channels(const float* stage, int C2, int M, int B, int ldb, int F, float* out,
                                     hipStream_t st) {
    const bool vec = ((reinterpret_cast<uintptr_t>(stage) | reinterpret_cast<uintptr_t>(out)) & 15) == 0 &&
                     ldb % 4 == 0 && B % 4 == 0;
    const size_t n = (size_t)(C2 / F) * M * (vec ? B / 4 : B);
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 1u << 20);
    if (vec)
        hipLaunchKernelGGL(stage_sum_channels_kernel<true>, dim3(grid), dim3(256), 0, st, stage, C2, M, B, ldb, F, out);
    else
        hipLaunchKernelGGL(stage_sum_channels_kernel<false>, dim3(grid), dim3(256), 0, st, stage, C2, M, B, ldb, F, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Incoherent beam (Section 3): sum over stations of each station's Stokes
// parameters, integrated like a tied-array beam.  out [K][T'][C'].
// Generic form: one thread per output (c', t'); loops channel, time, station.
// ---------------------------------------------------------------------------
template <int XT, int K>
__global__ __launch_bounds__(256) void incoherent_kernel(const void* __restrict__ x, int S, int C, int T, int t_int,
                                                         int f_int, float* __restrict__ out) {
    const int T2 = T / t_int, C2 = C / f_int;
    const size_t n = (size_t)C2 * T2;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(i % C2);
        const int t2 = (int)(i / C2);
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int dc = 0; dc < f_int; ++dc)
            for (int dt = 0; dt < t_int; ++dt)
                for (int s = 0; s < S; ++s) {
                    const int c = c2 * f_int + dc, t = t2 * t_int + dt;
                    const floatx4 v = Sample<XT>::load(x, ((size_t)s * C + c) * T + t);
                    const float xx = v[0] * v[0] + v[1] * v[1];
                    const float yy = v[2] * v[2] + v[3] * v[3];
                    acc[0] += xx + yy;
                    if (K == 4) {
                        acc[1] += xx - yy;
                        acc[2] += 2.0f * (v[0] * v[2] + v[1] * v[3]);
                        acc[3] += 2.0f * (v[1] * v[2] - v[0] * v[3]);
                    }
                }
        for (int k = 0; k < K; ++k) out[((size_t)k * T2 + t2) * C2 + c2] = acc[k];
    }
}

// Fast form, HBM-bound: one wave per (channel group c', run of 64 P samples),
// P = 16 / sample bytes, so each lane reads one 16-byte vector of P
// consecutive samples per station and channel; a wave's load covers 1 KiB of
// one (station, channel) row.  Per sample the lane sums |X|^2, |Y|^2 and
// X conj(Y) over stations and the f_int channels, then forms I, Q, U, V.
// t_int is a power of two dividing 64 P, so a period never leaves a wave's
// run: t_int <= P periods lie in one lane, longer ones span G = t_int / P
// lanes and are summed with an xor butterfly.
template <int XT> struct Vec16;
template <> struct Vec16<XT_CI8> {
    static constexpr int P = 4;
    __device__ static inline void decode(const intx4 v, float (*f)[4]) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            f[p][0] = (float)((v[p] << 24) >> 24);
            f[p][1] = (float)((v[p] << 16) >> 24);
            f[p][2] = (float)((v[p] << 8) >> 24);
            f[p][3] = (float)(v[p] >> 24);
        }
    }
};
template <> struct Vec16<XT_CI16> {
    static constexpr int P = 2;
    __device__ static inline void decode(const intx4 v, float (*f)[4]) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            f[p][0] = (float)((v[2 * p] << 16) >> 16);
            f[p][1] = (float)(v[2 * p] >> 16);
            f[p][2] = (float)((v[2 * p + 1] << 16) >> 16);
            f[p][3] = (float)(v[2 * p + 1] >> 16);
        }
    }
};
template <> struct Vec16<XT_CF32> {
    static constexpr int P = 1;
    __device__ static inline void decode(const intx4 v, float (*f)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) f[0][q] = __int_as_float(v[q]);
    }
};

// per-sample sums: a[0] |X|^2, a[1] |Y|^2, a[2] Re X conj Y, a[3] Im X conj Y
__device__ __forceinline__ void power_acc(const float* v, float* a) {
    a[0] = __builtin_fmaf(v[0], v[0], __builtin_fmaf(v[1], v[1], a[0]));
    a[1] = __builtin_fmaf(v[2], v[2], __builtin_fmaf(v[3], v[3], a[1]));
    a[2] = __builtin_fmaf(v[0], v[2], __builtin_fmaf(v[1], v[3], a[2]));
    a[3] = __builtin_fmaf(v[1], v[2], __builtin_fmaf(-v[0], v[3], a[3]));
}

template <int XT, int K>
__global__ __launch_bounds__(256) void incoherent_wave_kernel(const void* __restrict__ x, int S, int C, int T,
                                                              int t_int, int f_int, int nrun, float* __restrict__ out) {
    constexpr int P = Vec16<XT>::P;
    constexpr int SB = Sample<XT>::bytes;
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int C2 = C / f_int, T2 = T / t_int;
    if (wave >= (long)C2 * nrun) return;   // whole waves only; the kernel has no barrier
    const int c2 = (int)(wave / nrun);
    const int t0 = (int)(wave - (long)c2 * nrun) * 64 * P + lane * P;
    const size_t sstride = (size_t)C * T;   // samples between stations
    float a[P][4];
#pragma unroll
    for (int p = 0; p < P; ++p) a[p][0] = a[p][1] = a[p][2] = a[p][3] = 0.f;
    for (int dc = 0; dc < f_int; ++dc) {
        const size_t row = (size_t)(c2 * f_int + dc) * T + t0;   // station 0
        if (t0 + P <= T) {
            const intx4* q = reinterpret_cast<const intx4*>(static_cast<const char*>(x) + row * SB);
            const size_t qs = sstride * SB / 16;
            int s = 0;
            for (; s + 4 <= S; s += 4) {
                intx4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(q + (size_t)(s + u) * qs);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    float f[P][4];
                    Vec16<XT>::decode(v[u], f);
#pragma unroll
                    for (int p = 0; p < P; ++p) power_acc(f[p], a[p]);
                }
            }
            for (; s < S; ++s) {
                float f[P][4];
                Vec16<XT>::decode(__builtin_nontemporal_load(q + (size_t)s * qs), f);
#pragma unroll
                for (int p = 0; p < P; ++p) power_acc(f[p], a[p]);
            }
        } else {
            // the row's ragged end: per-sample loads of the samples before T
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    if (t0 + p < T) {
                        const floatx4 v = Sample<XT>::load(x, row + (size_t)s * sstride + p);
                        const float f[4] = {v[0], v[1], v[2], v[3]};
                        power_acc(f, a[p]);
                    }
        }
    }
    // Stokes per sample, then the period sums
    float st[P][K];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        st[p][0] = a[p][0] + a[p][1];
        if (K == 4) {
            st[p][1] = a[p][0] - a[p][1];
            st[p][2] = 2.f * a[p][2];
            st[p][3] = 2.f * a[p][3];
        }
    }
    if (t_int <= P) {
        for (int j = 0; j * t_int < P; ++j) {
            if (t0 + j * t_int >= T) break;
            const int t2 = t0 / t_int + j;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                float v = 0.f;
#pragma unroll
                for (int p = 0; p < P; ++p)
                    if (p >= j * t_int && p < (j + 1) * t_int) v += st[p][k];
                out[((size_t)k * T2 + t2) * C2 + c2] = v;
            }
        }
    } else {
        const int G = t_int / P;
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] = 0.f;
#pragma unroll
            for (int p = 0; p < P; ++p) v[k] += st[p][k];
            for (int o = 1; o < G; o <<= 1) v[k] += __shfl_xor(v[k], o, 64);
        }
        if ((lane & (G - 1)) == 0 && t0 < T) {
            const int t2 = t0 / t_int;
#pragma unroll
            for (int k = 0; k < K; ++k) out[((size_t)k * T2 + t2) * C2 + c2] = v[k];
        }
    }
}

hipError_t launch_incoherent(const void* x, int xtype, int S, int C, int T, int product, int t_int, int f_int,
                             float* out, hipStream_t st) {
    const int P = xtype == XT_CI8 ? 4 : xtype == XT_CI16 ? 2 : 1;
    const bool pow2 = (t_int & (t_int - 1)) == 0 && t_int <= 64 * P;
    const long nrun = (T + 64L * P - 1) / (64L * P);
    const long waves = (long)(C / f_int) * nrun;
    // 16-byte rows: every (station, channel) row starts on a 16-byte boundary
    const bool vec = ((size_t)T * (16 / P)) % 16 == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    if (pow2 && vec && waves <= 0x7fffffffL * 4L) {
        const dim3 g((unsigned)((waves + 3) / 4)), b(256);
#define LBF_INCW(XTV)                                                                                            \
    if (product == PR_IQUV)                                                                                      \
        hipLaunchKernelGGL((incoherent_wave_kernel<XTV, 4>), g, b, 0, st, x, S, C, T, t_int, f_int, (int)nrun, out); \
    else hipLaunchKernelGGL((incoherent_wave_kernel<XTV, 1>), g, b, 0, st, x, S, C, T, t_int, f_int, (int)nrun, out);
        if (xtype == XT_CI8) { LBF_INCW(XT_CI8) }
        else if (xtype == XT_CI16) { LBF_INCW(XT_CI16) }
        else { LBF_INCW(XT_CF32) }
#undef LBF_INCW
        return hipGetLastError();
    }
    const size_t n = (size_t)(C / f_int) * (T / t_int);
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    dim3 g((unsigned)blocks), b(256);
#define LBF_INC(XTV)                                                                                        \
    if (product == PR_IQUV) hipLaunchKernelGGL((incoherent_kernel<XTV, 4>), g, b, 0, st, x, S, C, T, t_int, f_int, out); \
    else hipLaunchKernelGGL((incoherent_kernel<XTV, 1>), g, b, 0, st, x, S, C, T, t_int, f_int, out);
    if (xtype == XT_CI8) { LBF_INC(XT_CI8) }
    else if (xtype == XT_CI16) { LBF_INC(XT_CI16) }
    else { LBF_INC(XT_CF32) }
#undef LBF_INC
    return hipGetLastError();
}

}  // namespace lbf
