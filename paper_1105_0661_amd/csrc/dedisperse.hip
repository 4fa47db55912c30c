// dedisperse.hip -- channel-level dedispersion (Section 4.4 of Mol & Romein).
// Each polarisation's beam voltages are cut into blocks of N (8, 64, 512 or 4096) samples; a
// block is Fourier transformed, multiplied bin by bin with the channel's
// precomputed complex chirp weights, and transformed back with a 1/N factor.
//
// One work group per (channel, beam, block) keeps both polarisations of the
// block in LDS (16 N bytes plus padding: 66 KiB at N = 4096) and runs Stockham
// passes of radix R = 16 at N = 4096 (three per transform), 8 otherwise.  Pass
// s (span Ns = R^s) reads R elements N/R apart, turns them by the twiddles
// exp(-2 pi i (j mod Ns) r / (R Ns)), takes an R-point DFT in registers and
// writes the results Ns apart from (j / Ns) R Ns + j mod Ns; after the last
// pass the spectrum is in natural order, with no bit reversal.
// Every pass reads all its inputs, meets a barrier, then writes, so one
// buffer serves in place.  The backward transform is the forward one applied
// to conjugated data: the last forward pass multiplies by the chirp and
// conjugates, the last backward pass conjugates and scales.  The first pass
// reads HBM and the last writes HBM, each as 16-byte vectors (both
// polarisations of one sample) of consecutive samples.  Roofline: HBM (each
// voltage is read and written once; the passes in between stay on chip).
// The Stokes form (Section 4.5 after Section 4.4) keeps the last backward
// pass in LDS and forms Stokes parameters integrated over t_int consecutive
// samples from there, so the dedispersed voltages never reach HBM.
#include "fft_device.h"
#include "lbf_launch.h"

namespace lbf {

constexpr int kDdThreads = 256;

// 8-point DFT, forward sign, in place: 4-point DFTs of the even and the odd
// elements, then X[k] = E[k] + W8^k O[k], X[k + 4] = E[k] - W8^k O[k]
__device__ __forceinline__ void dft8(cfl* v) {
    cfl e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cfl o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const float h = 0.70710678118654752f;                  // sqrt(1/2)
    const cfl t1 = mk(h * (o1.x + o1.y), h * (o1.y - o1.x));   // W8^1 o1
    const cfl t2 = mk(o2.y, -o2.x);                            // W8^2 o2 = -i o2
    const cfl t3 = mk(h * (o3.y - o3.x), -h * (o3.x + o3.y));  // W8^3 o3
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + t1;
    v[5] = e1 - t1;
    v[2] = e2 + t2;
    v[6] = e2 - t2;
    v[3] = e3 + t3;
    v[7] = e3 - t3;
}

// LDS words of one polarisation's block, with lds_index's padding
template <int N>
__host__ __device__ constexpr int lds_words() { return N + N / 32; }

// One Stockham pass over both polarisations.  SRC 0: the block in HBM,
// 1: LDS.  DST 0: LDS, 1: LDS after the chirp product and conjugation (last
// forward pass), 2: HBM after conjugation and 1/N (last backward pass), 3:
// LDS after conjugation and 1/N (last backward pass of the Stokes form).
template <int N, int SRC, int DST>
__device__ __forceinline__ void dd_pass(int Ns, cfl* buf, const floatx4* __restrict__ yb, const cfl* __restrict__ hc,
                                        floatx4* __restrict__ ob) {
    constexpr int Q = N / 8;                                // butterflies per polarisation
    constexpr int JPT = (Q + kDdThreads - 1) / kDdThreads;  // per thread
    cfl v[JPT][2][8];
    cfl w[8];                                               // twiddles of the thread's butterfly j
#pragma unroll
    for (int m = 0; m < JPT; ++m) {
        const int j = threadIdx.x + kDdThreads * m;
        if (Q % kDdThreads != 0 && j >= Q) continue;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = j + r * Q;
            if (SRC == 0) {
                const floatx4 q = __builtin_nontemporal_load(yb + i);
                v[m][0][r] = mk(q[0], q[1]);
                v[m][1][r] = mk(q[2], q[3]);
            } else {
                v[m][0][r] = buf[lds_index(i)];
                v[m][1][r] = buf[lds_words<N>() + lds_index(i)];
            }
        }
        if (Ns > 1) {
            // w[r] = exp(-2 pi i k r / (8 Ns)), k = j mod Ns: w[1] from sincospif
            // (exact argument: 4 Ns is a power of two), the others as products;
            // the thread's later butterflies j + 256 m share k while Ns divides 256
            if (m == 0 || kDdThreads % Ns != 0) {
                float sn, cs;
                sincospif(-(float)(j % Ns) / (float)(4 * Ns), &sn, &cs);
                w[1] = mk(cs, sn);
                w[2] = cmul(w[1], w[1]);
                w[4] = cmul(w[2], w[2]);
                w[3] = cmul(w[1], w[2]);
                w[5] = cmul(w[1], w[4]);
                w[6] = cmul(w[2], w[4]);
                w[7] = cmul(w[3], w[4]);
            }
#pragma unroll
            for (int r = 1; r < 8; ++r) {
                v[m][0][r] = cmul(v[m][0][r], w[r]);
                v[m][1][r] = cmul(v[m][1][r], w[r]);
            }
        }
        dft8(v[m][0]);
        dft8(v[m][1]);
    }
    if (DST != 2) __syncthreads();                         // every read of this pass before any write
#pragma unroll
    for (int m = 0; m < JPT; ++m) {
        const int j = threadIdx.x + kDdThreads * m;
        if (Q % kDdThreads != 0 && j >= Q) continue;
        const int d0 = (j / Ns) * Ns * 8 + j % Ns;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int n = d0 + r * Ns;
            cfl a = v[m][0][r], b = v[m][1][r];
            if (DST == 1) {
                const cfl w = hc[n];
                a = cmul(a, w);
                b = cmul(b, w);
                a.y = -a.y;
                b.y = -b.y;
            }
            if (DST == 3) {
                constexpr float inv = 1.0f / (float)N;      // a power of two: exact
                a = mk(a.x * inv, -a.y * inv);
                b = mk(b.x * inv, -b.y * inv);
            }
            if (DST == 2) {
                constexpr float inv = 1.0f / (float)N;      // a power of two: exact
                floatx4 q;
                q[0] = a.x * inv;
                q[1] = -a.y * inv;
                q[2] = b.x * inv;
                q[3] = -b.y * inv;
                __builtin_nontemporal_store(q, ob + n);
            } else {
                buf[lds_index(n)] = a;
                buf[lds_words<N>() + lds_index(n)] = b;
            }
        }
    }
    if (DST != 2) __syncthreads();                         // the writes before the next pass reads
}

// A radix-16 Stockham pass over both polarisations (N = 4096: one butterfly
// per thread and polarisation); SRC and DST as in dd_pass.  Twiddles
// exp(-2 pi i k r / (16 Ns)): w[1] from sincospif, the others as products.
template <int N, int SRC, int DST>
__device__ __forceinline__ void dd_pass16(int Ns, cfl* buf, const floatx4* __restrict__ yb, const cfl* __restrict__ hc,
                                          floatx4* __restrict__ ob) {
    constexpr int Q = N / 16;
    static_assert(Q == kDdThreads, "one butterfly per thread and polarisation");
    cfl v[2][16];
    const int j = threadIdx.x;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = j + r * Q;
        if (SRC == 0) {
            const floatx4 q = __builtin_nontemporal_load(yb + i);
            v[0][r] = mk(q[0], q[1]);
            v[1][r] = mk(q[2], q[3]);
        } else {
            v[0][r] = buf[lds_index(i)];
            v[1][r] = buf[lds_words<N>() + lds_index(i)];
        }
    }
    if (Ns > 1) {
        float sn, cs;
        sincospif(-(float)(j % Ns) / (float)(8 * Ns), &sn, &cs);
        cfl w[16];
        w[1] = mk(cs, sn);
        w[2] = cmul(w[1], w[1]);
        w[4] = cmul(w[2], w[2]);
        w[8] = cmul(w[4], w[4]);
        w[3] = cmul(w[1], w[2]);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
#pragma unroll
        for (int r = 1; r < 16; ++r) {
            v[0][r] = cmul(v[0][r], w[r]);
            v[1][r] = cmul(v[1][r], w[r]);
        }
    }
    dft16(v[0]);
    dft16(v[1]);
    if (DST != 2) __syncthreads();                         // every read of this pass before any write
    const int d0 = (j / Ns) * Ns * 16 + j % Ns;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int n = d0 + r * Ns;
        cfl a = v[0][r], b = v[1][r];
        if (DST == 1) {
            const cfl w = hc[n];
            a = cmul(a, w);
            b = cmul(b, w);
            a.y = -a.y;
            b.y = -b.y;
        }
        if (DST == 3) {
            constexpr float inv = 1.0f / (float)N;          // a power of two: exact
            a = mk(a.x * inv, -a.y * inv);
            b = mk(b.x * inv, -b.y * inv);
        }
        if (DST == 2) {
            constexpr float inv = 1.0f / (float)N;          // a power of two: exact
            floatx4 q;
            q[0] = a.x * inv;
            q[1] = -a.y * inv;
            q[2] = b.x * inv;
            q[3] = -b.y * inv;
            __builtin_nontemporal_store(q, ob + n);
        } else {
            buf[lds_index(n)] = a;
            buf[lds_words<N>() + lds_index(n)] = b;
        }
    }
    if (DST != 2) __syncthreads();                         // the writes before the next pass reads
}

// Stokes parameters of the dedispersed block in LDS, integrated over t_int
// consecutive samples; s points at period 0 of this block in the (c, b) row
// of [T'][K].  With G = max(1, N / 256) samples per thread:
//  - t_int < G: thread j takes samples j + 256 g (consecutive lanes on
//    consecutive samples: conflict-free LDS reads, coalesced stores); a period
//    spans t_int lanes and meets in an xor butterfly;
//  - t_int >= G: thread j takes samples [G j, G j + G), read in an order
//    rotated by j so that the lanes spread over the LDS banks; a longer period
//    spans t_int / G lanes of a wave and meets in an xor butterfly
//    (t_int <= 64 G).
template <int K>
__device__ __forceinline__ void dd_put(float* __restrict__ s, int period, const float (&v)[4]) {
    if (K == 4) {
        floatx4 o;
        o[0] = v[0] + v[1];
        o[1] = v[0] - v[1];
        o[2] = 2.0f * v[2];
        o[3] = 2.0f * v[3];
        reinterpret_cast<floatx4*>(s)[period] = o;
    } else {
        s[period] = v[0] + v[1];
    }
}

__device__ __forceinline__ void dd_terms(const cfl x, const cfl y, float (&v)[4]) {
    v[0] += x.x * x.x + x.y * x.y;                          // |X|^2
    v[1] += y.x * y.x + y.y * y.y;                          // |Y|^2
    v[2] += x.x * y.x + x.y * y.y;                          // Re X conj(Y)
    v[3] += x.y * y.x - x.x * y.y;                          // Im X conj(Y)
}

template <int N, int K>
__device__ __forceinline__ void dd_stokes(const cfl* buf, float* __restrict__ s, int t_int) {
    constexpr int G = N >= kDdThreads ? N / kDdThreads : 1;
    const int j = threadIdx.x;
    if (t_int < G) {
        for (int g = 0; g < G; ++g) {
            const int n = j + kDdThreads * g;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            dd_terms(buf[lds_index(n)], buf[lds_words<N>() + lds_index(n)], v);
            for (int m = 1; m < t_int; m <<= 1)
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], m, kWave);
            if ((j & (t_int - 1)) == 0) dd_put<K>(s, n / t_int, v);
        }
        return;
    }
    const bool live = j * G < N;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int n = live ? j * G + ((g + j) & (G - 1)) : 0;
        dd_terms(buf[lds_index(n)], buf[lds_words<N>() + lds_index(n)], v);
    }
    const int L = t_int / G;                                // lanes per period (a power of two <= 64)
    for (int m = 1; m < L; m <<= 1)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], m, kWave);
    if (live && (j & (L - 1)) == 0) dd_put<K>(s, j * G / t_int, v);
}

template <int N>
__global__ __launch_bounds__(kDdThreads) void dedisperse_kernel(const floatx4* __restrict__ y, const cfl* __restrict__ chirp,
                                                                floatx4* __restrict__ out, int B, int T) {
    __shared__ __attribute__((aligned(16))) cfl buf[2 * lds_words<N>()];
    const int nb = T / N;
    // consecutive (beam, block) groups of a channel on one XCD: its chirp
    // is then fetched into that XCD's L2 once rather than into every L2
    const long wg = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const long cb = wg / nb;                                // c B + b
    const int blk = (int)(wg - cb * nb);
    const int c = (int)(cb / B);
    const size_t base = (size_t)cb * T + (size_t)blk * N;   // in samples (16 bytes: both polarisations)
    const floatx4* yb = y + base;
    floatx4* ob = out + base;
    const cfl* hc = chirp + (size_t)c * N;
    if constexpr (N == 4096) {
        // three radix-16 passes per transform; the third forward pass applies
        // the chirp and conjugates, the third backward pass stores
        dd_pass16<N, 0, 0>(1, buf, yb, hc, ob);
        dd_pass16<N, 1, 0>(16, buf, yb, hc, ob);
        dd_pass16<N, 1, 1>(256, buf, yb, hc, ob);
        dd_pass16<N, 1, 0>(1, buf, yb, hc, ob);
        dd_pass16<N, 1, 0>(16, buf, yb, hc, ob);
        dd_pass16<N, 1, 2>(256, buf, yb, hc, ob);
        return;
    }
    constexpr int P = N == 8 ? 1 : N == 64 ? 2 : 3;
    // forward transform; its last pass applies the chirp and conjugates
    int Ns = 1;
    if (P == 1) {
        dd_pass<N, 0, 1>(Ns, buf, yb, hc, ob);
    } else {
        dd_pass<N, 0, 0>(Ns, buf, yb, hc, ob);
        Ns *= 8;
        for (int s = 1; s < P - 1; ++s, Ns *= 8) dd_pass<N, 1, 0>(Ns, buf, yb, hc, ob);
        dd_pass<N, 1, 1>(Ns, buf, yb, hc, ob);
    }
    // backward transform of the conjugated product; its last pass conjugates,
    // scales and stores
    Ns = 1;
    for (int s = 0; s < P - 1; ++s, Ns *= 8) dd_pass<N, 1, 0>(Ns, buf, yb, hc, ob);
    dd_pass<N, 1, 2>(Ns, buf, yb, hc, ob);
}

// Dedispersion then Stokes and integration: s [C][B][T/t_int][K]
template <int N, int K>
__global__ __launch_bounds__(kDdThreads) void dedisperse_stokes_kernel(const floatx4* __restrict__ y,
                                                                       const cfl* __restrict__ chirp,
                                                                       float* __restrict__ s, int B, int T, int t_int) {
    __shared__ __attribute__((aligned(16))) cfl buf[2 * lds_words<N>()];
    const int nb = T / N;
    // consecutive (beam, block) groups of a channel on one XCD: its chirp
    // is then fetched into that XCD's L2 once rather than into every L2
    const long wg = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const long cb = wg / nb;                                // c B + b
    const int blk = (int)(wg - cb * nb);
    const int c = (int)(cb / B);
    const floatx4* yb = y + (size_t)cb * T + (size_t)blk * N;
    const cfl* hc = chirp + (size_t)c * N;
    float* sb = s + ((size_t)cb * (T / t_int) + (size_t)blk * (N / t_int)) * K;
    if constexpr (N == 4096) {
        dd_pass16<N, 0, 0>(1, buf, yb, hc, nullptr);
        dd_pass16<N, 1, 0>(16, buf, yb, hc, nullptr);
        dd_pass16<N, 1, 1>(256, buf, yb, hc, nullptr);
        dd_pass16<N, 1, 0>(1, buf, yb, hc, nullptr);
        dd_pass16<N, 1, 0>(16, buf, yb, hc, nullptr);
        dd_pass16<N, 1, 3>(256, buf, yb, hc, nullptr);
    } else {
        constexpr int P = N == 8 ? 1 : N == 64 ? 2 : 3;
        int Ns = 1;
        if (P == 1) {
            dd_pass<N, 0, 1>(Ns, buf, yb, hc, nullptr);
        } else {
            dd_pass<N, 0, 0>(Ns, buf, yb, hc, nullptr);
            Ns *= 8;
            for (int p = 1; p < P - 1; ++p, Ns *= 8) dd_pass<N, 1, 0>(Ns, buf, yb, hc, nullptr);
            dd_pass<N, 1, 1>(Ns, buf, yb, hc, nullptr);
        }
        Ns = 1;
        for (int p = 0; p < P - 1; ++p, Ns *= 8) dd_pass<N, 1, 0>(Ns, buf, yb, hc, nullptr);
        dd_pass<N, 1, 3>(Ns, buf, yb, hc, nullptr);
    }
    dd_stokes<N, K>(buf, sb, t_int);                        // the last pass ended with a barrier
}

template <int N>
static void launch_dd_stokes(dim3 g, const floatx4* yv, const cfl* hv, float* s, int B, int T, int product, int t_int,
                             hipStream_t st) {
    if (product == PR_IQUV)
        hipLaunchKernelGGL((dedisperse_stokes_kernel<N, 4>), g, dim3(kDdThreads), 0, st, yv, hv, s, B, T, t_int);
    else
        hipLaunchKernelGGL((dedisperse_stokes_kernel<N, 1>), g, dim3(kDdThreads), 0, st, yv, hv, s, B, T, t_int);
}

hipError_t launch_dedisperse_stokes(const void* y, int C, int B, int T, int n_fft, const void* chirp, int product,
                                    int t_int, float* s, hipStream_t st) {
    const dim3 g((unsigned)((size_t)C * B * (T / n_fft)));
    const floatx4* yv = static_cast<const floatx4*>(y);
    const cfl* hv = static_cast<const cfl*>(chirp);
    switch (n_fft) {
        case 8: launch_dd_stokes<8>(g, yv, hv, s, B, T, product, t_int, st); break;
        case 64: launch_dd_stokes<64>(g, yv, hv, s, B, T, product, t_int, st); break;
        case 512: launch_dd_stokes<512>(g, yv, hv, s, B, T, product, t_int, st); break;
        case 4096: launch_dd_stokes<4096>(g, yv, hv, s, B, T, product, t_int, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dedisperse(const void* y, int C, int B, int T, int n_fft, const void* chirp, void* out,
                             hipStream_t st) {
    const unsigned groups = (unsigned)((size_t)C * B * (T / n_fft));
    const dim3 g(groups), b(kDdThreads);
    const floatx4* yv = static_cast<const floatx4*>(y);
    const cfl* hv = static_cast<const cfl*>(chirp);
    floatx4* ov = static_cast<floatx4*>(out);
    switch (n_fft) {
        case 8: hipLaunchKernelGGL(dedisperse_kernel<8>, g, b, 0, st, yv, hv, ov, B, T); break;
        case 64: hipLaunchKernelGGL(dedisperse_kernel<64>, g, b, 0, st, yv, hv, ov, B, T); break;
        case 512: hipLaunchKernelGGL(dedisperse_kernel<512>, g, b, 0, st, yv, hv, ov, B, T); break;
        case 4096: hipLaunchKernelGGL(dedisperse_kernel<4096>, g, b, 0, st, yv, hv, ov, B, T); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbf
