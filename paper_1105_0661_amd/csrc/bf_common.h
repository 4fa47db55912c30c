// bf_common.h -- pieces shared by the contraction kernels: operand loads and
// conversions, MFMA wrappers, weight staging and the Stokes epilogue.
//
// The contraction (Section 4.3 of Mol & Romein: each tied-array beam is a
// weighted complex sum of the station signals) runs per channel as a real
// GEMM on the matrix cores: time samples on the MFMA rows, beams on the
// columns, (station, re/im) on the reduction axis.  With the weight operand
// B = (w_re, w_im) the complex product splits into
//     Re y = A_r . B,  A_r = (x_re, -x_im);     Im y = A_i . B,  A_i = (x_im, x_re)
// so each lane ends up holding Re and Im of both polarisations of the same
// (sample, beam): the Stokes epilogue (Section 4.5) and the integration over
// up to 16 samples (Section 5.1) need no data exchange between lanes.
#pragma once
#include "bf_addr.h"
#include "lbf_device.h"
#include "lbf_launch.h"
#include "tile_table.h"

#define LBF_INLINE __device__ __forceinline__

namespace lbf {

constexpr int kBeamGroup = 128;                 // beams per work item (4 MFMA tiles)
constexpr int kBeamTiles = kBeamGroup / kTile;
constexpr int kStationChunk = 64;               // stations whose weights sit in LDS at once
constexpr int kWavesPerGroup = 4;
constexpr int kThreads = kWave * kWavesPerGroup;
constexpr int kThreadsH = 512;                 // fast workers: 8 waves, two per SIMD
constexpr int kWRow = kStationChunk + 4;        // LDS row of packed f16/bf16 weights (words)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// raw sample loads: one time sample of one station, both polarisations
// ---------------------------------------------------------------------------
template <int XT> struct Raw;
template <> struct Raw<XT_CI8> {
    typedef int type;
    LBF_INLINE static type load(const void* p, size_t i) { return reinterpret_cast<const int*>(p)[i]; }
    LBF_INLINE static floatx4 cvt(type v) {
        floatx4 r;
        r[0] = (float)(int8_t)(v & 0xff);
        r[1] = (float)(int8_t)((v >> 8) & 0xff);
        r[2] = (float)(int8_t)((v >> 16) & 0xff);
        r[3] = (float)(int8_t)((v >> 24) & 0xff);
        return r;
    }
    LBF_INLINE static type zero() { return 0; }
    // the re (h = 0) or im (h = 1) part of X and of Y; sh = 8 h, kept opaque
    // by the caller so that it stays one shift per value rather than a select
    LBF_INLINE static void half(type v, uint32_t sh, float& x, float& y) {
        x = (float)(int8_t)((uint32_t)v >> sh);
        y = (float)(int8_t)((uint32_t)v >> (sh + 16u));
    }
};
template <> struct Raw<XT_CI16> {
    typedef shortx4 type;
    LBF_INLINE static type load(const void* p, size_t i) { return reinterpret_cast<const shortx4*>(p)[i]; }
    LBF_INLINE static floatx4 cvt(type v) {
        floatx4 r;
        r[0] = (float)v[0];
        r[1] = (float)v[1];
        r[2] = (float)v[2];
        r[3] = (float)v[3];
        return r;
    }
    LBF_INLINE static type zero() { type z = {0, 0, 0, 0}; return z; }
    // as Raw<XT_CI8>::half, sh = 16 h
    LBF_INLINE static void half(type v, uint32_t sh, float& x, float& y) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 w = __builtin_bit_cast(u32x2, v);
        x = (float)(int16_t)(w[0] >> sh);
        y = (float)(int16_t)(w[1] >> sh);
    }
};
template <> struct Raw<XT_CF32> {
    typedef floatx4 type;
    LBF_INLINE static type load(const void* p, size_t i) { return reinterpret_cast<const floatx4*>(p)[i]; }
    LBF_INLINE static floatx4 cvt(type v) { return v; }
    LBF_INLINE static type zero() { type z = {0.f, 0.f, 0.f, 0.f}; return z; }
    LBF_INLINE static void half(type v, uint32_t sh, float& x, float& y) {
        x = sh ? v[1] : v[0];
        y = sh ? v[3] : v[2];
    }
};

// ---------------------------------------------------------------------------
// MFMA wrappers
// ---------------------------------------------------------------------------
template <int CT> struct MfmaH;
template <> struct MfmaH<CT_F16> {
    typedef halfx8 vec;
    LBF_INLINE static floatx16 mfma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct MfmaH<CT_BF16> {
    typedef bf16x8 vec;
    LBF_INLINE static floatx16 mfma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

LBF_INLINE floatx16 mfma_f32(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

LBF_INLINE floatx16 zero16() {
    floatx16 z;
#pragma unroll
    for (int k = 0; k < 16; ++k) z[k] = 0.f;
    return z;
}

// ---------------------------------------------------------------------------
// A operands of one station sample (X, Y) in 16-bit types, as packed words:
//   xr = (x_re, -x_im), xi = (x_im, x_re), likewise for Y.
// ---------------------------------------------------------------------------
struct APair {
    uint32_t xr, xi, yr, yi;
};

LBF_INLINE uint32_t neg_hi(uint32_t w) { return w ^ 0x80000000u; }
LBF_INLINE uint32_t swap16(uint32_t w) { return __builtin_amdgcn_alignbit(w, w, 16); }

template <int XT, int CT> struct Conv;

// complex int8 -> f16: bytes biased by 128 become the low mantissa byte of
// 1024 + b + 128 (exponent 0x64), then 1152 is subtracted (exact).
template <> struct Conv<XT_CI8, CT_F16> {
    LBF_INLINE static APair frag(int v) {
        const uint32_t u = (uint32_t)v ^ 0x80808080u;
        const uint32_t px = __builtin_amdgcn_perm(u, 0x64646464u, 0x00050004u);
        const uint32_t py = __builtin_amdgcn_perm(u, 0x64646464u, 0x00070006u);
        halfx2 hx = __builtin_bit_cast(halfx2, px), hy = __builtin_bit_cast(halfx2, py);
        const halfx2 bias = {(_Float16)-1152.0f, (_Float16)-1152.0f};
        hx = hx + bias;
        hy = hy + bias;
        const uint32_t fx = __builtin_bit_cast(uint32_t, hx), fy = __builtin_bit_cast(uint32_t, hy);
        APair a;
        a.xr = neg_hi(fx);
        a.xi = swap16(fx);
        a.yr = neg_hi(fy);
        a.yi = swap16(fy);
        return a;
    }
};

// complex int16 -> f16 (exact for |x| <= 2048, round-to-nearest-even beyond)
template <> struct Conv<XT_CI16, CT_F16> {
    LBF_INLINE static APair frag(shortx4 v) {
        halfx2 hx = {(_Float16)v[0], (_Float16)v[1]};
        halfx2 hy = {(_Float16)v[2], (_Float16)v[3]};
        const uint32_t fx = __builtin_bit_cast(uint32_t, hx), fy = __builtin_bit_cast(uint32_t, hy);
        APair a;
        a.xr = neg_hi(fx);
        a.xi = swap16(fx);
        a.yr = neg_hi(fy);
        a.yi = swap16(fy);
        return a;
    }
};

// Two floats to a word of two bf16 (lo first), rounded to nearest even by
// the hardware's packed conversion (v_cvt_pk_bf16_f32): one instruction per
// pair.  int8 values are exact in bf16, so their float bits can simply be
// truncated (pack_bf16_exact).
LBF_INLINE uint32_t pack_bf16(float lo, float hi) {
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    const bf16x2_t r = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, r);
}
LBF_INLINE uint32_t pack_bf16_exact(float lo, float hi) {
    return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
}

template <int XT> struct Conv<XT, CT_BF16> {
    LBF_INLINE static APair frag(typename Raw<XT>::type v) {
        const floatx4 f = Raw<XT>::cvt(v);
        uint32_t fx, fy;
        if (XT == XT_CI8) {
            fx = pack_bf16_exact(f[0], f[1]);
            fy = pack_bf16_exact(f[2], f[3]);
        } else {
            fx = pack_bf16(f[0], f[1]);
            fy = pack_bf16(f[2], f[3]);
        }
        APair a;
        a.xr = neg_hi(fx);
        a.xi = swap16(fx);
        a.yr = neg_hi(fy);
        a.yi = swap16(fy);
        return a;
    }
};

template <> struct Conv<XT_CF32, CT_F16> {
    LBF_INLINE static APair frag(floatx4 f) {
        halfx2 hx = {(_Float16)f[0], (_Float16)f[1]};
        halfx2 hy = {(_Float16)f[2], (_Float16)f[3]};
        const uint32_t fx = __builtin_bit_cast(uint32_t, hx), fy = __builtin_bit_cast(uint32_t, hy);
        APair a;
        a.xr = neg_hi(fx);
        a.xi = swap16(fx);
        a.yr = neg_hi(fy);
        a.yi = swap16(fy);
        return a;
    }
};

// Plain 16-bit operand words of one station sample: fx = (x_re, x_im),
// fy = (y_re, y_im) -- the fast workers put the re/im mixing of the complex
// product into two weight variants instead.
template <int XT, int CT> struct Conv2;

// complex int8 -> f16, exact: the byte-bias trick of Conv<XT_CI8, CT_F16>
template <> struct Conv2<XT_CI8, CT_F16> {
    LBF_INLINE static void xy(int v, uint32_t& fx, uint32_t& fy) {
        const uint32_t u = (uint32_t)v ^ 0x80808080u;
        halfx2 hx = __builtin_bit_cast(halfx2, __builtin_amdgcn_perm(u, 0x64646464u, 0x00050004u));
        halfx2 hy = __builtin_bit_cast(halfx2, __builtin_amdgcn_perm(u, 0x64646464u, 0x00070006u));
        const halfx2 bias = {(_Float16)-1152.0f, (_Float16)-1152.0f};
        fx = __builtin_bit_cast(uint32_t, hx + bias);
        fy = __builtin_bit_cast(uint32_t, hy + bias);
    }
};

// complex int16 -> f16 (exact for |x| <= 2048, round-to-nearest-even beyond).
// The two halves of a word convert in place: the second conversion writes
// the high half and keeps the low one (SDWA), so no packing instruction
// follows -- two vector instructions per complex value instead of three.
LBF_INLINE uint32_t cvt_i16x2_f16x2(uint32_t w) {
    uint32_t r;
    __asm__("v_cvt_f16_i16_sdwa %0, %1 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:WORD_0\n\t"
            "v_cvt_f16_i16_sdwa %0, %1 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1"
            : "=&v"(r)
            : "v"(w));
    return r;
}
template <> struct Conv2<XT_CI16, CT_F16> {
    LBF_INLINE static void xy(shortx4 v, uint32_t& fx, uint32_t& fy) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 w = __builtin_bit_cast(u32x2, v);
        fx = cvt_i16x2_f16x2(w[0]);
        fy = cvt_i16x2_f16x2(w[1]);
    }
};

// -> bf16: int8 exactly (float bits truncated), int16 round-to-nearest-even
template <int XT> struct Conv2<XT, CT_BF16> {
    LBF_INLINE static void xy(typename Raw<XT>::type v, uint32_t& fx, uint32_t& fy) {
        const floatx4 f = Raw<XT>::cvt(v);
        if (XT == XT_CI8) {
            fx = pack_bf16_exact(f[0], f[1]);
            fy = pack_bf16_exact(f[2], f[3]);
        } else {
            fx = pack_bf16(f[0], f[1]);
            fy = pack_bf16(f[2], f[3]);
        }
    }
};

// ---------------------------------------------------------------------------
// weight staging into LDS
// ---------------------------------------------------------------------------

// FP32 weights: wl[sl][ri][b] floats for stations [s0, s0+64) of beams
// [b0, b0+128) of channel c; zero outside [0,S) x [0,B).
LBF_INLINE void stage_weights_f32(float* wl, const BlockDesc& d, int c, int b0, int s0) {
    const float2* w = reinterpret_cast<const float2*>(d.w);
    for (int i = threadIdx.x; i < kStationChunk * kBeamGroup; i += blockDim.x) {
        const int sl = i % kStationChunk, bl = i / kStationChunk;
        const int s = s0 + sl, b = b0 + bl;
        float2 v = make_float2(0.f, 0.f);
        if (s < d.S && b < d.B) v = w[((size_t)c * d.B + b) * d.S + s];
        wl[(sl * 2 + 0) * kBeamGroup + bl] = v.x;
        wl[(sl * 2 + 1) * kBeamGroup + bl] = v.y;
    }
}

// FP16/BF16 weights: wh[b][sl] packed complex (32 bits), row stride kWRow
// words (64 stations + a 16-byte pad against LDS bank conflicts).
LBF_INLINE void stage_weights_h(uint32_t* wh, const BlockDesc& d, int c, int b0, int s0) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(d.w);
    for (int i = threadIdx.x; i < kStationChunk * kBeamGroup; i += blockDim.x) {
        const int sl = i % kStationChunk, bl = i / kStationChunk;
        const int s = s0 + sl, b = b0 + bl;
        uint32_t v = 0u;
        if (s < d.S && b < d.B) v = w[((size_t)c * d.B + b) * d.S + s];
        wh[bl * kWRow + sl] = v;
    }
}

// Weight descriptor of channel c: the channel's [B][S] block; beams >= B and
// stations past the block read as zero.
LBF_INLINE __amdgpu_buffer_rsrc_t weight_rsrc(const BlockDesc& d, int c, int bytes) {
    const uint64_t base = reinterpret_cast<uint64_t>(d.w) + weight_base(d, c, bytes);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    const uint32_t nrec = __builtin_amdgcn_readfirstlane(weight_range(d, bytes));
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, (int)nrec,
                                             0x00020000);
}

// ---------------------------------------------------------------------------
// epilogue: voltages, or Stokes + integration + beam-major store
// ---------------------------------------------------------------------------
struct EpiCtx {
    float* out;
    int B, T, C2, T2, K;
    int c;          // channel (voltages)
    int g;          // output channel c' (Stokes)
    int first;      // first channel of the f_int group: store, else accumulate
    int t_int;
    size_t sb, sk, st, sc;   // Stokes element strides of beam, parameter, t' and c'
};

LBF_INLINE void store_or_add(float* p, float v, int first) {
    if (first) *p = v;
    else *p = *p + v;
}

// Stokes sums over samples [k0, k0+n) of this lane half of one tile
// (acc = {Xre, Xim, Yre, Yim}).  IQUV: sums of |X|^2, |Y|^2, Re and Im of
// X conj(Y); Stokes I: one sum of |X|^2 + |Y|^2.
template <int PR, int N>
LBF_INLINE void stokes_sums(const floatx16 (&acc)[4], int k0, float (&s)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = 0.f;
#pragma unroll
    for (int k = k0; k < k0 + N; ++k) {
        const float xr = acc[0][k], xi = acc[1][k], yr = acc[2][k], yi = acc[3][k];
        if (PR == PR_I) {
            s[0] = __builtin_fmaf(xr, xr, s[0]);
            s[0] = __builtin_fmaf(xi, xi, s[0]);
            s[0] = __builtin_fmaf(yr, yr, s[0]);
            s[0] = __builtin_fmaf(yi, yi, s[0]);
        } else {
            s[0] = __builtin_fmaf(xi, xi, __builtin_fmaf(xr, xr, s[0]));
            s[1] = __builtin_fmaf(yi, yi, __builtin_fmaf(yr, yr, s[1]));
            s[2] = __builtin_fmaf(xi, yi, __builtin_fmaf(xr, yr, s[2]));
            s[3] = __builtin_fmaf(-xr, yi, __builtin_fmaf(xi, yr, s[3]));
        }
    }
}

// add sample k of a tile to the Stokes sums s (as stokes_sums, one sample)
template <int PR>
LBF_INLINE void stokes_add(const floatx16 (&acc)[4], int k, float (&s)[4]) {
    const float xr = acc[0][k], xi = acc[1][k], yr = acc[2][k], yi = acc[3][k];
    if (PR == PR_I) {
        s[0] = __builtin_fmaf(xr, xr, s[0]);
        s[0] = __builtin_fmaf(xi, xi, s[0]);
        s[0] = __builtin_fmaf(yr, yr, s[0]);
        s[0] = __builtin_fmaf(yi, yi, s[0]);
    } else {
        s[0] = __builtin_fmaf(xi, xi, __builtin_fmaf(xr, xr, s[0]));
        s[1] = __builtin_fmaf(yi, yi, __builtin_fmaf(yr, yr, s[1]));
        s[2] = __builtin_fmaf(xi, yi, __builtin_fmaf(xr, yr, s[2]));
        s[3] = __builtin_fmaf(-xr, yi, __builtin_fmaf(xi, yr, s[3]));
    }
}

// (I, Q, U, V) from the sums
template <int PR>
LBF_INLINE void stokes_from_sums(const float (&s)[4], float (&o)[4]) {
    if (PR == PR_I) {
        o[0] = s[0];
    } else {
        o[0] = s[0] + s[1];
        o[1] = s[0] - s[1];
        o[2] = 2.0f * s[2];
        o[3] = 2.0f * s[3];
    }
}

template <int PR, int TI, bool PLAIN = false>
LBF_INLINE void stokes_store_ti(const floatx16 (&acc)[4], const EpiCtx& e, int beam, int t0, int h) {
    constexpr int K = PR == PR_IQUV ? 4 : 1;
    constexpr int NOUT = 16 / TI;
    const int tq0 = (t0 + 16 * h) / TI;
    const bool bok = beam < e.B;
    float* base = e.out + (size_t)beam * e.sb + (size_t)e.g * e.sc;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        float s[4], v[4];
        stokes_sums<PR, TI>(acc, o * TI, s);
        stokes_from_sums<PR>(s, v);
        const int tq = tq0 + o;
        if (bok && tq < e.T2) {
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                float* p = base + (size_t)kk * e.sk + (size_t)tq * e.st;
                if (PLAIN) *p = v[kk];
                else store_or_add(p, v[kk], e.first);
            }
        }
    }
}

// epilogue of all beam tiles of one 32-sample tile for t_int < 32 (and voltages)
template <int PR, int TI, bool PLAIN = false>
LBF_INLINE void epilogue_tiles_ti(const floatx16 (&acc)[kBeamTiles][4], const EpiCtx& e, int b0, int r, int t0,
                                  int h) {
#pragma unroll
    for (int a = 0; a < kBeamTiles; ++a) {
        stokes_store_ti<PR, TI, PLAIN>(acc[a], e, b0 + a * kTile + r, t0, h);
        __builtin_amdgcn_sched_barrier(0);   // one beam tile's temporaries at a time
    }
}

template <int PR>
LBF_INLINE void epilogue_tiles(const floatx16 (&acc)[kBeamTiles][4], const EpiCtx& e, int b0, int r, int t0,
                               int h);

// epilogue of one 32x32 tile for t_int < 32 (and voltages)
template <int PR>
LBF_INLINE void epilogue_tile(const floatx16 (&acc)[4], const EpiCtx& e, int beam, int t0, int h) {
    if (PR == PR_VOLT) {
        if (beam >= e.B) return;
        floatx4* o = reinterpret_cast<floatx4*>(e.out) + ((size_t)e.c * e.B + beam) * e.T;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int t = t0 + 16 * h + k;
            if (t < e.T) {
                floatx4 v;
                v[0] = acc[0][k];
                v[1] = acc[1][k];
                v[2] = acc[2][k];
                v[3] = acc[3][k];
                o[t] = v;
            }
        }
    } else {
        switch (e.t_int) {
            case 1: stokes_store_ti<PR, 1>(acc, e, beam, t0, h); break;
            case 2: stokes_store_ti<PR, 2>(acc, e, beam, t0, h); break;
            case 4: stokes_store_ti<PR, 4>(acc, e, beam, t0, h); break;
            case 8: stokes_store_ti<PR, 8>(acc, e, beam, t0, h); break;
            default: stokes_store_ti<PR, 16>(acc, e, beam, t0, h); break;
        }
    }
}

// Branch-free stores of the fast workers.  The descriptor covers one channel
// of the output; a lane with nothing to store (beam >= B, sample past the
// end, no tile) uses the offset kNoStore, past the end of every output
// descriptor, which the hardware drops, so the epilogue has no control flow
// and interleaves freely with the MFMAs of the next tile.  Per-channel outputs
// are below 2^31 bytes (fast_path).

// off if ok, else kNoStore, as a lane select the compiler keeps (a plain ?:
// is turned into a branch around the store)
LBF_INLINE uint32_t store_off(bool ok, uint32_t off) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(ok);
    uint32_t r;
    __asm__("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(kNoStore), "v"(off), "s"(m));
    return r;
}

// output descriptor of channel c of the item's block (index c - c0)
LBF_INLINE __amdgpu_buffer_rsrc_t channel_rsrc(const BlockDesc& d, int c, uint32_t bytes_per_channel) {
    const uint64_t base = reinterpret_cast<uint64_t>(d.out) + out_base(d, c, bytes_per_channel);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0,
                                             (int)bytes_per_channel, 0x00020000);
}

// The Stokes parameters of one (t', beam) into the channel-major s[t'][b][k]
// of its channel (rows of ld floats per t'): one 16-byte store for IQUV.
template <int PR>
LBF_INLINE void stokes_store_row(const float (&v)[4], __amdgpu_buffer_rsrc_t rs, int ld, int tq, int beam, bool ok) {
    if (PR == PR_IQUV) {
        const uint32_t off = store_off(ok, stokes_off(tq, ld, beam, 4));
        floatx4 w;
        w[0] = v[0];
        w[1] = v[1];
        w[2] = v[2];
        w[3] = v[3];
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, w), rs, (int)off, 0, 0);
    } else {
        const uint32_t off = store_off(ok, stokes_off(tq, ld, beam, 1));
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[0]), rs, (int)off, 0, 0);
    }
}

// Stokes of one 32x32 tile into channel-major s[t'][b][k] of its channel
template <int PR, int TI>
LBF_INLINE void stokes_store_cm(const floatx16 (&acc)[4], __amdgpu_buffer_rsrc_t rs, int ld, int T2, int beam, int t0,
                                int h, bool ok) {
    constexpr int NOUT = 16 / TI;
    const int tq0 = (t0 + 16 * h) / TI;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        float sm[4], v[4];
        stokes_sums<PR, TI>(acc, o * TI, sm);
        stokes_from_sums<PR>(sm, v);
        const int tq = tq0 + o;
        stokes_store_row<PR>(v, rs, ld, tq, beam, ok && tq < T2);
    }
}

// complex voltages of one tile into y[b][t][p] of its channel
LBF_INLINE void volt_store_cm(const floatx16 (&acc)[4], __amdgpu_buffer_rsrc_t rs, int T, int beam, int t0, int h,
                              bool ok) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int t = t0 + 16 * h + k;
        const uint32_t off = store_off(ok && t < T, volt_off(beam, T, t));
        floatx4 v;
        v[0] = acc[0][k];
        v[1] = acc[1][k];
        v[2] = acc[2][k];
        v[3] = acc[3][k];
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, (int)off, 0, 0);
    }
}

template <int PR>
LBF_INLINE void epilogue_tiles(const floatx16 (&acc)[kBeamTiles][4], const EpiCtx& e, int b0, int r, int t0,
                               int h) {
    if (PR == PR_VOLT) {
#pragma unroll
        for (int a = 0; a < kBeamTiles; ++a) epilogue_tile<PR>(acc[a], e, b0 + a * kTile + r, t0, h);
        return;
    }
    switch (e.t_int) {
        case 1: epilogue_tiles_ti<PR, 1>(acc, e, b0, r, t0, h); break;
        case 2: epilogue_tiles_ti<PR, 2>(acc, e, b0, r, t0, h); break;
        case 4: epilogue_tiles_ti<PR, 4>(acc, e, b0, r, t0, h); break;
        case 8: epilogue_tiles_ti<PR, 8>(acc, e, b0, r, t0, h); break;
        default: epilogue_tiles_ti<PR, 16>(acc, e, b0, r, t0, h); break;
    }
}

// t_int >= 32: add this tile's 16-sample sums into running group sums
template <int PR>
LBF_INLINE void accumulate_tile_sums(const floatx16 (&acc)[4], float (&gs)[4]) {
    float s[4];
    stokes_sums<PR, 16>(acc, 0, s);
#pragma unroll
    for (int q = 0; q < 4; ++q) gs[q] += s[q];
}

// t_int >= 32: combine the two lane halves (samples 0-15 and 16-31 of each
// tile) and store the group's Stokes parameters
template <int PR>
LBF_INLINE void store_group_sums(float (&gs)[4], const EpiCtx& e, int beam, int tq, int h) {
    constexpr int K = PR == PR_IQUV ? 4 : 1;
    float tot[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float other = __shfl_xor(gs[q], 32, kWave);
        tot[q] = h == 0 ? gs[q] + other : other + gs[q];
    }
    float v[4];
    stokes_from_sums<PR>(tot, v);
    if (h != 0 || beam >= e.B || tq >= e.T2) return;
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
        store_or_add(e.out + (size_t)beam * e.sb + (size_t)kk * e.sk + (size_t)tq * e.st + (size_t)e.g * e.sc, v[kk],
                     e.first);
}

LBF_INLINE EpiCtx make_epi(const BlockDesc& d, int PR_, int g) {
    EpiCtx e;
    e.out = reinterpret_cast<float*>(d.out);
    e.B = d.B;
    e.T = d.T;
    e.K = PR_ == PR_IQUV ? 4 : 1;
    e.t_int = PR_ == PR_VOLT ? 1 : d.t_int;
    e.C2 = d.C / (PR_ == PR_VOLT ? 1 : d.f_int);
    e.T2 = d.T / e.t_int;
    e.g = g;
    e.c = 0;
    e.first = 1;
    if (d.order == 0) {          // [B][K][T'][C']
        e.sc = 1;
        e.st = (size_t)e.C2;
        e.sk = (size_t)e.T2 * e.C2;
        e.sb = (size_t)e.K * e.T2 * e.C2;
    } else {                     // [C'][T'][B][K], rows of ld_row floats per t'
        e.sk = 1;
        e.sb = (size_t)e.K;
        e.st = (size_t)d.ld_row;
        e.sc = (size_t)e.T2 * d.ld_row;
    }
    return e;
}

// Tiles of one wave: groups of tiles_per_group consecutive 32-sample tiles
// (one group per t_int >= 32 integration), groups dealt round-robin to waves.
struct WaveTiles {
    int wave, tpg, ntw;
    LBF_INLINE int tile(int k) const { return (wave + kWavesPerGroup * (k / tpg)) * tpg + k % tpg; }
    LBF_INLINE int group(int k) const { return wave + kWavesPerGroup * (k / tpg); }
};

LBF_INLINE WaveTiles wave_tiles(int wave, int T, int t_int) {
    WaveTiles w;
    w.wave = wave;
    w.tpg = t_int >= 32 ? t_int / 32 : 1;
    const int ntiles = (T + kTile - 1) / kTile;
    const int ngroups = (ntiles + w.tpg - 1) / w.tpg;
    const int mine = ngroups > wave ? (ngroups - wave + kWavesPerGroup - 1) / kWavesPerGroup : 0;
    w.ntw = mine * w.tpg;
    return w;
}

// K-steps of 8 stations of the fast FP16/BF16 worker: 4 to 8, the fewest that hold the stations (at least 4)
__host__ __device__ inline int fast_h_ksteps(int S) { return S <= 32 ? 4 : (S + 7) / 8; }

// Sample streams of the fast FP16/BF16 worker, the tile shape of its work
// items: 1, 2 or 4 streams of 32-sample tiles beside 8, 4 or 2 beam tiles of
// 32 (items of 256, 128 or 64 beams).  Fewer beams per item leave fewer waves
// idle when a block has few beams, and more streams give every step more
// samples to load; the measured table (tile_table.h) picks the count by
// input type, product, K-steps and beams of the block part.  Complex f32 samples
// always take one: a 16-byte chunk holds a single sample, and the loaders of
// more streams would need more registers.  A process-wide override serves
// the tuning sweep (lbf_set_tile_streams): each call copies it into its
// BlockDesc once (ns_force), so every part of one call sees the same value.
inline int fast_h_streams(const BlockDesc& d) {
    if (d.xtype == XT_CF32) return 1;
    if (d.ns_force) return d.ns_force;
    const int nb = d.b1 - d.b0;
    int bucket = 0;
    while (bucket < 4 && nb > kTileBeamMax[bucket]) ++bucket;
    return kTileStreams[d.xtype == XT_CI8 ? 0 : 1][d.product == PR_I ? 0 : 1][fast_h_ksteps(d.S) - 4][bucket];
}

// A block whose beams beyond the last whole 256-beam group number at most 128
// is taken in two parts: the 256-beam groups, and the rest as 128-beam items
// (half the padding of a last 256-beam group).  Returns the number of parts
// (1 or 2) written to part[].
inline int split_fast_h(const BlockDesc& d, BlockDesc* part) {
    const int nb = d.b1 - d.b0, tail = nb % 256;
    part[0] = d;
    if (nb <= 256 || tail == 0 || tail > 128) return 1;
    part[0].b1 = d.b0 + (nb - tail);
    part[1] = d;
    part[1].b0 = part[0].b1;
    return 2;
}

// Work items of the fast FP16/BF16 worker: (channel of [c0, c0 + nc), group
// of 256/NS beams, segment of 32-sample tiles: seg_tiles) -- long blocks are
// cut in time so that few-channel blocks still spread over all compute
// units.
inline int block_items_fast_h(const BlockDesc& d, int* nbg) {
    const int per = 8 / fast_h_streams(d) * kTile;
    *nbg = (d.b1 - d.b0 + per - 1) / per;
    const int ntiles = (d.T + kTile - 1) / kTile, seg = seg_tiles(d, *nbg);
    return d.nc * *nbg * ((ntiles + seg - 1) / seg);
}

// work items of the fast FP32 worker: (channel of [c0, c0 + nc), group of 128
// beams, segment)
inline int block_items_fast_f32(const BlockDesc& d, int* nbg) {
    *nbg = (d.B + kBeamGroup - 1) / kBeamGroup;
    const int ntiles = (d.T + kTile - 1) / kTile, seg = seg_tiles(d, *nbg);
    return d.nc * *nbg * ((ntiles + seg - 1) / seg);
}

// number of (channel group, beam group) work items of a block
inline int block_items(const BlockDesc& d, int* nbg) {
    *nbg = (d.B + kBeamGroup - 1) / kBeamGroup;
    const int ngroups_c = d.product == PR_VOLT ? d.C : d.C / d.f_int;
    return ngroups_c * *nbg;
}

// Floats per (c', t') row of the internal channel-major Stokes staging (B
// beams x K parameters): a multiple of 32, so that every row starts on a
// 128-byte line
__host__ __device__ constexpr int staging_ld(int B, int K) { return (B * K + 31) & ~31; }

__host__ __device__ constexpr int sample_bytes(int xtype) { return xtype == XT_CI8 ? 4 : xtype == XT_CI16 ? 8 : 16; }

// The fast workers take up to 64 stations of complex int8/int16/f32 samples,
// voltages or Stokes with t_int <= 16 and no channel integration, and 8
// stations' worth of one channel-major station plane addressable with 31-bit
// byte offsets.  Everything else runs the generic workers.
__host__ __device__ inline bool fast_path(const BlockDesc& d) {
    if (d.S > kStationChunk) return false;
    if (d.product != PR_VOLT && (d.t_int > 16 || d.f_int != 1)) return false;
    // one channel's output (addressed with 32-bit buffer offsets, 2^31 = "no store")
    const double out_ch = d.product == PR_VOLT ? 16.0 * d.B * (double)d.T
                                               : 4.0 * staging_ld(d.B, d.product) * (double)(d.T / d.t_int);
    if (out_ch >= 2147483648.0 - 4096.0) return false;
    return 8.0 * (double)d.C * (double)d.T * sample_bytes(d.xtype) < 2147483648.0 - 4096.0;
}

// A Stokes block with channel integration (f_int a power of two up to 64)
// whose channels the fast workers can form one at a time: their per-channel
// products (integrated in time only) go through staging, and the pass out of
// the staging sums each group of f_int channels.
__host__ __device__ inline bool fast_path_fint(const BlockDesc& d) {
    if (d.product == PR_VOLT || d.f_int < 2 || d.f_int > 64 || (d.f_int & (d.f_int - 1))) return false;
    BlockDesc e = d;
    e.f_int = 1;
    return fast_path(e);
}

// Descriptor over the planes of the valid stations of group [s0, s0 + 8)
// (group_base, group_range): offsets of stations >= S are out of range and
// read as zero; a group with no valid station has range 0.
LBF_INLINE __amdgpu_buffer_rsrc_t group_rsrc(const void* x, int s0, int S, uint32_t stride_bytes) {
    const uint64_t base = reinterpret_cast<uint64_t>(x) + group_base(s0, stride_bytes);
    // the values are wave-uniform; keep them in scalar registers so the
    // buffer instruction takes them directly
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    const uint32_t nrec = __builtin_amdgcn_readfirstlane(group_range(s0, S, stride_bytes));
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, (int)nrec,
                                             0x00020000);
}

template <int XT> LBF_INLINE typename Raw<XT>::type buffer_sample(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> LBF_INLINE int buffer_sample<XT_CI8>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}
template <> LBF_INLINE shortx4 buffer_sample<XT_CI16>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef int int2v __attribute__((ext_vector_type(2)));
    const int2v v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return __builtin_bit_cast(shortx4, v);
}
template <> LBF_INLINE floatx4 buffer_sample<XT_CF32>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}

}  // namespace lbf
