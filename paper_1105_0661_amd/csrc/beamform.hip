// beamform.hip -- the tied-array beam former on MFMA (gfx950).
//
// Per channel c the beam former is a complex GEMM (Section 4.3 of Mol &
// Romein: each beam is a weighted complex sum of the station signals):
//     y[c][b][t][p] = sum_s w[c][b][s] x[s][c][t][p].
// It runs on the matrix cores as a real GEMM with the time samples on the
// MFMA rows, the beams on the columns and (station, re/im) on the reduction
// axis.  The complex product is split into two real products that share the
// weight operand B = (w_re, w_im):
//     Re y = A_r . B   with A_r = ( x_re, -x_im)
//     Im y = A_i . B   with A_i = ( x_im,  x_re)
// so each lane ends up holding the real and imaginary parts of both
// polarisations of the same (sample, beam) -- the Stokes epilogue
// (Section 4.5) and the integration (Section 5.1) then need no data exchange
// for up to 16 integrated samples.
//
// Work item = (channel group of f_int channels, group of up to 128 beams).
// A work group of 4 waves holds that beam group's weights for one channel in
// LDS; each wave walks its own 32-sample tiles, streaming the station samples
// straight from HBM into MFMA operand registers (int -> float/f16/bf16 in
// registers, no extra pass), with a prefetch ring so loads overlap the MFMAs.
#include "lbf_device.h"
#include "lbf_launch.h"

namespace lbf {

constexpr int kBeamGroup = 128;                 // beams per work item (4 MFMA tiles)
constexpr int kBeamTiles = kBeamGroup / kTile;
constexpr int kStationChunk = 64;               // stations whose weights sit in LDS at once
constexpr int kWavesPerGroup = 4;
constexpr int kThreads = kWave * kWavesPerGroup;

// ---------------------------------------------------------------------------
// raw sample loads (kept raw in the prefetch ring, converted when used)
// ---------------------------------------------------------------------------
template <int XT> struct Raw;
template <> struct Raw<XT_CI8> {
    typedef int type;
    __device__ static inline type load(const void* p, size_t i) { return reinterpret_cast<const int*>(p)[i]; }
    __device__ static inline floatx4 cvt(type v) {
        floatx4 r;
        r[0] = (float)(int8_t)(v & 0xff);
        r[1] = (float)(int8_t)((v >> 8) & 0xff);
        r[2] = (float)(int8_t)((v >> 16) & 0xff);
        r[3] = (float)(int8_t)((v >> 24) & 0xff);
        return r;
    }
    __device__ static inline type zero() { return 0; }
};
template <> struct Raw<XT_CI16> {
    typedef shortx4 type;
    __device__ static inline type load(const void* p, size_t i) { return reinterpret_cast<const shortx4*>(p)[i]; }
    __device__ static inline floatx4 cvt(type v) {
        floatx4 r;
        r[0] = (float)v[0];
        r[1] = (float)v[1];
        r[2] = (float)v[2];
        r[3] = (float)v[3];
        return r;
    }
    __device__ static inline type zero() { type z = {0, 0, 0, 0}; return z; }
};
template <> struct Raw<XT_CF32> {
    typedef floatx4 type;
    __device__ static inline type load(const void* p, size_t i) { return reinterpret_cast<const floatx4*>(p)[i]; }
    __device__ static inline floatx4 cvt(type v) { return v; }
    __device__ static inline type zero() { type z = {0.f, 0.f, 0.f, 0.f}; return z; }
};

// ---------------------------------------------------------------------------
// epilogue: voltages, or Stokes + integration + beam-major store
// ---------------------------------------------------------------------------

// v[i] <- sum of v[i*ti .. i*ti+ti-1] for i < 16/ti (ti = 1, 2, 4, 8, 16)
__device__ inline void group_sum16(float (&v)[16], int ti) {
    if (ti >= 2) {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = v[2 * i] + v[2 * i + 1];
    }
    if (ti >= 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = v[2 * i] + v[2 * i + 1];
    }
    if (ti >= 8) {
#pragma unroll
        for (int i = 0; i < 2; ++i) v[i] = v[2 * i] + v[2 * i + 1];
    }
    if (ti >= 16) v[0] = v[0] + v[1];
}

struct EpiCtx {
    float* out;
    int B, T, C2, T2, K;
    int c;          // channel (voltages)
    int g;          // output channel c' (Stokes)
    int first;      // first channel of the f_int group: store, else accumulate
    int t_int;
};

// Stokes parameter kk of one sample from (Xr, Xi, Yr, Yi)
template <int KK>
__device__ inline float stokes_of(float xr, float xi, float yr, float yi) {
    if (KK == 0) return (xr * xr + xi * xi) + (yr * yr + yi * yi);
    if (KK == 1) return (xr * xr + xi * xi) - (yr * yr + yi * yi);
    if (KK == 2) return 2.0f * (xr * yr + xi * yi);
    return 2.0f * (xi * yr - xr * yi);
}

__device__ inline void store_or_add(float* p, float v, int first) {
    if (first) *p = v;
    else *p = *p + v;
}

// Stokes parameter KK of one 32x32 tile (acc = {Xre, Xim, Yre, Yim}) for a
// tile starting at sample t0, integrated over t_int (< 32) and stored.
template <int KK>
__device__ inline void stokes_tile_store(const floatx16 (&acc)[4], const EpiCtx& e, int beam, int t0, int h) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = stokes_of<KK>(acc[0][k], acc[1][k], acc[2][k], acc[3][k]);
    const int ti = e.t_int;
    group_sum16(v, ti);
    const int nout = 16 / ti;
    const int tq0 = (t0 + 16 * h) / ti;
    if (beam >= e.B) return;
    float* base = e.out + ((size_t)beam * e.K + KK) * e.T2 * (size_t)e.C2 + e.g;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i < nout) {
            const int tq = tq0 + i;
            if (tq < e.T2) store_or_add(base + (size_t)tq * e.C2, v[i], e.first);
        }
    }
}

// in-lane total of Stokes KK over the 16 samples of this lane half
template <int KK>
__device__ inline float stokes_tile_total(const floatx16 (&acc)[4]) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = stokes_of<KK>(acc[0][k], acc[1][k], acc[2][k], acc[3][k]);
    group_sum16(v, 16);
    return v[0];
}

template <int PR>
__device__ inline void epilogue_tile(const floatx16 (&acc)[4], const EpiCtx& e, int beam, int t0, int h) {
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
        stokes_tile_store<0>(acc, e, beam, t0, h);
        if (PR == PR_IQUV) {
            stokes_tile_store<1>(acc, e, beam, t0, h);
            stokes_tile_store<2>(acc, e, beam, t0, h);
            stokes_tile_store<3>(acc, e, beam, t0, h);
        }
    }
}

// add this tile's totals (t_int >= 32 path) into running group sums
template <int PR>
__device__ inline void accumulate_tile_totals(const floatx16 (&acc)[4], float (&gs)[4]) {
    gs[0] += stokes_tile_total<0>(acc);
    if (PR == PR_IQUV) {
        gs[1] += stokes_tile_total<1>(acc);
        gs[2] += stokes_tile_total<2>(acc);
        gs[3] += stokes_tile_total<3>(acc);
    }
}

template <int PR>
__device__ inline void store_group_totals(float (&gs)[4], const EpiCtx& e, int beam, int tq, int h) {
    constexpr int K = PR == PR_IQUV ? 4 : 1;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
        // lane half 0 and 1 cover samples 0-15 and 16-31 of each tile
        const float other = __shfl_xor(gs[kk], 32, kWave);
        gs[kk] = h == 0 ? gs[kk] + other : other + gs[kk];
    }
    if (h != 0 || beam >= e.B || tq >= e.T2) return;
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
        store_or_add(e.out + (((size_t)beam * e.K + kk) * e.T2 + tq) * (size_t)e.C2 + e.g, gs[kk], e.first);
}

// ---------------------------------------------------------------------------
// weight staging into LDS
// ---------------------------------------------------------------------------

// FP32 weights: wl[sl][ri][b] floats for stations [s0, s0+64) of beams
// [b0, b0+128) of channel c; zero outside [0,S) x [0,B).
__device__ inline void stage_weights_f32(float* wl, const BlockDesc& d, int c, int b0, int s0) {
    const float* w = reinterpret_cast<const float*>(d.w);
    for (int i = threadIdx.x; i < kStationChunk * kBeamGroup; i += kThreads) {
        const int sl = i % kStationChunk, bl = i / kStationChunk;
        const int s = s0 + sl, b = b0 + bl;
        float re = 0.f, im = 0.f;
        if (s < d.S && b < d.B) {
            const size_t o = (((size_t)c * d.B + b) * d.S + s) * 2;
            re = w[o];
            im = w[o + 1];
        }
        wl[(sl * 2 + 0) * kBeamGroup + bl] = re;
        wl[(sl * 2 + 1) * kBeamGroup + bl] = im;
    }
}

// FP16/BF16 weights: wh[b][sl] packed complex (32 bits), row stride
// kWRow words (64 stations + 16-byte pad against LDS bank conflicts).
constexpr int kWRow = kStationChunk + 4;
__device__ inline void stage_weights_h(uint32_t* wh, const BlockDesc& d, int c, int b0, int s0) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(d.w);
    for (int i = threadIdx.x; i < kStationChunk * kBeamGroup; i += kThreads) {
        const int sl = i % kStationChunk, bl = i / kStationChunk;
        const int s = s0 + sl, b = b0 + bl;
        uint32_t v = 0u;
        if (s < d.S && b < d.B) v = w[((size_t)c * d.B + b) * d.S + s];
        wh[bl * kWRow + sl] = v;
    }
}

// ---------------------------------------------------------------------------
// the per-item worker, FP32 operands (MFMA 32x32x2 f32, one station per step)
// ---------------------------------------------------------------------------
template <int XT, int PR>
__device__ void item_f32(const BlockDesc& d, int item, int nbg, float* wl) {
    typedef Raw<XT> R;
    const int g = item / nbg, bg = item % nbg;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int S = d.S, C = d.C, T = d.T;
    const int b0 = bg * kBeamGroup;
    const int ntl = min(kBeamTiles, (d.B - b0 + kTile - 1) / kTile);
    const int nchunk = (S + kStationChunk - 1) / kStationChunk;
    const int t_int = PR == PR_VOLT ? 1 : d.t_int;
    const int tiles_per_group = t_int >= 32 ? t_int / 32 : 1;
    const int ntiles = (T + kTile - 1) / kTile;
    const int ngroups = (ntiles + tiles_per_group - 1) / tiles_per_group;
    const int trow = tile_row_sample(r);

    EpiCtx e;
    e.out = reinterpret_cast<float*>(d.out);
    e.B = d.B; e.T = T; e.K = PR == PR_IQUV ? 4 : 1;
    e.C2 = C / (PR == PR_VOLT ? 1 : d.f_int);
    e.T2 = T / t_int; e.t_int = t_int; e.g = g;
    const int f_int = PR == PR_VOLT ? 1 : d.f_int;

    for (int j = 0; j < f_int; ++j) {
        const int c = g * f_int + j;
        e.c = c;
        e.first = j == 0;
        if (nchunk == 1) {
            __syncthreads();
            stage_weights_f32(wl, d, c, b0, 0);
            __syncthreads();
        }
        for (int grp0 = 0; grp0 < ngroups; grp0 += kWavesPerGroup) {
            const int grp = grp0 + wave;
            const bool active = grp < ngroups;
            float gs[kBeamTiles][4];
#pragma unroll
            for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) gs[a][q] = 0.f;
            for (int tg = 0; tg < tiles_per_group; ++tg) {
                const int tile = grp * tiles_per_group + tg;
                const int t0 = tile * kTile;
                const int t = t0 + trow;
                const bool tok = active && t < T;
                floatx16 acc[kBeamTiles][4];
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int k = 0; k < 16; ++k) acc[a][q][k] = 0.f;
                for (int ch = 0; ch < nchunk; ++ch) {
                    const int s0 = ch * kStationChunk;
                    if (nchunk > 1) {
                        __syncthreads();
                        stage_weights_f32(wl, d, c, b0, s0);
                        __syncthreads();
                    }
                    if (!active) continue;
                    const int ns = min(kStationChunk, S - s0);
                    const size_t stride = (size_t)C * T;            // samples between stations
                    size_t idx = ((size_t)s0 * C + c) * T + t;
                    // prefetch ring of 4 stations
                    typename R::type ring[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        ring[i] = (tok && i < ns) ? R::load(d.x, idx + i * stride) : R::zero();
                    for (int sl = 0; sl < ns; sl += 4) {
                        typename R::type cur[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) cur[i] = ring[i];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int sn = sl + 4 + i;
                            ring[i] = (tok && sn < ns) ? R::load(d.x, idx + (size_t)sn * stride) : R::zero();
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (sl + i < ns) {
                                const floatx4 v = R::cvt(cur[i]);
                                const float aXr = h ? -v[1] : v[0];
                                const float aXi = h ? v[0] : v[1];
                                const float aYr = h ? -v[3] : v[2];
                                const float aYi = h ? v[2] : v[3];
                                const float* wrow = wl + ((sl + i) * 2 + h) * kBeamGroup + r;
#pragma unroll
                                for (int a = 0; a < kBeamTiles; ++a) {
                                    if (a < ntl) {
                                        const float bw = wrow[a * kTile];
                                        acc[a][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(aXr, bw, acc[a][0], 0, 0, 0);
                                        acc[a][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(aXi, bw, acc[a][1], 0, 0, 0);
                                        acc[a][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(aYr, bw, acc[a][2], 0, 0, 0);
                                        acc[a][3] = __builtin_amdgcn_mfma_f32_32x32x2f32(aYi, bw, acc[a][3], 0, 0, 0);
                                    }
                                }
                            }
                        }
                    }
                }
                if (!active) continue;
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a) {
                    if (a < ntl) {
                        const int beam = b0 + a * kTile + r;
                        if (PR == PR_VOLT || t_int < 32) epilogue_tile<PR>(acc[a], e, beam, t0, h);
                        else accumulate_tile_totals<PR>(acc[a], gs[a]);
                    }
                }
            }
            if (PR != PR_VOLT && t_int >= 32 && active) {
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a)
                    if (a < ntl) store_group_totals<PR>(gs[a], e, b0 + a * kTile + r, grp, h);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// the per-item worker, FP16/BF16 operands (MFMA 32x32x16, 8 stations/step)
// ---------------------------------------------------------------------------
template <int CT> struct MfmaH;
template <> struct MfmaH<CT_F16> {
    typedef halfx8 vec;
    __device__ static inline floatx16 mfma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct MfmaH<CT_BF16> {
    typedef bf16x8 vec;
    __device__ static inline floatx16 mfma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int XT, int CT, int PR>
__device__ void item_h(const BlockDesc& d, int item, int nbg, uint32_t* wh) {
    typedef Raw<XT> R;
    typedef typename MfmaH<CT>::vec V;
    const int g = item / nbg, bg = item % nbg;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int S = d.S, C = d.C, T = d.T;
    const int b0 = bg * kBeamGroup;
    const int ntl = min(kBeamTiles, (d.B - b0 + kTile - 1) / kTile);
    const int nchunk = (S + kStationChunk - 1) / kStationChunk;
    const int t_int = PR == PR_VOLT ? 1 : d.t_int;
    const int tiles_per_group = t_int >= 32 ? t_int / 32 : 1;
    const int ntiles = (T + kTile - 1) / kTile;
    const int ngroups = (ntiles + tiles_per_group - 1) / tiles_per_group;
    const int trow = tile_row_sample(r);

    EpiCtx e;
    e.out = reinterpret_cast<float*>(d.out);
    e.B = d.B; e.T = T; e.K = PR == PR_IQUV ? 4 : 1;
    e.C2 = C / (PR == PR_VOLT ? 1 : d.f_int);
    e.T2 = T / t_int; e.t_int = t_int; e.g = g;
    const int f_int = PR == PR_VOLT ? 1 : d.f_int;

    for (int j = 0; j < f_int; ++j) {
        const int c = g * f_int + j;
        e.c = c;
        e.first = j == 0;
        if (nchunk == 1) {
            __syncthreads();
            stage_weights_h(wh, d, c, b0, 0);
            __syncthreads();
        }
        for (int grp0 = 0; grp0 < ngroups; grp0 += kWavesPerGroup) {
            const int grp = grp0 + wave;
            const bool active = grp < ngroups;
            float gs[kBeamTiles][4];
#pragma unroll
            for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) gs[a][q] = 0.f;
            for (int tg = 0; tg < tiles_per_group; ++tg) {
                const int tile = grp * tiles_per_group + tg;
                const int t0 = tile * kTile;
                const int t = t0 + trow;
                const bool tok = active && t < T;
                floatx16 acc[kBeamTiles][4];
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int k = 0; k < 16; ++k) acc[a][q][k] = 0.f;
                for (int ch = 0; ch < nchunk; ++ch) {
                    const int s0 = ch * kStationChunk;
                    if (nchunk > 1) {
                        __syncthreads();
                        stage_weights_h(wh, d, c, b0, s0);
                        __syncthreads();
                    }
                    if (!active) continue;
                    const int ns = min(kStationChunk, S - s0);
                    const int nk = (ns + 7) / 8;                      // K-steps of 8 stations
                    const size_t stride = (size_t)C * T;
                    const size_t idx0 = ((size_t)s0 * C + c) * T + t;
                    // this lane's 4 stations of K-step kk are s0 + 8kk + 4h + i
                    typename R::type ring[2][4];
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int sl = 8 * p + 4 * h + i;
                            ring[p][i] = (tok && p < nk && sl < ns) ? R::load(d.x, idx0 + (size_t)sl * stride) : R::zero();
                        }
                    for (int kk = 0; kk < nk; ++kk) {
                        typename R::type cur[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) { cur[i] = ring[0][i]; ring[0][i] = ring[1][i]; }
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int sl = 8 * (kk + 2) + 4 * h + i;
                            ring[1][i] = (tok && sl < ns) ? R::load(d.x, idx0 + (size_t)sl * stride) : R::zero();
                        }
                        uint32_t ar[2][4], ai[2][4];            // A_r, A_i for X (0) and Y (1)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const floatx4 v = R::cvt(cur[i]);
                            ar[0][i] = pack16(f32_to_bits<CT>(v[0]), f32_to_bits<CT>(-v[1]));
                            ai[0][i] = pack16(f32_to_bits<CT>(v[1]), f32_to_bits<CT>(v[0]));
                            ar[1][i] = pack16(f32_to_bits<CT>(v[2]), f32_to_bits<CT>(-v[3]));
                            ai[1][i] = pack16(f32_to_bits<CT>(v[3]), f32_to_bits<CT>(v[2]));
                        }
                        u32x4 uxr = {ar[0][0], ar[0][1], ar[0][2], ar[0][3]};
                        u32x4 uxi = {ai[0][0], ai[0][1], ai[0][2], ai[0][3]};
                        u32x4 uyr = {ar[1][0], ar[1][1], ar[1][2], ar[1][3]};
                        u32x4 uyi = {ai[1][0], ai[1][1], ai[1][2], ai[1][3]};
                        const V axr = __builtin_bit_cast(V, uxr);
                        const V axi = __builtin_bit_cast(V, uxi);
                        const V ayr = __builtin_bit_cast(V, uyr);
                        const V ayi = __builtin_bit_cast(V, uyi);
                        const uint32_t* wrow = wh + r * kWRow + 8 * kk + 4 * h;
#pragma unroll
                        for (int a = 0; a < kBeamTiles; ++a) {
                            if (a < ntl) {
                                const u32x4 wb = *reinterpret_cast<const u32x4*>(wrow + a * kTile * kWRow);
                                const V bw = __builtin_bit_cast(V, wb);
                                acc[a][0] = MfmaH<CT>::mfma(axr, bw, acc[a][0]);
                                acc[a][1] = MfmaH<CT>::mfma(axi, bw, acc[a][1]);
                                acc[a][2] = MfmaH<CT>::mfma(ayr, bw, acc[a][2]);
                                acc[a][3] = MfmaH<CT>::mfma(ayi, bw, acc[a][3]);
                            }
                        }
                    }
                }
                if (!active) continue;
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a) {
                    if (a < ntl) {
                        const int beam = b0 + a * kTile + r;
                        if (PR == PR_VOLT || t_int < 32) epilogue_tile<PR>(acc[a], e, beam, t0, h);
                        else accumulate_tile_totals<PR>(acc[a], gs[a]);
                    }
                }
            }
            if (PR != PR_VOLT && t_int >= 32 && active) {
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a)
                    if (a < ntl) store_group_totals<PR>(gs[a], e, b0 + a * kTile + r, grp, h);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <int XT, int PR>
__global__ __launch_bounds__(kThreads) void bf_f32_kernel(BlockDesc d, int nbg, int nitems) {
    __shared__ float wl[kStationChunk * 2 * kBeamGroup];
    item_f32<XT, PR>(d, xcd_remap(blockIdx.x, nitems), nbg, wl);
}

template <int XT, int CT, int PR>
__global__ __launch_bounds__(kThreads) void bf_h_kernel(BlockDesc d, int nbg, int nitems) {
    __shared__ __attribute__((aligned(16))) uint32_t wh[kBeamGroup * kWRow];
    item_h<XT, CT, PR>(d, xcd_remap(blockIdx.x, nitems), nbg, wh);
}

// Persistent batch kernel: work items (block, channel group, beam group) from
// several blocks, pulled from a device counter until the list is exhausted.
// Every work group leaves the loop once the counter passes the item count.
struct BatchArgs {
    BlockDesc blk[kMaxBatch];
    int item_start[kMaxBatch + 1];   // prefix sums of items per block
    int nbg[kMaxBatch];
    int n;
};

template <int CT>
__device__ void batch_dispatch(const BlockDesc& d, int item, int nbg, uint32_t* wh) {
    if (d.xtype == XT_CI8) {
        if (d.product == PR_I) item_h<XT_CI8, CT, PR_I>(d, item, nbg, wh);
        else item_h<XT_CI8, CT, PR_IQUV>(d, item, nbg, wh);
    } else if (d.xtype == XT_CI16) {
        if (d.product == PR_I) item_h<XT_CI16, CT, PR_I>(d, item, nbg, wh);
        else item_h<XT_CI16, CT, PR_IQUV>(d, item, nbg, wh);
    } else {
        if (d.product == PR_I) item_h<XT_CF32, CT, PR_I>(d, item, nbg, wh);
        else item_h<XT_CF32, CT, PR_IQUV>(d, item, nbg, wh);
    }
}

template <int CT>
__global__ __launch_bounds__(kThreads) void bf_batch_kernel(BatchArgs a, int* counter) {
    __shared__ __attribute__((aligned(16))) uint32_t wh[kBeamGroup * kWRow];
    __shared__ int next;
    const int total = a.item_start[a.n];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        if (it >= total) break;
        int j = 0;
        while (j + 1 < a.n && a.item_start[j + 1] <= it) ++j;
        batch_dispatch<CT>(a.blk[j], it - a.item_start[j], a.nbg[j], wh);
    }
}

__global__ void fill_int_kernel(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int items_of(const BlockDesc& d, int* nbg) {
    *nbg = (d.B + kBeamGroup - 1) / kBeamGroup;
    const int ngroups_c = d.product == PR_VOLT ? d.C : d.C / d.f_int;
    return ngroups_c * *nbg;
}

template <int XT>
static hipError_t launch_f32(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    dim3 grid(n), block(kThreads);
    switch (d.product) {
        case PR_VOLT: hipLaunchKernelGGL((bf_f32_kernel<XT, PR_VOLT>), grid, block, 0, st, d, nbg, n); break;
        case PR_I: hipLaunchKernelGGL((bf_f32_kernel<XT, PR_I>), grid, block, 0, st, d, nbg, n); break;
        default: hipLaunchKernelGGL((bf_f32_kernel<XT, PR_IQUV>), grid, block, 0, st, d, nbg, n); break;
    }
    return hipGetLastError();
}

template <int XT, int CT>
static hipError_t launch_h(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    dim3 grid(n), block(kThreads);
    switch (d.product) {
        case PR_VOLT: hipLaunchKernelGGL((bf_h_kernel<XT, CT, PR_VOLT>), grid, block, 0, st, d, nbg, n); break;
        case PR_I: hipLaunchKernelGGL((bf_h_kernel<XT, CT, PR_I>), grid, block, 0, st, d, nbg, n); break;
        default: hipLaunchKernelGGL((bf_h_kernel<XT, CT, PR_IQUV>), grid, block, 0, st, d, nbg, n); break;
    }
    return hipGetLastError();
}

hipError_t launch_beamform(const BlockDesc& d, hipStream_t st) {
    int nbg;
    const int n = items_of(d, &nbg);
    if (d.ctype == CT_F32) {
        if (d.xtype == XT_CI8) return launch_f32<XT_CI8>(d, nbg, n, st);
        if (d.xtype == XT_CI16) return launch_f32<XT_CI16>(d, nbg, n, st);
        return launch_f32<XT_CF32>(d, nbg, n, st);
    }
    if (d.ctype == CT_F16) {
        if (d.xtype == XT_CI8) return launch_h<XT_CI8, CT_F16>(d, nbg, n, st);
        if (d.xtype == XT_CI16) return launch_h<XT_CI16, CT_F16>(d, nbg, n, st);
        return launch_h<XT_CF32, CT_F16>(d, nbg, n, st);
    }
    if (d.xtype == XT_CI8) return launch_h<XT_CI8, CT_BF16>(d, nbg, n, st);
    if (d.xtype == XT_CI16) return launch_h<XT_CI16, CT_BF16>(d, nbg, n, st);
    return launch_h<XT_CF32, CT_BF16>(d, nbg, n, st);
}

hipError_t launch_beamform_batch(const BlockDesc* blks, int n, int* d_counter, hipStream_t st) {
    BatchArgs a;
    a.n = n;
    a.item_start[0] = 0;
    for (int j = 0; j < n; ++j) {
        a.blk[j] = blks[j];
        int nbg;
        const int items = items_of(blks[j], &nbg);
        a.nbg[j] = nbg;
        a.item_start[j + 1] = a.item_start[j] + items;
    }
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, st, d_counter, 1, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one resident work group per slot the hardware offers: the queue, not the
    // grid, spreads the uneven items
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (blks[0].ctype == CT_F16)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bf_batch_kernel<CT_F16>, kThreads, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bf_batch_kernel<CT_BF16>, kThreads, 0);
    if (per_cu < 1) per_cu = 1;
    const int total = a.item_start[n];
    const int slots = cus * per_cu;
    const int grid = total < slots ? total : slots;
    if (blks[0].ctype == CT_F16)
        hipLaunchKernelGGL(bf_batch_kernel<CT_F16>, dim3(grid), dim3(kThreads), 0, st, a, d_counter);
    else
        hipLaunchKernelGGL(bf_batch_kernel<CT_BF16>, dim3(grid), dim3(kThreads), 0, st, a, d_counter);
    return hipGetLastError();
}

}  // namespace lbf
