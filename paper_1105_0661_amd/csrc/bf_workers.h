// bf_workers.h -- the per-work-item contraction workers.
//
// Fast workers (up to 64 stations of complex int8/int16, t_int <= 16, no
// channel integration): item_f32_fast and item_h_fast, described where they
// are defined; they write Stokes products channel-major.
//
// Generic workers (any station count, complex float input, channel
// integration, t_int >= 32): work item = (channel group of f_int channels,
// group of up to 128 beams).  A work group of 4 waves stages that beam group's
// weights for one channel in LDS; each wave walks its own 32-sample tiles
// (groups of tiles when t_int >= 32), streaming station samples from HBM
// straight into MFMA operand registers, and ends each tile with the fused
// Stokes / integration / store epilogue in either output order.
#pragma once
#include <type_traits>

#include "bf_common.h"

namespace lbf {

// ===========================================================================
// fast workers: up to 64 stations of complex int8/int16 samples
// ===========================================================================

// FP32 operands (MFMA 32x32x2 f32: one station per MFMA, K = (re, im)).
//
// A work item is one channel, 128 beams and a segment of sample tiles
// (seg_tiles); a work group has 8 waves (two per SIMD).  The weights of the
// 128 beams sit in LDS as three planes p0 = w_re, p1 = -w_im, p2 = w_im
// ([beam][station] rows), so that lane half h (the K index) multiplies the
// plain sample component a = (h ? x_im : x_re) by  wr = (h ? p1 : p0)  for
// Re y and by  wi = (h ? p0 : p2)  for Im y.  Wave w owns beam tile w % 4 and
// every other sample tile (stream w / 4); its two accumulator sets (4 x 16
// floats each, in VGPRs) alternate between tiles, and the Stokes epilogue of
// the previous tile is spread between the MFMAs of the current one (a wave's
// own VALU work overlaps its MFMAs).  Samples stream from HBM through an
// 8-deep register ring, one group of 8 stations ahead.
constexpr int kPlaneWords = kBeamGroup * kWRow;          // one plane: 34 KB

LBF_INLINE void stage_weights_f32_planes(float* pl, const BlockDesc& d, int c, int b0) {
    constexpr int R = kStationChunk * kBeamGroup / kThreadsH;   // 16 per thread
    constexpr int RS = kThreadsH / kStationChunk;                // beam rows per pass
    typedef float float2v __attribute__((ext_vector_type(2)));
    const int sl = threadIdx.x % kStationChunk, b1 = threadIdx.x / kStationChunk;
    const __amdgpu_buffer_rsrc_t rs = weight_rsrc(d, c, 8);
    const bool sok = sl < d.S;
    float2v v[R];
#pragma unroll
    for (int k = 0; k < R; ++k)
        v[k] = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)weight_off(b0 + b1 + RS * k, d.S, sl, 8), 0, 0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int bl = b1 + RS * k;
        const float wre = sok ? v[k][0] : 0.f, wim = sok ? v[k][1] : 0.f;
        pl[bl * kWRow + sl] = wre;
        pl[kPlaneWords + bl * kWRow + sl] = -wim;
        pl[2 * kPlaneWords + bl * kWRow + sl] = wim;
    }
}

template <int XT, int PR, int TI>
LBF_INLINE void item_f32_fast(const BlockDesc& d, int item, int nbg, float* pl) {
    typedef Raw<XT> R;
    typedef typename R::type RT;
    constexpr int BYTES = sizeof(RT);
    constexpr int NOUT = PR == PR_VOLT ? 1 : 16 / TI;
    const int T = d.T, S = d.S, B = d.B;
    const ItemPos ip = item_pos(d, item, nbg);
    const int c = ip.c, bg = ip.bg, tile_lo = ip.tile_lo, ntiles = ip.ntiles;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int bt = wave & 3, ts = wave >> 2;
    const int b0 = bg * kBeamGroup;
    const int beam = b0 + bt * kTile + r;
    const int nmine = ntiles > ts ? (ntiles - ts + 1) / 2 : 0;  // this wave's tiles
    // groups of 8 stations, rounded up to an even count so that group n of the
    // wave's sequence always sits in ring slot n % 2 = gi % 2 (a group past
    // the stations reads zeros and has zero weights)
    const int ngrp = min(8, ((S + 7) / 8 + 1) & ~1);
    const uint32_t stride_bytes = (uint32_t)((size_t)d.C * T * BYTES);
    const int T2 = PR == PR_VOLT ? T : T / TI;
    const __amdgpu_buffer_rsrc_t ors = channel_rsrc(d, c, out_channel_bytes(d, PR, T2));
    const int trow = tile_row_sample(r);
    // weights read one quad of stations ahead (8 more registers): where they
    // fit without spills -- not with complex float samples (16-byte ring
    // entries) nor beside the 16 output sums of unintegrated Stokes
    constexpr bool PF = XT != XT_CF32 && (PR == PR_VOLT || TI >= 2);

    stage_weights_f32_planes(pl, d, c, b0);
    __syncthreads();
    if (nmine == 0 || b0 + bt * kTile >= B) return;             // nothing of this wave's (no barrier follows)
    // LDS rows of this lane: the plane for Re y and the one for Im y
    int wro = (h ? kPlaneWords : 0) + (bt * kTile + r) * kWRow;
    int wio = (h ? 0 : 2 * kPlaneWords) + (bt * kTile + r) * kWRow;
    __asm__ volatile("" : "+v"(wro), "+v"(wio));
    // bit offset of this lane half's component in a raw sample word
    uint32_t hsh = (uint32_t)h * (XT == XT_CI8 ? 8u : 16u);
    __asm__ volatile("" : "+v"(hsh));

    auto tile_of = [&](int k) { return tile_lo + ts + 2 * k; };
    // Two-deep ring of 8-station groups: group n of the wave's sequence
    // (tile n / ngrp, group n % ngrp) lands in slot n % 2 two groups before
    // it is used, which covers a cache-missing load.
    RT ring[2][8];
    auto load_quad = [&](int slot, int q4, int n) {            // stations 4 q4 .. 4 q4 + 3 of group n
        const int k = min(n / ngrp, nmine - 1), g = n % ngrp;
        const int t = min(tile_of(k) * kTile + trow, T - 1);
        const __amdgpu_buffer_rsrc_t rs = group_rsrc(d.x, 8 * g, S, stride_bytes);
#pragma unroll
        for (int i = 4 * q4; i < 4 * q4 + 4; ++i)
            ring[slot][i] = buffer_sample<XT>(rs, sample_off(i, stride_bytes, c, T, t, BYTES));
    };
    auto epi_sample = [&](const floatx16 (&prev)[4], int tprev, bool okprev, int smp, float (&sm)[NOUT][4]) {
        if (PR == PR_VOLT) {
            const int t = tprev * kTile + 16 * h + smp;
            const uint32_t off = store_off(okprev && beam < B && t < T, volt_off(beam, T, t));
            floatx4 vv;
            vv[0] = prev[0][smp];
            vv[1] = prev[1][smp];
            vv[2] = prev[2][smp];
            vv[3] = prev[3][smp];
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, vv), ors, (int)off, 0, 0);
        } else {
            stokes_add<PR>(prev, smp, sm[smp / TI]);
        }
    };

    // one tile: MFMAs into acc, with the epilogue of prev (tile k-1) spread
    // over the station groups (two of its 16 samples per group)
    auto step = [&](int k, floatx16 (&acc)[4], const floatx16 (&prev)[4]) {
        const int tprev = tile_of(k - 1);
        const bool okprev = k >= 1;
        float sm[NOUT][4];
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
            for (int q = 0; q < 4; ++q) sm[o][q] = 0.f;
        // weights of the first 4 stations; with PF each later quad's are read
        // one quad ahead, so that the LDS latency passes under 16 MFMAs
        floatx4 br, bi;
        if constexpr (PF) {
            br = *reinterpret_cast<const floatx4*>(pl + wro);
            bi = *reinterpret_cast<const floatx4*>(pl + wio);
        }
#pragma unroll
        for (int gi = 0; gi < 8; ++gi) {
            if (gi < ngrp) {                                   // uniform
                // group n = k ngrp + gi sits in slot gi % 2; as soon as a quad
                // of its stations is converted, the same registers are
                // refilled with that quad of group n + 2
#pragma unroll
                for (int i4 = 0; i4 < 2; ++i4) {               // 4 stations at a time
                    const int s4 = 8 * gi + 4 * i4;
                    float ax[4], ay[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) R::half(ring[gi & 1][4 * i4 + i], hsh, ax[i], ay[i]);
                    load_quad(gi & 1, i4, k * ngrp + gi + 2);
                    floatx4 nbr, nbi;
                    if constexpr (PF) {
                        const int s4n = s4 + 4 < 8 * ngrp ? s4 + 4 : s4;    // the last quad reads itself again
                        nbr = *reinterpret_cast<const floatx4*>(pl + wro + s4n);
                        nbi = *reinterpret_cast<const floatx4*>(pl + wio + s4n);
                    }
                    __builtin_amdgcn_sched_barrier(0);                     // those reads issue before the MFMAs
                    if constexpr (!PF) {
                        br = *reinterpret_cast<const floatx4*>(pl + wro + s4);
                        bi = *reinterpret_cast<const floatx4*>(pl + wio + s4);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const bool first = gi == 0 && i4 == 0 && i == 0;
                        acc[0] = mfma_f32(ax[i], br[i], first ? zero16() : acc[0]);
                        acc[1] = mfma_f32(ax[i], bi[i], first ? zero16() : acc[1]);
                        acc[2] = mfma_f32(ay[i], br[i], first ? zero16() : acc[2]);
                        acc[3] = mfma_f32(ay[i], bi[i], first ? zero16() : acc[3]);
                    }
                    if constexpr (PF) {
                        br = nbr;
                        bi = nbi;
                    }
                }
            }
            epi_sample(prev, tprev, okprev, 2 * gi, sm);
            epi_sample(prev, tprev, okprev, 2 * gi + 1, sm);
            if (PR != PR_VOLT) {
#pragma unroll
                for (int o = 0; o < NOUT; ++o)
#pragma unroll
                    for (int q = 0; q < 4; ++q) __asm__ volatile("" : "+v"(sm[o][q]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (PR != PR_VOLT) {
            const int tq0 = (tprev * kTile + 16 * h) / TI;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                float v[4];
                stokes_from_sums<PR>(sm[o], v);
                const int tq = tq0 + o;
                stokes_store_row<PR>(v, ors, d.ld_row, tq, beam, okprev && beam < B && tq < T2);
            }
        }
    };
    auto final_epilogue = [&](const floatx16 (&prev)[4], int klast) {
        const int tile = tile_of(klast);
        const bool ok = klast >= 0 && beam < B;
        if (PR == PR_VOLT) volt_store_cm(prev, ors, T, beam, tile * kTile, h, ok);
        else stokes_store_cm<PR, TI>(prev, ors, d.ld_row, T2, beam, tile * kTile, h, ok);
    };

    load_quad(0, 0, 0);
    load_quad(0, 1, 0);
    load_quad(1, 0, 1);
    load_quad(1, 1, 1);
    floatx16 acc0[4], acc1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc1[q] = zero16();
    int k = 0;
    for (; k + 1 < nmine; k += 2) {
        step(k, acc0, acc1);
        step(k + 1, acc1, acc0);
    }
    if (k < nmine) {
        step(k, acc0, acc1);
        final_epilogue(acc0, k);
    } else {
        final_epilogue(acc1, k - 1);
    }
}

// FP16/BF16 operands (MFMA 32x32x16: 8 stations per K-step, NK K-steps:
// 4 to 8, the fewest that hold the block's stations).
//
// A work group of 8 waves (two per SIMD) takes one channel and NBT = 8/NS
// beam tiles of 32 beams; its tiles of 32 samples are split into NS streams.
// Each wave owns one beam tile and keeps that tile's weights for all K-steps
// in registers, as two variants  wr = (w_re, -w_im),  wi = (w_im, w_re),  so
// that with the plain sample operand a = (x_re, x_im) along K
//     Re y = a . wr,   Im y = a . wi.
// The samples of each 32-sample tile are loaded once per work group with
// 16-byte loads, converted once, and left in LDS (double buffered, one
// barrier per step) for all beam tiles to read.  Each wave runs a tile's
// epilogue between the MFMAs of its next tile (two accumulator sets), or,
// where the registers hold only one set, waves 4-7 run it at the start of
// the next step, so on every SIMD one wave's epilogue (VALU) meets the
// other wave's MFMAs.
constexpr int kARow = 68;                          // words per (sample, polarisation) row of an A tile
constexpr int kATileWords = kTile * 2 * kARow;     // 17 KB

// Word of station s, polarisation p, sample t (0..31) in an A tile.  Groups of
// 4 stations are XOR-swizzled by a_swz(t) so that neither the loaders' stores
// (lanes 4 samples apart for 8 consecutive t/4) nor the MFMA operand reads
// (lanes at samples t, t + 16 of the row map) collide in the banks; a lane
// still reads its 4 stations as one aligned 16-byte word.
LBF_INLINE int a_swz(int t) { return ((t >> 2) & 7) ^ ((t >> 4) & 1); }
LBF_INLINE int a_word(int t, int p, int s) { return (2 * t + p) * kARow + 4 * ((s >> 2) ^ a_swz(t)) + (s & 3); }

// 16 bytes of one station's consecutive samples -> operand words of sample j
template <int XT, int CT> struct Chunk;
template <int CT> struct Chunk<XT_CI8, CT> {
    static constexpr int samples = 4;
    LBF_INLINE static void xy(const u32x4& v, int j, uint32_t& fx, uint32_t& fy) {
        Conv2<XT_CI8, CT>::xy((int)v[j], fx, fy);
    }
};
template <int CT> struct Chunk<XT_CI16, CT> {
    static constexpr int samples = 2;
    LBF_INLINE static void xy(const u32x4& v, int j, uint32_t& fx, uint32_t& fy) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 w = {v[2 * j], v[2 * j + 1]};
        Conv2<XT_CI16, CT>::xy(__builtin_bit_cast(shortx4, w), fx, fy);
    }
};

// complex f32: one sample per 16-byte chunk, rounded to the operand type
// (round-to-nearest-even)
template <> struct Chunk<XT_CF32, CT_F16> {
    static constexpr int samples = 1;
    LBF_INLINE static void xy(const u32x4& v, int, uint32_t& fx, uint32_t& fy) {
        const floatx4 f = __builtin_bit_cast(floatx4, v);
        const halfx2 hx = {(_Float16)f[0], (_Float16)f[1]};
        const halfx2 hy = {(_Float16)f[2], (_Float16)f[3]};
        fx = __builtin_bit_cast(uint32_t, hx);
        fy = __builtin_bit_cast(uint32_t, hy);
    }
};
template <> struct Chunk<XT_CF32, CT_BF16> {
    static constexpr int samples = 1;
    LBF_INLINE static void xy(const u32x4& v, int, uint32_t& fx, uint32_t& fy) {
        const floatx4 f = __builtin_bit_cast(floatx4, v);
        fx = pack_bf16(f[0], f[1]);
        fy = pack_bf16(f[2], f[3]);
    }
};

// FP32 values of one packed 16-bit complex operand word (re low, im high)
template <int CT> LBF_INLINE void unpack2(uint32_t w, float& re, float& im);
template <> LBF_INLINE void unpack2<CT_F16>(uint32_t w, float& re, float& im) {
    const halfx2 v = __builtin_bit_cast(halfx2, w);
    re = (float)v[0];
    im = (float)v[1];
}
template <> LBF_INLINE void unpack2<CT_BF16>(uint32_t w, float& re, float& im) {
    re = __uint_as_float(w << 16);
    im = __uint_as_float(w & 0xffff0000u);
}

// Floats of LDS the incoherent-beam form of item_h_fast adds: per step
// parity, sample stream, wave of the stream and tile sample, four sums.
constexpr int kIncLdsFloats = 2 * 8 * kTile * 4;

// The worker's INC form also forms the incoherent beam (Section 3: the
// stations' powers summed, unweighted) of its channel and samples from the
// sample tile staged in LDS, so that one read of the station data gives both
// products.  Only the items of the first beam group do this, one per
// (channel, sample segment).  Each wave of a stream sums |X|^2, |Y|^2 and
// X conj(Y) over its share of the stations (lanes: tile sample; lane halves:
// halves of the share; products of 16-bit values are exact in FP32), the
// shares meet in LDS and are summed in wave order by the stream's first wave
// after the step's barrier, which then integrates t_int consecutive samples
// in an xor butterfly and stores I (Q, U, V) into inc [K][T'][C].
template <int XT, int CT, int PR, int TI, int NK, int NS, bool INC = false>
LBF_INLINE void item_h_fast(const BlockDesc& d, int item, int nbg, uint32_t* at) {
    typedef typename MfmaH<CT>::vec V;
    constexpr int BYTES = sample_bytes(XT);
    constexpr int NBT = 8 / NS;                            // beam tiles per item
    constexpr int SPC = Chunk<XT, CT>::samples;            // samples per 16-byte chunk
    constexpr int CPS = kTile / SPC;                       // chunks per station per tile
    constexpr int CPTILE = 8 * NK * CPS;                   // chunks per tile
    constexpr int CPT = (NS * CPTILE + kThreadsH - 1) / kThreadsH;   // chunks per thread per step
    // item = (channel, beam group, segment of sample tiles: seg_tiles)
    const int T = d.T;
    const ItemPos ip = item_pos(d, item, nbg);             // tiles [tile_lo, tile_lo + ntiles)
    const int c = ip.c, bg = ip.bg, tile_lo = ip.tile_lo, ntiles = ip.ntiles;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int bt = wave % NBT, sigma = wave / NBT;         // beam tile, sample stream
    const int S = d.S, bend = d.b1;
    const int beam = d.b0 + (bg * NBT + bt) * kTile + r;
    // a wave whose beam tile lies wholly past the block's beams forms nothing
    // (it still loads, stages and meets the barriers): its SIMD partner has
    // the matrix pipe to itself
    const bool idle = d.b0 + (bg * NBT + bt) * kTile >= d.b1;
    const int nsteps = (ntiles + NS - 1) / NS;
    const uint32_t stride_bytes = (uint32_t)((size_t)d.C * T * BYTES);
    const int T2 = PR == PR_VOLT ? T : T / TI;
    const __amdgpu_buffer_rsrc_t ors = channel_rsrc(d, c, out_channel_bytes(d, PR, T2));

    // this wave's weights, both variants, all K-steps
    u32x4 wr[NK], wi[NK];
    {
        const __amdgpu_buffer_rsrc_t rs = weight_rsrc(d, c, 4);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
            const u32x4 w = __builtin_bit_cast(
                u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)weight_off(beam, S, 8 * kk + 4 * h, 4), 0, 0));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                wr[kk][i] = neg_hi(w[i]);
                wi[kk][i] = swap16(w[i]);
            }
        }
    }

    // loaders: chunk j = tid + 512 i of a step covers stream j / CPTILE,
    // station (j % CPTILE) / CPS and samples SPC * (j % CPS) + [0, SPC)
    u32x4 raw[CPT];
    auto load_chunks_to = [&](int k, u32x4 (&dst)[CPT]) {
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const Chunk16 ch = h_chunk(tid + kThreadsH * i, k, NS, CPTILE, CPS, tile_lo, ntiles);
            // descriptor over the whole planes of the group's stations, the
            // channel in the offset: a ragged last tile reads past the end of
            // the channel into the next one, or past the last valid station
            // (out of range: zeros), never past the array
            const __amdgpu_buffer_rsrc_t rs = group_rsrc(d.x, ch.s & ~7, S, stride_bytes);
            const uint32_t off = sample_off(ch.s & 7, stride_bytes, c, T, ch.tile * kTile + ch.q * SPC, BYTES);
            dst[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
        }
    };
    auto load_chunks = [&](int k) { load_chunks_to(k, raw); };
    auto store_chunk_from = [&](int k, int i, const u32x4 (&src)[CPT]) {
        const int j = tid + kThreadsH * i;
        const int sg = j / CPTILE, jt = j % CPTILE, s = jt / CPS, q = jt % CPS;
        if (NS * CPTILE % kThreadsH == 0 || j < NS * CPTILE) {
            uint32_t* ab = at + (sg * 2 + (k & 1)) * kATileWords;
#pragma unroll
            for (int js = 0; js < SPC; ++js) {
                uint32_t fx, fy;
                Chunk<XT, CT>::xy(src[i], js, fx, fy);
                const int t = q * SPC + js;
                ab[a_word(t, 0, s)] = fx;
                ab[a_word(t, 1, s)] = fy;
            }
        }
    };
    auto store_chunk = [&](int k, int i) { store_chunk_from(k, i, raw); };

    // One step k, written out in the order it should run: K-step kk's four
    // MFMAs (operands read one K-step ahead from LDS), then 1/NK of the
    // epilogue of step k-1 from the other accumulator set, with scheduling
    // barriers between the slices so that the compiler keeps the VALU work
    // next to the MFMAs it is meant to overlap (a wave's own VALU
    // instructions run while its MFMAs do; another wave's on the same SIMD do
    // not).  The samples of step k+1 are loaded at the start and staged in
    // the last two slices.
    const int trow = tile_row_sample(r);
    const int sw = a_swz(trow);
    // two accumulator sets, unless the loaders' registers leave no room
    // (complex int16 with several streams, more than two chunks per thread)
    constexpr bool PIPE = !(XT == XT_CI16 && NS >= 2) && CPT <= 2;
    constexpr int NOUT = PR == PR_VOLT ? 1 : 16 / TI;

    // incoherent beam of the item's tiles (INC form, first beam group only)
    constexpr int SPW = 8 * NK / NBT;                      // stations per wave of a stream
    constexpr int SPH = (SPW + 1) / 2;                     // of which lane half 0 takes SPH, half 1 the rest
    float* incl = reinterpret_cast<float*>(at + NS * 2 * kATileWords);
    const bool inc_on = INC && PR != PR_VOLT && bg == 0 && d.b0 == 0;
    auto inc_partial = [&](int k) {                        // the tile of step k: this wave's share
        const uint32_t* tb = at + (sigma * 2 + (k & 1)) * kATileWords;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < SPH; ++i) {
            if (h * SPH + i >= SPW) break;                 // an odd share: half 1 has one station less
            const int s = bt * SPW + h * SPH + i;
            float xr, xi, yr, yi;
            unpack2<CT>(tb[a_word(r, 0, s)], xr, xi);
            unpack2<CT>(tb[a_word(r, 1, s)], yr, yi);
            v[0] = __builtin_fmaf(xi, xi, __builtin_fmaf(xr, xr, v[0]));
            v[1] = __builtin_fmaf(yi, yi, __builtin_fmaf(yr, yr, v[1]));
            v[2] = __builtin_fmaf(xi, yi, __builtin_fmaf(xr, yr, v[2]));
            v[3] = __builtin_fmaf(-xr, yi, __builtin_fmaf(xi, yr, v[3]));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], 32, kWave);   // the two lane halves
        if (h == 0) {
            floatx4 o;
            o[0] = v[0];
            o[1] = v[1];
            o[2] = v[2];
            o[3] = v[3];
            *reinterpret_cast<floatx4*>(incl + ((((k & 1) * NS + sigma) * NBT + bt) * kTile + r) * 4) = o;
        }
    };
    auto inc_finish = [&](int k) {                         // after the barrier: step k's tile, first wave of the stream
        const int tile = tile_lo + sigma + NS * k;
        if (bt != 0 || k < 0 || tile >= tile_lo + ntiles) return;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int w = 0; w < NBT; ++w) {
            const floatx4 p = *reinterpret_cast<const floatx4*>(incl + ((((k & 1) * NS + sigma) * NBT + w) * kTile + r) * 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += p[q];
        }
#pragma unroll
        for (int m = 1; m < TI; m <<= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], m, kWave);
        float o[4];
        stokes_from_sums<PR_IQUV>(v, o);                   // I, Q, U, V from |X|^2, |Y|^2, X conj(Y)
        const int tq = (tile * kTile + r) / TI;
        if (h == 0 && (r & (TI - 1)) == 0 && tq < T2) {
            constexpr int K = PR == PR_IQUV ? 4 : 1;
#pragma unroll
            for (int kk = 0; kk < K; ++kk) d.inc[((size_t)kk * T2 + tq) * d.C + c] = o[kk];
        }
    };
    auto step = [&](int k, floatx16 (&acc)[4], const floatx16 (&prev)[4]) {
        load_chunks(k + 1);
        int rowx = (sigma * 2 + (k & 1)) * kATileWords + 2 * trow * kARow;
        __asm__ volatile("" : "+v"(rowx));
        const uint32_t* ax0 = at + rowx;
        u32x4 ax[2], ay[2];
        ax[0] = *reinterpret_cast<const u32x4*>(ax0 + 4 * (h ^ sw));
        ay[0] = *reinterpret_cast<const u32x4*>(ax0 + kARow + 4 * (h ^ sw));
        const int tprev = tile_lo + sigma + NS * (k - 1);
        const bool okprev = k >= 1 && tprev < tile_lo + ntiles && beam < bend;
        float sm[NOUT][4];
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
            for (int q = 0; q < 4; ++q) sm[o][q] = 0.f;
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
            if (kk + 1 < NK) {
                const int off = 4 * ((2 * (kk + 1) + h) ^ sw);
                ax[(kk + 1) & 1] = *reinterpret_cast<const u32x4*>(ax0 + off);
                ay[(kk + 1) & 1] = *reinterpret_cast<const u32x4*>(ax0 + kARow + off);
            }
            const V a = __builtin_bit_cast(V, ax[kk & 1]), b = __builtin_bit_cast(V, ay[kk & 1]);
            const V br = __builtin_bit_cast(V, wr[kk]), bi = __builtin_bit_cast(V, wi[kk]);
            acc[0] = MfmaH<CT>::mfma(a, br, kk == 0 ? zero16() : acc[0]);
            acc[1] = MfmaH<CT>::mfma(a, bi, kk == 0 ? zero16() : acc[1]);
            acc[2] = MfmaH<CT>::mfma(b, br, kk == 0 ? zero16() : acc[2]);
            acc[3] = MfmaH<CT>::mfma(b, bi, kk == 0 ? zero16() : acc[3]);
            // epilogue slice: samples [16 kk / NK, 16 (kk + 1) / NK) of the previous tile
#pragma unroll
            for (int smp = 16 * kk / NK; smp < 16 * (kk + 1) / NK; ++smp) {
                if (PR == PR_VOLT) {
                    const int t = tprev * kTile + 16 * h + smp;
                    const uint32_t off = store_off(okprev && t < T, volt_off(beam, T, t));
                    floatx4 v;
                    v[0] = prev[0][smp];
                    v[1] = prev[1][smp];
                    v[2] = prev[2][smp];
                    v[3] = prev[3][smp];
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), ors, (int)off, 0, 0);
                } else {
                    stokes_add<PR>(prev, smp, sm[smp / TI]);
                }
            }
            if (kk >= NK - 2) {                              // stage step k+1's samples
#pragma unroll
                for (int i = 0; i < CPT; ++i)
                    if (i % 2 == kk - (NK - 2)) store_chunk(k + 1, i);
            }
            if (INC && inc_on) {
                if (kk == 0) inc_partial(k);
                if (kk == 1) inc_finish(k - 1);
            }
            // keep this slice's sums here (left alone, the compiler sinks the
            // whole epilogue below the last MFMA)
            if (PR != PR_VOLT) {
#pragma unroll
                for (int o = 0; o < NOUT; ++o)
#pragma unroll
                    for (int q = 0; q < 4; ++q) __asm__ volatile("" : "+v"(sm[o][q]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (PR != PR_VOLT) {
            const int tq0 = (tprev * kTile + 16 * h) / TI;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                float v[4];
                stokes_from_sums<PR>(sm[o], v);
                const int tq = tq0 + o;
                stokes_store_row<PR>(v, ors, d.ld_row, tq, beam, okprev && tq < T2);
            }
        }
        __syncthreads();
    };
    // the step of an idle wave: the loaders' and the incoherent beam's share only
    auto idle_step = [&](int k) {
        load_chunks(k + 1);
        if (INC && inc_on) inc_partial(k);
#pragma unroll
        for (int i = 0; i < CPT; ++i) store_chunk(k + 1, i);
        if (INC && inc_on) inc_finish(k - 1);
        __syncthreads();
    };
    // the last tile's epilogue: one more step without MFMAs
    auto final_epilogue = [&](const floatx16 (&prev)[4], int klast) {
        const int tile = tile_lo + sigma + NS * klast;
        const bool ok = klast >= 0 && tile < tile_lo + ntiles && beam < bend;
        if (PR == PR_VOLT) volt_store_cm(prev, ors, T, beam, tile * kTile, h, ok);
        else stokes_store_cm<PR, TI>(prev, ors, d.ld_row, T2, beam, tile * kTile, h, ok);
    };

    load_chunks(0);
#pragma unroll
    for (int i = 0; i < CPT; ++i) store_chunk(0, i);
    __syncthreads();
    if (!PIPE) {
        // one accumulator set (the loaders' registers leave no room for a
        // second): MFMAs, then the epilogue.
        // The samples of step j sit in rr[j % 2], loaded two steps ahead.
        floatx16 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = zero16();
        u32x4 rr[2][CPT];
        load_chunks_to(1, rr[1]);
        // waves 4-7 (the second wave of each SIMD) run a tile's epilogue at
        // the start of the next step, so that on every SIMD one wave's
        // epilogue (VALU) meets the other wave's MFMAs
        const bool late = wave >= 4;
        auto plain_step = [&](int k, u32x4 (&mine)[CPT], u32x4 (&next)[CPT]) {
            load_chunks_to(k + 2, mine);                       // mine held step k's samples, now in LDS
            if (idle) {
                if (INC && inc_on) {
                    inc_finish(k - 1);
                    inc_partial(k);
                }
#pragma unroll
                for (int i = 0; i < CPT; ++i) store_chunk_from(k + 1, i, next);
                __syncthreads();
                return;
            }
            if (late) final_epilogue(acc, k - 1);
            int rowx = (sigma * 2 + (k & 1)) * kATileWords + 2 * trow * kARow;
            __asm__ volatile("" : "+v"(rowx));
            const uint32_t* ax0 = at + rowx;
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
                const int off = 4 * ((2 * kk + h) ^ sw);
                const V a = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(ax0 + off));
                const V b = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(ax0 + kARow + off));
                const V br = __builtin_bit_cast(V, wr[kk]), bi = __builtin_bit_cast(V, wi[kk]);
                acc[0] = MfmaH<CT>::mfma(a, br, kk == 0 ? zero16() : acc[0]);
                acc[1] = MfmaH<CT>::mfma(a, bi, kk == 0 ? zero16() : acc[1]);
                acc[2] = MfmaH<CT>::mfma(b, br, kk == 0 ? zero16() : acc[2]);
                acc[3] = MfmaH<CT>::mfma(b, bi, kk == 0 ? zero16() : acc[3]);
            }
            if (INC && inc_on) {
                inc_finish(k - 1);
                inc_partial(k);
            }
            if (!late) final_epilogue(acc, k);
#pragma unroll
            for (int i = 0; i < CPT; ++i) store_chunk_from(k + 1, i, next);
            __syncthreads();
        };
        int k = 0;
        for (; k + 1 < nsteps; k += 2) {
            plain_step(k, rr[0], rr[1]);
            plain_step(k + 1, rr[1], rr[0]);
        }
        if (k < nsteps) plain_step(k, rr[0], rr[1]);
        if (late && !idle) final_epilogue(acc, nsteps - 1);
        if (INC && inc_on) inc_finish(nsteps - 1);
        return;
    }
    if (idle) {
        for (int k = 0; k < nsteps; ++k) idle_step(k);
        if (INC && inc_on) inc_finish(nsteps - 1);
        return;
    }
    floatx16 acc0[4], acc1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc1[q] = zero16();
    int k = 0;
    for (; k + 1 < nsteps; k += 2) {
        step(k, acc0, acc1);
        step(k + 1, acc1, acc0);
    }
    if (k < nsteps) {
        step(k, acc0, acc1);
        final_epilogue(acc0, k);
    } else {
        final_epilogue(acc1, k - 1);
    }
    if (INC && inc_on) inc_finish(nsteps - 1);
}

// ===========================================================================
// generic workers: any station count (chunks of 64), any input type
// ===========================================================================
template <int XT, int PR>
LBF_INLINE void item_f32_generic(const BlockDesc& d, int item, int nbg, float* wl) {
    typedef Raw<XT> R;
    const int g = item / nbg, bg = item % nbg;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int S = d.S, C = d.C, T = d.T;
    const int b0 = bg * kBeamGroup;
    const int nchunk = (S + kStationChunk - 1) / kStationChunk;
    const int f_int = PR == PR_VOLT ? 1 : d.f_int;
    EpiCtx e = make_epi(d, PR, g);
    const int tpg = e.t_int >= 32 ? e.t_int / 32 : 1;
    const int ntiles = (T + kTile - 1) / kTile;
    const int ngroups = (ntiles + tpg - 1) / tpg;
    const int trow = tile_row_sample(r);
    const size_t stride = (size_t)C * T;
    const int nw = blockDim.x / kWave;          // waves sharing the groups

    for (int j = 0; j < f_int; ++j) {
        const int c = g * f_int + j;
        e.c = c;
        e.first = j == 0;
        for (int grp0 = 0; grp0 < ngroups; grp0 += nw) {
            const int grp = grp0 + wave;
            const bool active = grp < ngroups;
            float gs[kBeamTiles][4];
#pragma unroll
            for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) gs[a][q] = 0.f;
            for (int tg = 0; tg < tpg; ++tg) {
                const int t0 = (grp * tpg + tg) * kTile;
                const int t = t0 + trow;
                const bool tok = active && t < T;
                floatx16 acc[kBeamTiles][4];
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[a][q] = zero16();
                for (int ch = 0; ch < nchunk; ++ch) {
                    const int s0 = ch * kStationChunk;
                    __syncthreads();
                    stage_weights_f32(wl, d, c, b0, s0);
                    __syncthreads();
                    if (!active) continue;
                    const int ns = min(kStationChunk, S - s0);
                    const size_t idx = ((size_t)s0 * C + c) * T + (tok ? t : 0);
                    for (int sl = 0; sl < ns; ++sl) {
                        const floatx4 v = tok ? R::cvt(R::load(d.x, idx + (size_t)sl * stride)) : R::cvt(R::zero());
                        const float aXr = h ? -v[1] : v[0];
                        const float aXi = h ? v[0] : v[1];
                        const float aYr = h ? -v[3] : v[2];
                        const float aYi = h ? v[2] : v[3];
                        const float* wrow = wl + (sl * 2 + h) * kBeamGroup + r;
#pragma unroll
                        for (int a = 0; a < kBeamTiles; ++a) {
                            const float bw = wrow[a * kTile];
                            acc[a][0] = mfma_f32(aXr, bw, acc[a][0]);
                            acc[a][1] = mfma_f32(aXi, bw, acc[a][1]);
                            acc[a][2] = mfma_f32(aYr, bw, acc[a][2]);
                            acc[a][3] = mfma_f32(aYi, bw, acc[a][3]);
                        }
                    }
                }
                if (!active) continue;
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a) {
                    const int beam = b0 + a * kTile + r;
                    if (PR == PR_VOLT || e.t_int < 32) epilogue_tile<PR>(acc[a], e, beam, t0, h);
                    else accumulate_tile_sums<PR>(acc[a], gs[a]);
                }
            }
            if (PR != PR_VOLT && e.t_int >= 32 && active) {
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a) store_group_sums<PR>(gs[a], e, b0 + a * kTile + r, grp, h);
            }
        }
    }
}

template <int XT, int CT, int PR>
LBF_INLINE void item_h_generic(const BlockDesc& d, int item, int nbg, uint32_t* wh) {
    typedef Raw<XT> R;
    typedef typename MfmaH<CT>::vec V;
    const int g = item / nbg, bg = item % nbg;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int S = d.S, C = d.C, T = d.T;
    const int b0 = bg * kBeamGroup;
    const int nchunk = (S + kStationChunk - 1) / kStationChunk;
    const int f_int = PR == PR_VOLT ? 1 : d.f_int;
    EpiCtx e = make_epi(d, PR, g);
    const int tpg = e.t_int >= 32 ? e.t_int / 32 : 1;
    const int ntiles = (T + kTile - 1) / kTile;
    const int ngroups = (ntiles + tpg - 1) / tpg;
    const int trow = tile_row_sample(r);
    const size_t stride = (size_t)C * T;
    const int nw = blockDim.x / kWave;          // waves sharing the groups

    for (int j = 0; j < f_int; ++j) {
        const int c = g * f_int + j;
        e.c = c;
        e.first = j == 0;
        for (int grp0 = 0; grp0 < ngroups; grp0 += nw) {
            const int grp = grp0 + wave;
            const bool active = grp < ngroups;
            float gs[kBeamTiles][4];
#pragma unroll
            for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) gs[a][q] = 0.f;
            for (int tg = 0; tg < tpg; ++tg) {
                const int t0 = (grp * tpg + tg) * kTile;
                const int t = t0 + trow;
                const bool tok = active && t < T;
                floatx16 acc[kBeamTiles][4];
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[a][q] = zero16();
                for (int ch = 0; ch < nchunk; ++ch) {
                    const int s0 = ch * kStationChunk;
                    __syncthreads();
                    stage_weights_h(wh, d, c, b0, s0);
                    __syncthreads();
                    if (!active) continue;
                    const int ns = min(kStationChunk, S - s0);
                    const int nk = (ns + 7) / 8;
                    const size_t idx0 = ((size_t)s0 * C + c) * T + (tok ? t : 0);
                    for (int kk = 0; kk < nk; ++kk) {
                        APair p[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int sl = 8 * kk + 4 * h + i;
                            const typename R::type v = (tok && sl < ns) ? R::load(d.x, idx0 + (size_t)sl * stride)
                                                                        : R::zero();
                            p[i] = Conv<XT, CT>::frag(v);
                        }
                        const u32x4 uxr = {p[0].xr, p[1].xr, p[2].xr, p[3].xr};
                        const u32x4 uxi = {p[0].xi, p[1].xi, p[2].xi, p[3].xi};
                        const u32x4 uyr = {p[0].yr, p[1].yr, p[2].yr, p[3].yr};
                        const u32x4 uyi = {p[0].yi, p[1].yi, p[2].yi, p[3].yi};
                        const V axr = __builtin_bit_cast(V, uxr), axi = __builtin_bit_cast(V, uxi);
                        const V ayr = __builtin_bit_cast(V, uyr), ayi = __builtin_bit_cast(V, uyi);
                        const uint32_t* wrow = wh + r * kWRow + 8 * kk + 4 * h;
#pragma unroll
                        for (int a = 0; a < kBeamTiles; ++a) {
                            const V bw = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(wrow + a * kTile * kWRow));
                            acc[a][0] = MfmaH<CT>::mfma(axr, bw, acc[a][0]);
                            acc[a][1] = MfmaH<CT>::mfma(axi, bw, acc[a][1]);
                            acc[a][2] = MfmaH<CT>::mfma(ayr, bw, acc[a][2]);
                            acc[a][3] = MfmaH<CT>::mfma(ayi, bw, acc[a][3]);
                        }
                    }
                }
                if (!active) continue;
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a) {
                    const int beam = b0 + a * kTile + r;
                    if (PR == PR_VOLT || e.t_int < 32) epilogue_tile<PR>(acc[a], e, beam, t0, h);
                    else accumulate_tile_sums<PR>(acc[a], gs[a]);
                }
            }
            if (PR != PR_VOLT && e.t_int >= 32 && active) {
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a) store_group_sums<PR>(gs[a], e, b0 + a * kTile + r, grp, h);
            }
        }
    }
}

}  // namespace lbf
