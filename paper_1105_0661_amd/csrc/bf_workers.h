// bf_workers.h -- the per-work-item contraction workers.
//
// Work item = (channel group of f_int channels, group of up to 128 beams).
// A work group of 4 waves stages that beam group's weights for one channel in
// LDS; each wave walks its own 32-sample tiles (groups of tiles when t_int >=
// 32), streaming station samples from HBM straight into MFMA operand registers
// (int -> f32/f16/bf16 in registers, no separate conversion pass), and ends
// each tile with the fused Stokes / integration / beam-major store epilogue.
#pragma once
#include <type_traits>

#include "bf_common.h"

namespace lbf {

// ===========================================================================
// fast workers: up to 64 stations of complex int8/int16 samples
// ===========================================================================

// FP32 operands (MFMA 32x32x2 f32: one station per step, K = re/im).
// Station samples stream through an 8-deep register ring so each load has
// 8 stations' worth of MFMAs (8 x 16 x 64 cycles) to arrive.  Rows of a
// ragged last tile read a valid sample and are never stored.
template <int XT, int PR, int TI>
LBF_INLINE void item_f32_fast(const BlockDesc& d, int item, int nbg, float* wl) {
    typedef Raw<XT> R;
    typedef typename R::type RT;
    constexpr int BYTES = sizeof(RT);
    const int g = item / nbg, bg = item % nbg;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int S = d.S, C = d.C, T = d.T;
    const int b0 = bg * kBeamGroup;
    const int f_int = 1;                             // fast path: no channel integration
    EpiCtx e = make_epi(d, PR, g);
    const WaveTiles wt = wave_tiles(wave, T, TI);
    const int trow = tile_row_sample(r);
    const int ngrp = (S + 7) / 8;                    // groups of 8 stations
    const uint32_t stride_bytes = (uint32_t)((size_t)C * T * BYTES);

    for (int j = 0; j < f_int; ++j) {
        const int c = g * f_int + j;
        e.c = c;
        e.first = j == 0;
        __syncthreads();
        stage_weights_f32_fast(wl, d, c, b0);
        __syncthreads();
        for (int k = 0; k < wt.ntw; ++k) {
            const int t0 = wt.tile(k) * kTile;
            const uint32_t toff = (uint32_t)min(t0 + trow, T - 1) * BYTES;
            int widx = h * kBeamGroup + r;                // LDS reads stay in the loop
            __asm__ volatile("" : "+v"(widx));
            const float* wcol = wl + widx;
            floatx16 acc[kBeamTiles][4];
            RT ring[8];
            __amdgpu_buffer_rsrc_t rs = station_group_rsrc(d.x, BYTES, 0, S, c, T, stride_bytes);
#pragma unroll
            for (int i = 0; i < 8; ++i) ring[i] = buffer_sample<XT>(rs, toff + (uint32_t)i * stride_bytes);
            // one group of 8 stations; the very first station starts the
            // accumulators from zero (peeled so the choice is compile-time)
            auto group8 = [&](int gi, auto first_tag) {
                constexpr bool FIRST = decltype(first_tag)::value;
                const __amdgpu_buffer_rsrc_t rn = station_group_rsrc(d.x, BYTES, 8 * gi + 8, S, c, T, stride_bytes);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int s = gi * 8 + i;
                    const floatx4 v = R::cvt(ring[i]);
                    ring[i] = buffer_sample<XT>(rn, toff + (uint32_t)i * stride_bytes);
                    const float aXr = h ? -v[1] : v[0];
                    const float aXi = h ? v[0] : v[1];
                    const float aYr = h ? -v[3] : v[2];
                    const float aYi = h ? v[2] : v[3];
                    float bw[kBeamTiles];
#pragma unroll
                    for (int a = 0; a < kBeamTiles; ++a) bw[a] = wcol[s * 2 * kBeamGroup + a * kTile];
#pragma unroll
                    for (int a = 0; a < kBeamTiles; ++a) {
                        if (FIRST && i == 0) {
                            acc[a][0] = mfma_f32(aXr, bw[a], zero16());
                            acc[a][1] = mfma_f32(aXi, bw[a], zero16());
                            acc[a][2] = mfma_f32(aYr, bw[a], zero16());
                            acc[a][3] = mfma_f32(aYi, bw[a], zero16());
                        } else {
                            acc[a][0] = mfma_f32(aXr, bw[a], acc[a][0]);
                            acc[a][1] = mfma_f32(aXi, bw[a], acc[a][1]);
                            acc[a][2] = mfma_f32(aYr, bw[a], acc[a][2]);
                            acc[a][3] = mfma_f32(aYi, bw[a], acc[a][3]);
                        }
                    }
                }
            };
            group8(0, std::true_type{});
            for (int gi = 1; gi < ngrp; ++gi) group8(gi, std::false_type{});
            epilogue_tiles_fixed<PR, TI>(acc, e, b0, r, t0, h);
        }
    }
}

// FP16/BF16 operands (MFMA 32x32x16: 8 stations per step).  NK = K-steps
// (8-station groups) covering the stations.  A work item is one channel and
// a super-group of up to 512 beams: the 4 waves split into BW beam groups of
// 128 beams (weights of all of them in LDS) times 4/BW sample streams, so a
// channel's samples are read once and the XCD-aware item order puts 32
// adjacent channels -- one full 128-byte line of the beam-major output -- on
// each XCD at a time.  Lane half h takes stations 8kk + 4h + i of K-step kk.
template <int XT, int CT, int PR, int TI, int NK>
LBF_INLINE void item_h_fast(const BlockDesc& d, int item, int nsg, uint32_t* wh) {
    typedef Raw<XT> R;
    typedef typename R::type RT;
    typedef typename MfmaH<CT>::vec V;
    constexpr int BYTES = sizeof(RT);
    const int c = item / nsg, sg = item % nsg;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r = lane & 31, h = lane >> 5;
    const int S = d.S, T = d.T;
    const int bsg0 = sg * kSuperGroup;
    const int nb = min(kSuperGroup, d.B - bsg0);
    const int BW = nb <= kBeamGroup ? 1 : (nb <= 2 * kBeamGroup ? 2 : 4);
    const int TW = kWavesPerGroup / BW;
    const int bw = wave % BW, tw = wave / BW;
    const int b0 = bsg0 + bw * kBeamGroup;
    EpiCtx e = make_epi(d, PR, c);
    e.c = c;
    e.first = 1;
    const int ntiles = (T + kTile - 1) / kTile;
    const int ntw = ntiles > tw ? (ntiles - tw + TW - 1) / TW : 0;
    const int trow = tile_row_sample(r);
    const uint32_t stride_bytes = (uint32_t)((size_t)d.C * T * BYTES);
    const uint32_t hoff = (uint32_t)h * 4u * stride_bytes;
    const int wbase = bw * kBeamGroup * kWRow;

    for (int g = 0; g < BW; ++g) stage_weights_h_fast(wh + g * kBeamGroup * kWRow, d, c, bsg0 + g * kBeamGroup);
    __syncthreads();
    {
        // Rolling prefetch: slot kk holds K-step kk of the current tile until
        // it is converted, then is refilled with K-step kk of the next tile,
        // so every load has a whole tile of MFMAs to arrive.
        RT buf[NK][4];
        auto load_step = [&](int tile, int kk) {
            const uint32_t off = hoff + (uint32_t)min(tile * kTile + trow, T - 1) * BYTES;
            const __amdgpu_buffer_rsrc_t rs = station_group_rsrc(d.x, BYTES, 8 * kk, S, c, T, stride_bytes);
#pragma unroll
            for (int i = 0; i < 4; ++i) buf[kk][i] = buffer_sample<XT>(rs, off + (uint32_t)i * stride_bytes);
        };
        if (ntw > 0) {
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) load_step(tw, kk);
        }
        for (int k = 0; k < ntw; ++k) {
            const int t0 = (tw + TW * k) * kTile;
            const int tnext = tw + TW * (k + 1 < ntw ? k + 1 : k);
            // read the weight fragments from LDS inside the tile loop: kept
            // live across tiles they would take 128 VGPRs
            int widx = wbase + r * kWRow + 4 * h;
            __asm__ volatile("" : "+v"(widx));
            const uint32_t* wrow = wh + widx;
            floatx16 acc[kBeamTiles][4];
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
                APair p[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) p[i] = Conv<XT, CT>::frag(buf[kk][i]);
                load_step(tnext, kk);
                const u32x4 uxr = {p[0].xr, p[1].xr, p[2].xr, p[3].xr};
                const u32x4 uxi = {p[0].xi, p[1].xi, p[2].xi, p[3].xi};
                const u32x4 uyr = {p[0].yr, p[1].yr, p[2].yr, p[3].yr};
                const u32x4 uyi = {p[0].yi, p[1].yi, p[2].yi, p[3].yi};
                const V axr = __builtin_bit_cast(V, uxr), axi = __builtin_bit_cast(V, uxi);
                const V ayr = __builtin_bit_cast(V, uyr), ayi = __builtin_bit_cast(V, uyi);
                V bfr[kBeamTiles];
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a)
                    bfr[a] = __builtin_bit_cast(V, *reinterpret_cast<const u32x4*>(wrow + a * kTile * kWRow + 8 * kk));
#pragma unroll
                for (int a = 0; a < kBeamTiles; ++a) {
                    acc[a][0] = MfmaH<CT>::mfma(axr, bfr[a], kk == 0 ? zero16() : acc[a][0]);
                    acc[a][1] = MfmaH<CT>::mfma(axi, bfr[a], kk == 0 ? zero16() : acc[a][1]);
                    acc[a][2] = MfmaH<CT>::mfma(ayr, bfr[a], kk == 0 ? zero16() : acc[a][2]);
                    acc[a][3] = MfmaH<CT>::mfma(ayi, bfr[a], kk == 0 ? zero16() : acc[a][3]);
                }
            }
            epilogue_tiles_fixed<PR, TI>(acc, e, b0, r, t0, h);
        }
    }
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

    for (int j = 0; j < f_int; ++j) {
        const int c = g * f_int + j;
        e.c = c;
        e.first = j == 0;
        for (int grp0 = 0; grp0 < ngroups; grp0 += kWavesPerGroup) {
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

    for (int j = 0; j < f_int; ++j) {
        const int c = g * f_int + j;
        e.c = c;
        e.first = j == 0;
        for (int grp0 = 0; grp0 < ngroups; grp0 += kWavesPerGroup) {
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
