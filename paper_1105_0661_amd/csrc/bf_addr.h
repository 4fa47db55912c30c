// bf_addr.h -- the buffer addressing of the fast contraction workers as plain
// integer arithmetic, shared by the kernels and by a host-side walk
// (bf_addr_check.cpp) that checks every access of a block against its
// buffers before anything runs on a device.
//
// The workers address HBM through buffer descriptors: a base address, a range
// in bytes (accesses at or beyond it read zeros or store nothing) and 32-bit
// byte offsets.  What must hold: every descriptor lies inside its buffer, and
// no 32-bit offset wraps.  fast_path() bounds the sizes so that the offsets
// below stay under 2^31.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbf_device.h"

#define LBF_HD __host__ __device__ inline

namespace lbf {

// Work items cut a block's samples into segments of kSegTiles 32-sample
// tiles, or of 2, 4 or 8 times as many while the block keeps at least
// kMinItems items that way: a longer item spreads its prologue (weights into
// registers, the first loads) and its last step over more steps, and enough
// items remain to keep every compute unit busy to the end.
constexpr int kSegTiles = 24, kSegTilesMax = 192, kMinItems = 2048;

LBF_HD int seg_tiles(const BlockDesc& d, int nbg) {
    const int ntiles = (d.T + kTile - 1) / kTile;
    int seg = kSegTiles;
    while (seg < kSegTilesMax && seg < ntiles &&
           (int64_t)d.nc * nbg * ((ntiles + 2 * seg - 1) / (2 * seg)) >= kMinItems)
        seg *= 2;
    return seg;
}

// "no store": an offset past every output descriptor, which the hardware
// drops.  2^31, not 2^32 - 1: the range check adds the access size to the
// offset, and the latter would wrap around to an in-range value.
constexpr uint32_t kNoStore = 0x80000000u;

// A work item of the fast workers: channel c (of [c0, c0 + nc)), beam group
// bg, sample tiles [tile_lo, tile_lo + ntiles) (nbg beam groups).
struct ItemPos {
    int c, bg, tile_lo, ntiles;
};

LBF_HD ItemPos item_pos(const BlockDesc& d, int item, int nbg) {
    const int ntiles_all = (d.T + kTile - 1) / kTile;
    const int seg = seg_tiles(d, nbg);
    const int nseg = (ntiles_all + seg - 1) / seg;
    ItemPos p;
    p.c = d.c0 + item / nseg / nbg;
    p.bg = item / nseg % nbg;
    p.tile_lo = item % nseg * seg;
    const int left = ntiles_all - p.tile_lo;
    p.ntiles = left < seg ? left : seg;
    return p;
}

// Station samples x[s][c][t] (sample_bytes each, station planes stride_bytes
// = C T sample_bytes apart).  A descriptor covers the whole planes of the
// valid stations of one group of 8, [s0, min(s0 + 8, S)); the channel and
// time go into the offset, so a ragged last tile reads past its channel into
// the next one (rows the epilogue never stores) but never past the array.
LBF_HD uint64_t group_base(int s0, uint32_t stride_bytes) { return (uint64_t)s0 * stride_bytes; }

LBF_HD uint32_t group_range(int s0, int S, uint32_t stride_bytes) {
    int n = S - s0;
    n = n < 0 ? 0 : (n > 8 ? 8 : n);
    return (uint32_t)n * stride_bytes;
}

// station s0 + i of a group, channel c, sample t
LBF_HD uint32_t sample_off(int i, uint32_t stride_bytes, int c, int T, int t, int bytes) {
    return (uint32_t)i * stride_bytes + (uint32_t)(c * T + t) * (uint32_t)bytes;
}

// Weights w[c][b][s] (bytes per complex weight): one descriptor per channel.
LBF_HD uint64_t weight_base(const BlockDesc& d, int c, int bytes) { return (uint64_t)c * d.B * d.S * bytes; }
LBF_HD uint32_t weight_range(const BlockDesc& d, int bytes) { return (uint32_t)d.B * (uint32_t)d.S * (uint32_t)bytes; }
LBF_HD uint32_t weight_off(int beam, int S, int s, int bytes) { return ((uint32_t)beam * S + s) * (uint32_t)bytes; }

// The FP16/BF16 worker's sample loaders: chunk j (thread tid + 512 i) of step
// k covers stream sg, station s and samples SPC q .. SPC q + SPC - 1 of tile
// `tile` (the stream's tile of that step, or its last tile once it has run
// out).  Chunks past the step's ns tiles (a step of fewer chunks than
// threads) load the tiles of a later step (in range, clamped to the item's
// last tile), which warms the cache for that step, and are not staged.
// (Skipping their loads, with an out-of-range offset, costs registers that
// the two headline shapes do not have.)
struct Chunk16 {
    int s, q, tile;
};

LBF_HD Chunk16 h_chunk(int j, int k, int ns, int cptile, int cps, int tile_lo, int ntiles) {
    const int sg = j / cptile, jt = j % cptile;
    Chunk16 ch;
    ch.s = jt / cps;
    ch.q = jt % cps;
    const int i = sg + ns * k;
    ch.tile = tile_lo + (i < ntiles - 1 ? i : ntiles - 1);
    return ch;
}

// Output of one channel (order 1 staging, or voltages): one descriptor per
// channel of the item's block, output index c - c0.
LBF_HD uint32_t out_channel_bytes(const BlockDesc& d, int product, int T2) {
    return product == PR_VOLT ? (uint32_t)d.B * d.T * 16u : (uint32_t)T2 * d.ld_row * 4u;
}

LBF_HD uint64_t out_base(const BlockDesc& d, int c, uint32_t channel_bytes) {
    return (uint64_t)(c - d.c0) * channel_bytes;
}

// voltages y[b][t][p] of the channel, 16 bytes per sample
LBF_HD uint32_t volt_off(int beam, int T, int t) { return ((uint32_t)beam * T + t) * 16u; }

// Stokes s[t'][b][k] of the channel, rows of ld floats: 16 bytes (IQUV) or 4 (I)
LBF_HD uint32_t stokes_off(int tq, int ld, int beam, int K) {
    return ((uint32_t)tq * (uint32_t)ld + (uint32_t)beam * (uint32_t)K) * 4u;
}

}  // namespace lbf
