// bf_addr_check.cpp -- host-side walk of every buffer access the fast
// contraction workers make for a block, with the kernels' own addressing
// (bf_addr.h): each descriptor of non-zero range must lie inside its buffer,
// no 32-bit offset may wrap, and every store the epilogue means to make must fall inside its
// descriptor.  No device access.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <thread>
#include <vector>

#include "bf_common.h"

namespace lbf {

namespace {

struct Walk {
    uint64_t n = 0;
    bool bad = false;
    char msg[320] = {0};

    void fail(const char* fmt, ...) {
        if (bad) return;
        bad = true;
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(msg, sizeof(msg), fmt, ap);
        va_end(ap);
    }

    // an access of `size` bytes at 32-bit offset off32 (exact value off64) of
    // a descriptor at byte `base` of a buffer of `buf` bytes, range `range`;
    // `land`: a store the epilogue means to make (it must be in range)
    void access(const char* what, uint64_t base, uint64_t range, uint64_t off64, uint32_t off32, int size,
                uint64_t buf, bool land) {
        ++n;
        if (bad) return;
        if (range > 0xffffffffull) return fail("%s: descriptor range %llu does not fit 32 bits", what,
                                               (unsigned long long)range);
        // a descriptor of range 0 (a station group past S) is never dereferenced
        if (range > 0 && base + range > buf)
            return fail("%s: descriptor [%llu, %llu) past its buffer of %llu bytes", what, (unsigned long long)base,
                        (unsigned long long)(base + range), (unsigned long long)buf);
        if (off64 != off32)
            return fail("%s: 32-bit offset wraps (%llu != %u)", what, (unsigned long long)off64, off32);
        const bool in_range = off64 + (uint64_t)size <= range;
        if (land && !in_range)
            return fail("%s: a store meant to land at offset %llu is outside its descriptor of %llu bytes", what,
                        (unsigned long long)off64, (unsigned long long)range);
        if (!land && off32 == kNoStore && in_range) return fail("%s: the no-store offset is in range", what);
    }
};

int ti_of(const BlockDesc& d) { return d.product == PR_VOLT ? 1 : d.t_int; }

// the output descriptor of channel c and its buffer
void out_desc(const BlockDesc& d, int c, uint64_t* base, uint64_t* range, uint64_t* buf) {
    const int T2 = d.T / ti_of(d);
    const uint32_t bpc = out_channel_bytes(d, d.product, T2);
    *base = out_base(d, c, bpc);
    *range = bpc;
    *buf = (uint64_t)d.nc * bpc;
}

// Epilogue stores of one wave lane for one 32-sample tile.
void stores_of_tile(Walk& w, const BlockDesc& d, int c, int beam, int bend, int tile, int h, bool tile_ok) {
    uint64_t base, range, buf;
    out_desc(d, c, &base, &range, &buf);
    const int T = d.T;
    if (d.product == PR_VOLT) {
        for (int smp = 0; smp < 16; ++smp) {
            const int t = tile * kTile + 16 * h + smp;
            const bool ok = tile_ok && beam < bend && t < T;
            const uint32_t off = ok ? volt_off(beam, T, t) : kNoStore;
            const uint64_t o64 = ok ? ((uint64_t)beam * T + t) * 16u : kNoStore;
            w.access("voltage store", base, range, o64, off, 16, buf, ok);
        }
        return;
    }
    const int TI = ti_of(d), T2 = T / TI, K = d.product == PR_IQUV ? 4 : 1;
    for (int o = 0; o < 16 / TI; ++o) {
        const int tq = (tile * kTile + 16 * h) / TI + o;
        const bool ok = tile_ok && beam < bend && tq < T2;
        const uint32_t off = ok ? stokes_off(tq, d.ld_row, beam, K) : kNoStore;
        const uint64_t o64 = ok ? ((uint64_t)tq * d.ld_row + (uint64_t)beam * K) * 4u : kNoStore;
        w.access("Stokes store", base, range, o64, off, 4 * K, buf, ok);
    }
}

// items [lo, hi) of the FP16/BF16 worker
void walk_h(Walk& w, const BlockDesc& d, int lo, int hi) {
    const int bytes = sample_bytes(d.xtype);
    const uint64_t xbuf = (uint64_t)d.S * d.C * d.T * bytes, wbuf = (uint64_t)d.C * d.B * d.S * 4;
    const uint64_t stride64 = (uint64_t)d.C * d.T * bytes;
    const uint32_t stride = (uint32_t)stride64;
    if (stride != stride64) return w.fail("station stride does not fit 32 bits");
    const int NS = fast_h_streams(d), NK = fast_h_ksteps(d.S), NBT = 8 / NS;
    const int SPC = 16 / bytes, CPS = kTile / SPC, CPTILE = 8 * NK * CPS;
    const int CPT = (NS * CPTILE + kThreadsH - 1) / kThreadsH;
    int nbg;
    const int items = block_items_fast_h(d, &nbg);
    for (int item = lo; item < std::min(hi, items) && !w.bad; ++item) {
        const ItemPos ip = item_pos(d, item, nbg);
        const int nsteps = (ip.ntiles + NS - 1) / NS;
        for (int tid = 0; tid < kThreadsH; ++tid) {
            const int lane = tid & 63, wave = tid / 64, r = lane & 31, h = lane >> 5;
            const int bt = wave % NBT, sigma = wave / NBT;
            const int beam = d.b0 + (ip.bg * NBT + bt) * kTile + r;
            for (int kk = 0; kk < NK; ++kk)
                w.access("weight load", weight_base(d, ip.c, 4), weight_range(d, 4),
                         ((uint64_t)beam * d.S + 8 * kk + 4 * h) * 4u, weight_off(beam, d.S, 8 * kk + 4 * h, 4), 16,
                         wbuf, false);
            // the loaders run up to two steps ahead of the last one
            for (int k = 0; k < nsteps + 2; ++k)
                for (int i = 0; i < CPT; ++i) {
                    const Chunk16 ch = h_chunk(tid + kThreadsH * i, k, NS, CPTILE, CPS, ip.tile_lo, ip.ntiles);
                    const int s0 = ch.s & ~7, t = ch.tile * kTile + ch.q * SPC;
                    const uint64_t o64 = (uint64_t)(ch.s & 7) * stride64 + ((uint64_t)ip.c * d.T + t) * bytes;
                    w.access("sample load", group_base(s0, stride), group_range(s0, d.S, stride), o64,
                             sample_off(ch.s & 7, stride, ip.c, d.T, t, bytes), 16, xbuf, false);
                }
            for (int k = 0; k < nsteps; ++k) {
                const int tile = ip.tile_lo + sigma + NS * k;
                stores_of_tile(w, d, ip.c, beam, d.b1, tile, h, tile < ip.tile_lo + ip.ntiles);
            }
        }
    }
}

// items [lo, hi) of the FP32 worker
void walk_f32(Walk& w, const BlockDesc& d, int lo, int hi) {
    const int bytes = sample_bytes(d.xtype);
    const uint64_t xbuf = (uint64_t)d.S * d.C * d.T * bytes, wbuf = (uint64_t)d.C * d.B * d.S * 8;
    const uint64_t stride64 = (uint64_t)d.C * d.T * bytes;
    const uint32_t stride = (uint32_t)stride64;
    if (stride != stride64) return w.fail("station stride does not fit 32 bits");
    const int ngrp = std::min(8, ((d.S + 7) / 8 + 1) & ~1);
    int nbg;
    const int items = block_items_fast_f32(d, &nbg);
    for (int item = lo; item < std::min(hi, items) && !w.bad; ++item) {
        const ItemPos ip = item_pos(d, item, nbg);
        const int b0 = ip.bg * kBeamGroup;
        for (int tid = 0; tid < kThreadsH; ++tid) {        // weight planes: beam b0 + tid/64 + 8k, station tid % 64
            for (int k = 0; k < kStationChunk * kBeamGroup / kThreadsH; ++k) {
                const int beam = b0 + tid / kStationChunk + (kThreadsH / kStationChunk) * k, sl = tid % kStationChunk;
                w.access("weight load", weight_base(d, ip.c, 8), weight_range(d, 8), ((uint64_t)beam * d.S + sl) * 8u,
                         weight_off(beam, d.S, sl, 8), 8, wbuf, false);
            }
        }
        for (int wave = 0; wave < 8; ++wave) {
            const int bt = wave & 3, ts = wave >> 2;
            const int nmine = ip.ntiles > ts ? (ip.ntiles - ts + 1) / 2 : 0;
            if (nmine == 0 || b0 + bt * kTile >= d.B) continue;
            for (int lane = 0; lane < 64; ++lane) {
                const int r = lane & 31, h = lane >> 5, trow = tile_row_sample(r);
                const int beam = b0 + bt * kTile + r;
                // the ring is refilled two groups ahead of the last one used
                for (int n = 0; n < nmine * ngrp + 2; ++n) {
                    const int k = std::min(n / ngrp, nmine - 1), g = n % ngrp;
                    const int t = std::min((ip.tile_lo + ts + 2 * k) * kTile + trow, d.T - 1);
                    for (int i = 0; i < 8; ++i)
                        w.access("sample load", group_base(8 * g, stride), group_range(8 * g, d.S, stride),
                                 (uint64_t)i * stride64 + ((uint64_t)ip.c * d.T + t) * bytes,
                                 sample_off(i, stride, ip.c, d.T, t, bytes), bytes, xbuf, false);
                }
                for (int k = 0; k < nmine; ++k)
                    stores_of_tile(w, d, ip.c, beam, d.B, ip.tile_lo + ts + 2 * k, h, true);
            }
        }
    }
}

}  // namespace

// Walk the fast workers' accesses of block d (as launched: channel range,
// output order, beam parts).  Returns false with a message on the first
// access that breaks a rule.
// The items are walked by `threads` host threads.
bool check_fast_addressing(const BlockDesc& d, int threads, uint64_t* accesses, char* msg, size_t msglen) {
    BlockDesc part[2];
    int np = 1, items[2];
    part[0] = d;
    if (d.ctype != CT_F32) np = split_fast_h(d, part);
    for (int p = 0; p < np; ++p) {
        int nbg;
        items[p] = d.ctype == CT_F32 ? block_items_fast_f32(part[p], &nbg) : block_items_fast_h(part[p], &nbg);
    }
    threads = std::max(1, std::min(threads, 64));
    std::vector<Walk> w(threads * np);
    std::vector<std::thread> th;
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < threads; ++i) {
            const int lo = (int)((long long)items[p] * i / threads), hi = (int)((long long)items[p] * (i + 1) / threads);
            Walk* wk = &w[p * threads + i];
            const BlockDesc* dp = &part[p];
            th.emplace_back([=] {
                if (dp->ctype == CT_F32) walk_f32(*wk, *dp, lo, hi);
                else walk_h(*wk, *dp, lo, hi);
            });
        }
    for (std::thread& t : th) t.join();
    uint64_t n = 0;
    const Walk* first_bad = nullptr;
    for (const Walk& wk : w) {
        n += wk.n;
        if (wk.bad && !first_bad) first_bad = &wk;
    }
    if (accesses) *accesses = n;
    if (first_bad && msg && msglen) snprintf(msg, msglen, "%s", first_bad->msg);
    return first_bad == nullptr;
}

int check_block_addressing(const BlockDesc& d0, bool channel_major, size_t cap, int threads, uint64_t* accesses,
                           char* msg, size_t msglen) {
    if (accesses) *accesses = 0;
    if (!fast_path(d0) && !fast_path_fint(d0)) return 0;
    BlockDesc d = d0;
    if (channel_major) d.order = 1;
    BlockDesc passes[1];
    int nc = d.C;
    const bool staged = needs_staging(d);
    if (staged) {
        // as launch_beamform_staged: channel passes into the staging buffer
        nc = cap ? staging_chunk(d, cap) : d.C;
        if (nc < 1) return 2;
    }
    uint64_t total = 0;
    for (int c0 = 0; c0 < d.C; c0 += nc) {
        passes[0] = d;
        if (staged) {
            passes[0].order = 1;
            passes[0].ld_row = staging_ld(d.B, d.product == PR_IQUV ? 4 : 1);
            passes[0].f_int = 1;                           // channel sums follow, out of the staging
            passes[0].c0 = c0;
            passes[0].nc = d.C - c0 < nc ? d.C - c0 : nc;
        }
        uint64_t n = 0;
        char m[320];
        const bool good = check_fast_addressing(passes[0], threads, &n, m, sizeof(m));
        total += n;
        if (!good) {
            snprintf(msg, msglen, "channels [%d, %d): %s", passes[0].c0, passes[0].c0 + passes[0].nc, m);
            if (accesses) *accesses = total;
            return 1;
        }
    }
    if (accesses) *accesses = total;
    return 0;
}

}  // namespace lbf
