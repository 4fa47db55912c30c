// abi.cpp -- the extern "C" entry points of liblbf: argument validation,
// error reporting and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbf.h"
#include "lbf_internal.h"
#include "lbf_launch.h"

static_assert(LBF_MAX_BATCH == lbf::kMaxBatch, "batch bound mismatch");

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(LBF_E_HIP, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

int ok() {
    return LBF_OK;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int bytes_per_complex(int xtype) { return xtype == LBF_CI8 ? 2 : xtype == LBF_CI16 ? 4 : 8; }
int weight_bytes(int ctype) { return ctype == LBF_F32 ? 8 : 4; }

// Validate a block; `where` names the entry point in the error text.
int check_block(const lbf_block* b, const char* where) {
    if (!b) return fail(LBF_E_INVAL, "%s: block is NULL", where);
    if (b->S < 1 || b->C < 1 || b->T < 1 || b->B < 1)
        return fail(LBF_E_INVAL, "%s: sizes must be >= 1 (S=%d C=%d T=%d B=%d)", where, b->S, b->C, b->T, b->B);
    if (!b->d_x || !b->d_w || !b->d_out) return fail(LBF_E_INVAL, "%s: NULL device pointer", where);
    if (b->xtype < LBF_CI8 || b->xtype > LBF_CF32) return fail(LBF_E_INVAL, "%s: unknown xtype %d", where, b->xtype);
    if (b->ctype < LBF_F32 || b->ctype > LBF_BF16) return fail(LBF_E_INVAL, "%s: unknown ctype %d", where, b->ctype);
    if (b->product != LBF_VOLTAGES && b->product != LBF_STOKES_I && b->product != LBF_STOKES_IQUV)
        return fail(LBF_E_INVAL, "%s: unknown product %d", where, b->product);
    if (b->t_int < 1 || b->f_int < 1)
        return fail(LBF_E_INVAL, "%s: t_int and f_int must be >= 1 (%d, %d)", where, b->t_int, b->f_int);
    if (b->product == LBF_VOLTAGES) {
        if (b->t_int != 1 || b->f_int != 1)
            return fail(LBF_E_INVAL, "%s: voltages take t_int = f_int = 1", where);
    } else {
        if (b->T % b->t_int) return fail(LBF_E_INVAL, "%s: T=%d not a multiple of t_int=%d", where, b->T, b->t_int);
        if (b->C % b->f_int) return fail(LBF_E_INVAL, "%s: C=%d not a multiple of f_int=%d", where, b->C, b->f_int);
        if (!is_pow2(b->t_int))
            return fail(LBF_E_UNSUPPORTED, "%s: fused Stokes needs a power-of-two t_int (got %d); "
                        "use VOLTAGES + lbf_stokes", where, b->t_int);
    }
    if ((long long)b->C * b->T > (1LL << 40) || (long long)b->B * b->S > (1LL << 31))
        return fail(LBF_E_INVAL, "%s: block too large", where);
    return LBF_OK;
}

lbf::BlockDesc to_desc(const lbf_block* b) {
    lbf::BlockDesc d;
    d.x = b->d_x;
    d.w = b->d_w;
    d.out = b->d_out;
    d.S = b->S; d.C = b->C; d.T = b->T; d.B = b->B;
    d.xtype = b->xtype; d.ctype = b->ctype; d.product = b->product;
    d.t_int = b->product == LBF_VOLTAGES ? 1 : b->t_int;
    d.f_int = b->product == LBF_VOLTAGES ? 1 : b->f_int;
    d.order = 0;
    d.b0 = 0;
    d.b1 = b->B;
    d.ld_row = b->B * (b->product == LBF_STOKES_IQUV ? 4 : 1);
    d.c0 = 0;
    d.nc = b->C;
    d.inc = nullptr;
    d.ns_force = lbf::g_tile_streams_override.load(std::memory_order_relaxed);
    return d;
}

// Work counters of the persistent batch kernel: a ring of slots per device so
// that batches queued on different streams do not share a counter (a slot
// comes round again after kCounterSlots calls; the header states that limit).
constexpr int kCounterSlots = 1024;
std::mutex g_counter_mu;
int* g_counters[64] = {nullptr};
unsigned g_counter_next[64] = {0};

int counter_slot(int** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "lbf_beamform_batch");
    if (dev < 0 || dev >= 64) return fail(LBF_E_UNSUPPORTED, "lbf_beamform_batch: device %d", dev);
    std::lock_guard<std::mutex> lk(g_counter_mu);
    if (!g_counters[dev]) {
        e = hipMalloc((void**)&g_counters[dev], sizeof(int) * kCounterSlots);
        if (e != hipSuccess) return hip_fail(e, "lbf_beamform_batch: counter allocation");
    }
    *out = g_counters[dev] + (g_counter_next[dev]++ % kCounterSlots);
    return LBF_OK;
}

}  // namespace

size_t lbf::block_staging_channel_bytes(const lbf_block* b) {
    const lbf::BlockDesc d = to_desc(b);
    return lbf::needs_staging(d) ? lbf::staging_channel_bytes(d) : 0;
}

int lbf::run_block(const lbf_block* blk, void* stage, size_t cap, void* stream, const char* where) {
    int rc = check_block(blk, where);
    if (rc) return rc;
    const lbf::BlockDesc d = to_desc(blk);
    if (stage != nullptr && lbf::needs_staging(d) && lbf::staging_chunk(d, cap) < 1)
        return fail(LBF_E_NOMEM, "%s: staging of %zu bytes holds less than one channel (%zu bytes)", where, cap,
                    lbf::staging_channel_bytes(d));
    hipError_t e = stage ? lbf::launch_beamform_staged(d, stage, cap, (hipStream_t)stream)
                         : lbf::launch_beamform(d, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, where);
    return ok();
}

int lbf::run_batch(const lbf_block* blks, int n, void* const* stage, const size_t* cap, void* stream,
                   const char* where) {
    if (!blks) return fail(LBF_E_INVAL, "%s: blocks is NULL", where);
    if (n < 1 || n > LBF_MAX_BATCH) return fail(LBF_E_INVAL, "%s: n=%d outside 1..%d", where, n, LBF_MAX_BATCH);
    lbf::BlockDesc d[lbf::kMaxBatch];
    for (int i = 0; i < n; ++i) {
        int rc = check_block(&blks[i], where);
        if (rc) return rc;
        if (blks[i].product == LBF_VOLTAGES)
            return fail(LBF_E_UNSUPPORTED, "%s: block %d: batches take Stokes products", where, i);
        if (blks[i].ctype == LBF_F32)
            return fail(LBF_E_UNSUPPORTED, "%s: block %d: batches take F16 or BF16 operands", where, i);
        if (blks[i].ctype != blks[0].ctype)
            return fail(LBF_E_UNSUPPORTED, "%s: all blocks of a batch share one ctype", where);
        d[i] = to_desc(&blks[i]);
        if (stage != nullptr && lbf::needs_staging(d[i]) &&
            (stage[i] == nullptr || lbf::staging_chunk(d[i], cap[i]) < 1))
            return fail(LBF_E_NOMEM, "%s: block %d: staging holds less than one channel", where, i);
    }
    int* counter = nullptr;
    int rc = counter_slot(&counter);
    if (rc) return rc;
    hipError_t e = lbf::launch_beamform_batch(d, n, counter, stage, cap, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, where);
    return ok();
}

std::atomic<int> lbf::g_tile_streams_override{0};

int lbf::set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" {

const char* lbf_last_error(void) { return g_err.c_str(); }

const char* lbf_version(void) { return "lbf 1.0 gfx950"; }

int lbf_compute_weights(const double* d_station_xyz, int S, const double* d_beam_dir, int B, const double* ref_dir,
                        const double* d_station_delay, const double* d_freq_hz, int C, int wtype, void* d_w,
                        double* d_tau, void* stream) {
    if (S < 1 || B < 1 || C < 1)
        return fail(LBF_E_INVAL, "lbf_compute_weights: sizes must be >= 1 (S=%d B=%d C=%d)", S, B, C);
    if (!d_station_xyz || !d_beam_dir || !d_freq_hz || !d_w)
        return fail(LBF_E_INVAL, "lbf_compute_weights: NULL device pointer");
    if (wtype < LBF_F32 || wtype > LBF_BF16) return fail(LBF_E_INVAL, "lbf_compute_weights: unknown wtype %d", wtype);
    if ((long long)B * S > (1LL << 30) || C > 65535 * 32)
        return fail(LBF_E_INVAL, "lbf_compute_weights: too large (B*S=%lld, C=%d)", (long long)B * S, C);
    const double rx = ref_dir ? ref_dir[0] : 0.0, ry = ref_dir ? ref_dir[1] : 0.0, rz = ref_dir ? ref_dir[2] : 0.0;
    hipError_t e = lbf::launch_weights(d_station_xyz, S, d_beam_dir, B, rx, ry, rz, d_station_delay, d_freq_hz, C,
                                       wtype, d_w, d_tau, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_compute_weights");
    return ok();
}

int lbf_beamform(const lbf_block* blk, void* stream) {
    return lbf::run_block(blk, nullptr, 0, stream, "lbf_beamform");
}

int lbf_beamform_incoherent(const lbf_block* blk, float* d_inc, void* stream) {
    int rc = check_block(blk, "lbf_beamform_incoherent");
    if (rc) return rc;
    if (blk->product == LBF_VOLTAGES)
        return fail(LBF_E_INVAL, "lbf_beamform_incoherent: the incoherent beam comes with a Stokes product");
    if (!d_inc) return fail(LBF_E_INVAL, "lbf_beamform_incoherent: NULL device pointer");
    const size_t inc_bytes = (size_t)blk->product * (blk->T / blk->t_int) * (blk->C / blk->f_int) * sizeof(float);
    const size_t out_bytes = (size_t)blk->B * inc_bytes;
    const size_t x_bytes = (size_t)blk->S * blk->C * blk->T * 2 * bytes_per_complex(blk->xtype);
    const char* ic = (const char*)d_inc;
    const char* o = (const char*)blk->d_out;
    const char* x = (const char*)blk->d_x;
    if ((ic < o + out_bytes && o < ic + inc_bytes) || (ic < x + x_bytes && x < ic + inc_bytes))
        return fail(LBF_E_INVAL, "lbf_beamform_incoherent: the incoherent beam overlaps the samples or the output");
    lbf::BlockDesc d = to_desc(blk);
    hipError_t e;
    if (lbf::fuses_incoherent(d)) {
        d.inc = d_inc;                                    // formed by the contraction's first beam group
        e = lbf::launch_beamform(d, (hipStream_t)stream);
    } else {
        e = lbf::launch_beamform(d, (hipStream_t)stream);
        if (e == hipSuccess)
            e = lbf::launch_incoherent(blk->d_x, blk->xtype, blk->S, blk->C, blk->T, blk->product, blk->t_int,
                                       blk->f_int, d_inc, (hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(e, "lbf_beamform_incoherent");
    return ok();
}

int lbf_beamform_noalloc(const lbf_block* blk, void* stream) {
    int rc = check_block(blk, "lbf_beamform_noalloc");
    if (rc) return rc;
    static_assert(LBF_NOALLOC_SCRATCH_BYTES == lbf::kNoAllocScratchBytes, "scratch size mismatch");
    const lbf::BlockDesc d = to_desc(blk);
    hipError_t e;
    if (lbf::needs_staging(d)) {
        const size_t per = lbf::staging_channel_bytes(d);
        if (lbf::staging_chunk(d, lbf::kNoAllocScratchBytes) < 1)
            return fail(LBF_E_NOMEM, "lbf_beamform_noalloc: the Stokes staging of one channel (%zu bytes: T' x B x K "
                        "floats, rows padded to 32), times f_int with channel integration, exceeds the %llu-byte "
                        "scratch", per, (unsigned long long)lbf::kNoAllocScratchBytes);
        void* scratch = nullptr;
        e = lbf::noalloc_scratch(&scratch);
        if (e != hipSuccess) return hip_fail(e, "lbf_beamform_noalloc: scratch address");
        e = lbf::launch_beamform_staged(d, scratch, lbf::kNoAllocScratchBytes, (hipStream_t)stream);
    } else {
        e = lbf::launch_beamform_direct(d, (hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(e, "lbf_beamform_noalloc");
    return ok();
}

int lbf_beamform_channel_major(const lbf_block* blk, void* stream) {
    int rc = check_block(blk, "lbf_beamform_channel_major");
    if (rc) return rc;
    lbf::BlockDesc d = to_desc(blk);
    d.order = 1;
    hipError_t e = lbf::launch_beamform(d, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_beamform_channel_major");
    return ok();
}

int lbf_beam_major(const float* d_in, int C2, int K, int T2, int B, float* d_out, void* stream) {
    if (C2 < 1 || T2 < 1 || B < 1) return fail(LBF_E_INVAL, "lbf_beam_major: sizes must be >= 1");
    if (K != 1 && K != 4) return fail(LBF_E_INVAL, "lbf_beam_major: K must be 1 or 4 (got %d)", K);
    if (!d_in || !d_out) return fail(LBF_E_INVAL, "lbf_beam_major: NULL device pointer");
    const size_t bytes = (size_t)C2 * K * T2 * B * sizeof(float);
    const char* a = (const char*)d_in;
    const char* b = (const char*)d_out;
    if (a < b + bytes && b < a + bytes) return fail(LBF_E_INVAL, "lbf_beam_major: input and output overlap");
    if ((long long)K * T2 > 0x7fffffffLL || C2 > (1 << 26) || B > (1 << 26))
        return fail(LBF_E_INVAL, "lbf_beam_major: too large");
    hipError_t e = lbf::launch_stage_to_beam_major(d_in, C2, T2, B * K, B * K, d_out, (size_t)C2, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_beam_major");
    return ok();
}

int lbf_beamform_batch(const lbf_block* blks, int n, void* stream) {
    return lbf::run_batch(blks, n, nullptr, nullptr, stream, "lbf_beamform_batch");
}

int lbf_stokes(const float* d_y, int B, int C, int T, int product, int t_int, int f_int, float* d_s, void* stream) {
    if (B < 1 || C < 1 || T < 1) return fail(LBF_E_INVAL, "lbf_stokes: sizes must be >= 1");
    if (!d_y || !d_s) return fail(LBF_E_INVAL, "lbf_stokes: NULL device pointer");
    if (product != LBF_STOKES_I && product != LBF_STOKES_IQUV)
        return fail(LBF_E_INVAL, "lbf_stokes: product must be STOKES_I or STOKES_IQUV (got %d)", product);
    if (t_int < 1 || f_int < 1 || T % t_int || C % f_int)
        return fail(LBF_E_INVAL, "lbf_stokes: t_int=%d must divide T=%d and f_int=%d must divide C=%d", t_int, T,
                    f_int, C);
    hipError_t e = lbf::launch_stokes(d_y, B, C, T, product, t_int, f_int, d_s, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_stokes");
    return ok();
}

int lbf_transpose(const void* d_in, int C2, int B, int T2, int K, int elem_bytes, void* d_out, void* stream) {
    if (C2 < 1 || B < 1 || T2 < 1 || K < 1) return fail(LBF_E_INVAL, "lbf_transpose: sizes must be >= 1");
    if (!d_in || !d_out) return fail(LBF_E_INVAL, "lbf_transpose: NULL device pointer");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(LBF_E_INVAL, "lbf_transpose: elem_bytes must be 4 or 8");
    const size_t bytes = (size_t)C2 * B * T2 * K * elem_bytes;
    const char* a = (const char*)d_in;
    const char* b = (const char*)d_out;
    if (a < b + bytes && b < a + bytes) return fail(LBF_E_INVAL, "lbf_transpose: input and output overlap");
    if ((long long)B * T2 * K > (1LL << 40) / 32) return fail(LBF_E_INVAL, "lbf_transpose: too large");
    hipError_t e = lbf::launch_transpose(d_in, C2, B, T2, K, elem_bytes, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_transpose");
    return ok();
}

int lbf_incoherent(const void* d_x, int xtype, int S, int C, int T, int product, int t_int, int f_int, float* d_out,
                   void* stream) {
    if (S < 1 || C < 1 || T < 1) return fail(LBF_E_INVAL, "lbf_incoherent: sizes must be >= 1");
    if (!d_x || !d_out) return fail(LBF_E_INVAL, "lbf_incoherent: NULL device pointer");
    if (xtype < LBF_CI8 || xtype > LBF_CF32) return fail(LBF_E_INVAL, "lbf_incoherent: unknown xtype %d", xtype);
    if (product != LBF_STOKES_I && product != LBF_STOKES_IQUV)
        return fail(LBF_E_INVAL, "lbf_incoherent: product must be STOKES_I or STOKES_IQUV");
    if (t_int < 1 || f_int < 1 || T % t_int || C % f_int)
        return fail(LBF_E_INVAL, "lbf_incoherent: t_int must divide T and f_int must divide C");
    hipError_t e = lbf::launch_incoherent(d_x, xtype, S, C, T, product, t_int, f_int, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_incoherent");
    return ok();
}

int lbf_superstation(const void* d_x, int xtype, int S, int C, int T, const float* d_w, int G, const int* offsets,
                     const int* members, float* d_out, void* stream) {
    if (S < 1 || C < 1 || T < 1) return fail(LBF_E_INVAL, "lbf_superstation: sizes must be >= 1");
    if (xtype < LBF_CI8 || xtype > LBF_CF32) return fail(LBF_E_INVAL, "lbf_superstation: unknown xtype %d", xtype);
    if (G < 1 || G > lbf::kSsMaxGroups)
        return fail(LBF_E_INVAL, "lbf_superstation: G=%d outside 1..%d", G, lbf::kSsMaxGroups);
    if (!offsets || !members) return fail(LBF_E_INVAL, "lbf_superstation: NULL group table");
    if (!d_x || !d_out) return fail(LBF_E_INVAL, "lbf_superstation: NULL device pointer");
    if (((uintptr_t)d_x | (uintptr_t)d_out) & 15) return fail(LBF_E_INVAL, "lbf_superstation: buffers must be 16-byte aligned");
    if (((uintptr_t)d_w) & 7) return fail(LBF_E_INVAL, "lbf_superstation: weights must be 8-byte aligned");
    lbf::SsGroups gr;
    gr.G = G;
    if (offsets[0] != 0) return fail(LBF_E_INVAL, "lbf_superstation: offsets[0] must be 0");
    for (int g = 0; g <= G; ++g) {
        if (g > 0 && offsets[g] < offsets[g - 1]) return fail(LBF_E_INVAL, "lbf_superstation: offsets must not decrease");
        gr.off[g] = offsets[g];
    }
    if (offsets[G] > lbf::kSsMaxMembers)
        return fail(LBF_E_INVAL, "lbf_superstation: %d members, at most %d", offsets[G], lbf::kSsMaxMembers);
    for (int m = 0; m < offsets[G]; ++m) {
        if (members[m] < 0 || members[m] >= S)
            return fail(LBF_E_INVAL, "lbf_superstation: member %d is station %d, outside 0..%d", m, members[m], S - 1);
        gr.mem[m] = members[m];
    }
    if ((long long)G * C * ((T + 255) / 256) > 0x7fffffffLL) return fail(LBF_E_INVAL, "lbf_superstation: too large");
    const size_t in_bytes = (size_t)S * C * T * (xtype == LBF_CI8 ? 4 : xtype == LBF_CI16 ? 8 : 16);
    const size_t out_bytes = (size_t)G * C * T * 16;
    const char* a = (const char*)d_x;
    const char* o = (const char*)d_out;
    const char* wv = (const char*)d_w;
    if (a < o + out_bytes && o < a + in_bytes) return fail(LBF_E_INVAL, "lbf_superstation: input and output overlap");
    if (wv && wv < o + out_bytes && o < wv + (size_t)C * S * 8)
        return fail(LBF_E_INVAL, "lbf_superstation: weights and output overlap");
    hipError_t e = lbf::launch_superstation(d_x, xtype, S, C, T, d_w, gr, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_superstation");
    return ok();
}

int lbf_channelize(const void* d_x, int xtype, int S, int NSB, int T_in, int T_sb, int nch, const int* d_shift,
                   float* d_out, void* stream) {
    if (S < 1 || NSB < 1 || T_in < 1 || T_sb < 1) return fail(LBF_E_INVAL, "lbf_channelize: sizes must be >= 1");
    if (nch < 2 || nch > 256 || (nch & (nch - 1)))
        return fail(LBF_E_INVAL, "lbf_channelize: nch must be a power of two from 2 to 256 (got %d)", nch);
    if (T_sb % nch) return fail(LBF_E_INVAL, "lbf_channelize: T_sb=%d is not a multiple of nch=%d", T_sb, nch);
    if (xtype < LBF_CI8 || xtype > LBF_CF32) return fail(LBF_E_INVAL, "lbf_channelize: unknown xtype %d", xtype);
    if (!d_x || !d_out) return fail(LBF_E_INVAL, "lbf_channelize: NULL device pointer");
    if (((uintptr_t)d_x | (uintptr_t)d_out) & 15) return fail(LBF_E_INVAL, "lbf_channelize: buffers must be 16-byte aligned");
    if (((uintptr_t)d_shift) & 3) return fail(LBF_E_INVAL, "lbf_channelize: shift must be 4-byte aligned");
    const long long tiles = (T_sb / nch + lbf::kChTile / nch - 1) / (lbf::kChTile / nch);
    if ((long long)S * NSB * tiles > 0x7fffffffLL) return fail(LBF_E_INVAL, "lbf_channelize: too large");
    const size_t in_bytes = (size_t)S * NSB * T_in * (xtype == LBF_CI8 ? 4 : xtype == LBF_CI16 ? 8 : 16);
    const size_t out_bytes = (size_t)S * NSB * T_sb * 16;
    const char* a = (const char*)d_x;
    const char* o = (const char*)d_out;
    if (a < o + out_bytes && o < a + in_bytes) return fail(LBF_E_INVAL, "lbf_channelize: input and output overlap");
    const char* sh = (const char*)d_shift;
    if (sh && sh < o + out_bytes && o < sh + (size_t)S * sizeof(int))
        return fail(LBF_E_INVAL, "lbf_channelize: shift and output overlap");
    hipError_t e = lbf::launch_channelize(d_x, xtype, S, NSB, T_in, T_sb, nch, d_shift, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_channelize");
    return ok();
}

int lbf_dedisperse(const void* d_y, int C, int B, int T, int n_fft, const void* d_chirp, void* d_out, void* stream) {
    if (C < 1 || B < 1 || T < 1) return fail(LBF_E_INVAL, "lbf_dedisperse: sizes must be >= 1");
    if (n_fft != 8 && n_fft != 64 && n_fft != 512 && n_fft != 4096)
        return fail(LBF_E_INVAL, "lbf_dedisperse: n_fft must be 8, 64, 512 or 4096 (got %d)", n_fft);
    if (T % n_fft) return fail(LBF_E_INVAL, "lbf_dedisperse: T=%d is not a multiple of n_fft=%d", T, n_fft);
    if (!d_y || !d_chirp || !d_out) return fail(LBF_E_INVAL, "lbf_dedisperse: NULL device pointer");
    if (((uintptr_t)d_y | (uintptr_t)d_chirp | (uintptr_t)d_out) & 15)
        return fail(LBF_E_INVAL, "lbf_dedisperse: buffers must be 16-byte aligned");
    if ((long long)C * B * (T / n_fft) > 0x7fffffffLL) return fail(LBF_E_INVAL, "lbf_dedisperse: too many blocks");
    const size_t bytes = (size_t)C * B * T * 16;
    const char* a = (const char*)d_y;
    const char* o = (const char*)d_out;
    if (a != o && a < o + bytes && o < a + bytes) return fail(LBF_E_INVAL, "lbf_dedisperse: input and output overlap");
    const char* h = (const char*)d_chirp;
    const size_t hbytes = (size_t)C * n_fft * 8;
    if (h < o + bytes && o < h + hbytes) return fail(LBF_E_INVAL, "lbf_dedisperse: chirp and output overlap");
    hipError_t e = lbf::launch_dedisperse(d_y, C, B, T, n_fft, d_chirp, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_dedisperse");
    return ok();
}

int lbf_dedisperse_stokes(const void* d_y, int C, int B, int T, int n_fft, const void* d_chirp, int product, int t_int,
                          float* d_s, void* stream) {
    if (C < 1 || B < 1 || T < 1) return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: sizes must be >= 1");
    if (n_fft != 8 && n_fft != 64 && n_fft != 512 && n_fft != 4096)
        return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: n_fft must be 8, 64, 512 or 4096 (got %d)", n_fft);
    if (T % n_fft) return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: T=%d is not a multiple of n_fft=%d", T, n_fft);
    if (product != LBF_STOKES_I && product != LBF_STOKES_IQUV)
        return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: product must be STOKES_I or STOKES_IQUV (got %d)", product);
    const int tmax = 64 * (n_fft >= 256 ? n_fft / 256 : 1);
    if (!is_pow2(t_int) || t_int > n_fft || t_int > tmax)
        return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: t_int=%d must be a power of two up to %d", t_int,
                    n_fft < tmax ? n_fft : tmax);
    if (!d_y || !d_chirp || !d_s) return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: NULL device pointer");
    if (((uintptr_t)d_y | (uintptr_t)d_chirp | (uintptr_t)d_s) & 15)
        return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: buffers must be 16-byte aligned");
    if ((long long)C * B * (T / n_fft) > 0x7fffffffLL)
        return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: too many blocks");
    const size_t ybytes = (size_t)C * B * T * 16, sbytes = (size_t)C * B * (T / t_int) * product * 4;
    const char* a = (const char*)d_y;
    const char* o = (const char*)d_s;
    if (a < o + sbytes && o < a + ybytes) return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: input and output overlap");
    const char* h = (const char*)d_chirp;
    if (h < o + sbytes && o < h + (size_t)C * n_fft * 8)
        return fail(LBF_E_INVAL, "lbf_dedisperse_stokes: chirp and output overlap");
    hipError_t e = lbf::launch_dedisperse_stokes(d_y, C, B, T, n_fft, d_chirp, product, t_int, d_s, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_dedisperse_stokes");
    return ok();
}

int lbf_probe(int kind, int iters, const void* d_src, void* d_dst, uint64_t bytes, double* work, void* stream) {
    if (!work || !d_dst) return fail(LBF_E_INVAL, "lbf_probe: NULL pointer");
    if (kind < 0 || kind > 3) return fail(LBF_E_INVAL, "lbf_probe: unknown kind %d", kind);
    if (kind < 2 && iters < 1) return fail(LBF_E_INVAL, "lbf_probe: iters must be >= 1");
    if (kind >= 2 && (!d_src || bytes < 16))
        return fail(LBF_E_INVAL, "lbf_probe: copy and read need a source and >= 16 bytes");
    hipError_t e = lbf::launch_probe(kind, iters, d_src, d_dst, (size_t)bytes, work, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbf_probe");
    return LBF_OK;
}

int lbf_check_addressing(const lbf_block* blk, int channel_major, uint64_t staging_cap, int threads,
                         uint64_t* accesses) {
    int rc = check_block(blk, "lbf_check_addressing");
    if (rc) return rc;
    if (threads < 1 || threads > 64) return fail(LBF_E_INVAL, "lbf_check_addressing: threads must be 1..64");
    char msg[400];
    const int r = lbf::check_block_addressing(to_desc(blk), channel_major != 0, (size_t)staging_cap, threads, accesses,
                                              msg, sizeof(msg));
    if (r == 2) return fail(LBF_E_NOMEM, "lbf_check_addressing: staging holds less than one channel");
    if (r != 0) return fail(LBF_E_INVAL, "lbf_check_addressing: %s", msg);
    return ok();
}

int lbf_set_tile_streams(int streams) {
    if (streams != 0 && streams != 1 && streams != 2 && streams != 4)
        return fail(LBF_E_INVAL, "lbf_set_tile_streams: streams must be 0, 1, 2 or 4 (got %d)", streams);
    lbf::g_tile_streams_override.store(streams, std::memory_order_relaxed);
    return ok();
}

int lbf_block_footprint(const lbf_block* b, lbf_block_sizes* out) {
    if (!out) return fail(LBF_E_INVAL, "lbf_block_footprint: out is NULL");
    if (!b) return fail(LBF_E_INVAL, "lbf_block_footprint: block is NULL");
    if (b->S < 1 || b->C < 1 || b->T < 1 || b->B < 1 || b->t_int < 1 || b->f_int < 1)
        return fail(LBF_E_INVAL, "lbf_block_footprint: sizes must be >= 1");
    if (b->xtype < LBF_CI8 || b->xtype > LBF_CF32 || b->ctype < LBF_F32 || b->ctype > LBF_BF16)
        return fail(LBF_E_INVAL, "lbf_block_footprint: unknown type");
    if (b->product != LBF_VOLTAGES && b->product != LBF_STOKES_I && b->product != LBF_STOKES_IQUV)
        return fail(LBF_E_INVAL, "lbf_block_footprint: unknown product");
    const uint64_t S = b->S, C = b->C, T = b->T, B = b->B;
    out->input_bytes = S * C * T * 2 * bytes_per_complex(b->xtype);
    out->weight_bytes = C * B * S * weight_bytes(b->ctype);
    if (b->product == LBF_VOLTAGES) out->output_bytes = C * B * T * 2 * 8;
    else out->output_bytes = B * (uint64_t)b->product * (T / b->t_int) * (C / b->f_int) * 4;
    out->flops = 8.0 * (double)B * (double)S * (double)C * (double)T * 2.0;
    out->staging_channel_bytes = 0;
    out->staging_bytes = 0;
    if (b->product != LBF_VOLTAGES && b->T % b->t_int == 0 && b->C % b->f_int == 0) {
        lbf_block v = *b;
        v.d_x = v.d_w = v.d_out = (void*)b;   // sizes only: any non-NULL pointer
        out->staging_channel_bytes = lbf::block_staging_channel_bytes(&v);
        out->staging_bytes = out->staging_channel_bytes * C;
    }
    return ok();
}

}  // extern "C"
