// bf_generic.hip -- contraction workers for any station count and input type
// (stations in chunks of 64 whose weights are restaged in LDS per tile).  The
// fast workers in bf_fast.hip cover up to 64 stations of complex int8/int16;
// these cover the rest (more stations, complex float32 input).
#include "bf_common.h"
#include "bf_workers.h"

#include <mutex>

namespace lbf {

template <int XT, int PR>
__global__ __launch_bounds__(kThreads) void bf_f32_generic_kernel(BlockDesc d, int nbg, int nitems) {
    __shared__ float wl[kStationChunk * 2 * kBeamGroup];
    item_f32_generic<XT, PR>(d, xcd_remap(blockIdx.x, nitems), nbg, wl);
}

template <int XT, int CT, int PR>
__global__ __launch_bounds__(kThreads) void bf_h_generic_kernel(BlockDesc d, int nbg, int nitems) {
    __shared__ __attribute__((aligned(16))) uint32_t wh[kBeamGroup * kWRow];
    item_h_generic<XT, CT, PR>(d, xcd_remap(blockIdx.x, nitems), nbg, wh);
}

template <int XT>
static hipError_t launch_f32(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    dim3 grid(n), block(kThreads);
    switch (d.product) {
        case PR_VOLT: hipLaunchKernelGGL((bf_f32_generic_kernel<XT, PR_VOLT>), grid, block, 0, st, d, nbg, n); break;
        case PR_I: hipLaunchKernelGGL((bf_f32_generic_kernel<XT, PR_I>), grid, block, 0, st, d, nbg, n); break;
        default: hipLaunchKernelGGL((bf_f32_generic_kernel<XT, PR_IQUV>), grid, block, 0, st, d, nbg, n); break;
    }
    return hipGetLastError();
}

template <int XT, int CT>
static hipError_t launch_h(const BlockDesc& d, int nbg, int n, hipStream_t st) {
    dim3 grid(n), block(kThreads);
    switch (d.product) {
        case PR_VOLT: hipLaunchKernelGGL((bf_h_generic_kernel<XT, CT, PR_VOLT>), grid, block, 0, st, d, nbg, n); break;
        case PR_I: hipLaunchKernelGGL((bf_h_generic_kernel<XT, CT, PR_I>), grid, block, 0, st, d, nbg, n); break;
        default: hipLaunchKernelGGL((bf_h_generic_kernel<XT, CT, PR_IQUV>), grid, block, 0, st, d, nbg, n); break;
    }
    return hipGetLastError();
}

hipError_t launch_beamform_generic(const BlockDesc& d, hipStream_t st) {
    int nbg;
    const int n = block_items(d, &nbg);
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

static hipError_t launch_fast(const BlockDesc& d, hipStream_t st) {
    if (d.ctype == CT_F32) return launch_fast_f32(d, st);
    if (d.ctype == CT_F16) return launch_fast_f16(d, st);
    return launch_fast_bf16(d, st);
}

// Staging buffers come from the device's default stream-ordered pool.  The
// pool keeps freed memory (instead of unmapping it at every synchronisation),
// so a block's staging costs no page mapping once the pool has grown.
hipError_t staging_alloc(void** p, size_t bytes, hipStream_t st) {
    static std::once_flag flags[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) {
        std::call_once(flags[dev], [dev] {
            hipMemPool_t pool;
            if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
                uint64_t keep = ~0ull;
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            }
        });
    }
    return hipMallocAsync(p, bytes, st);
}

// The fast workers write Stokes products channel-major ([C'][T'][B][K], one
// 16-byte store per beam and period for IQUV); a beam-major block (order 0)
// goes through a staging buffer of that layout, rows padded to a multiple of
// 32 floats, and a tiled transpose.
// Stokes staging: the final order from the fast workers (the reorder follows
// them), and channel integration on the fast workers in either order (the
// channel sums follow them)
bool needs_staging(const BlockDesc& d) {
    if (d.product == PR_VOLT) return false;
    return (d.order == 0 && fast_path(d)) || fast_path_fint(d);
}

bool fuses_incoherent(const BlockDesc& d) {
    return fast_path(d) && d.ctype != CT_F32 && d.product != PR_VOLT && fast_h_streams(d) >= 2;
}

size_t staging_channel_bytes(const BlockDesc& d) {
    const int K = d.product == PR_IQUV ? 4 : 1;
    return (size_t)(d.T / d.t_int) * staging_ld(d.B, K) * sizeof(float);
}

// Channels per pass through a staging buffer of `cap` bytes: all of them if
// they fit, else the most that fit rounded down to a multiple of 64 (or 4), so
// that the reorder keeps its 16-byte stores, and always whole groups of f_int
// channels (f_int a power of two up to 64); 0 if not even one group fits.
int staging_chunk(const BlockDesc& d, size_t cap) {
    const size_t n = cap / staging_channel_bytes(d);
    const int F = d.product == PR_VOLT ? 1 : d.f_int;
    if (n >= (size_t)d.C) return d.C;
    if (n >= 64) return (int)(n / 64 * 64);
    if (n >= 4 && F <= 4) return (int)(n / 4 * 4);
    return (int)(n / F * F);
}

hipError_t launch_beamform_direct(const BlockDesc& d, hipStream_t st) {
    if (!fast_path(d)) return launch_beamform_generic(d, st);
    return launch_fast(d, st);
}

// A block through caller-provided staging of `cap` bytes: the channels in
// passes of staging_chunk(d, cap), each pass the contraction into the staging
// buffer (per channel, integrated in time) and then, out of the staging, the
// reorder into the final order or, with channel integration, the sums over
// each group of f_int channels (in channel order, into the final order or the
// channel-major one); the passes are ordered by the stream, so they reuse the
// buffer.
hipError_t launch_beamform_staged(const BlockDesc& d, void* stage, size_t cap, hipStream_t st) {
    if (!needs_staging(d)) return launch_beamform_direct(d, st);
    const int K = d.product == PR_IQUV ? 4 : 1;
    const int F = d.f_int;
    const int T2 = d.T / d.t_int;
    const int ld = staging_ld(d.B, K);
    const int nc = staging_chunk(d, cap);
    if (nc < 1 || stage == nullptr) return hipErrorInvalidValue;
    for (int c0 = 0; c0 < d.C; c0 += nc) {
        BlockDesc ds = d;
        ds.out = stage;
        ds.order = 1;
        ds.ld_row = ld;
        ds.f_int = 1;
        ds.c0 = c0;
        ds.nc = d.C - c0 < nc ? d.C - c0 : nc;
        hipError_t e = launch_fast(ds, st);
        if (e != hipSuccess) return e;
        if (d.order == 1)          // [c][t'][b k] -> channel sums [c'][t'][b k] (rows of B K floats)
            e = launch_stage_sum_channels((const float*)stage, ds.nc, T2, d.B * K, ld, F,
                                          (float*)d.out + (size_t)(c0 / F) * T2 * d.B * K, st);
        else if (F == 1)           // [c][t'][b k] -> [b k][t'][c]: the beam-major final order [b][k][t'][c]
            e = launch_stage_to_beam_major((const float*)stage, ds.nc, T2, d.B * K, ld, (float*)d.out + c0,
                                           (size_t)d.C, st);
        else                       // the same with the channel sums
            e = launch_stage_sum_to_beam_major((const float*)stage, ds.nc, T2, d.B * K, ld, F,
                                               (float*)d.out + c0 / F, (size_t)(d.C / F), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Staging of lbf_beamform_noalloc: a fixed array in device memory, one per
// GPU the library runs on (mapped when the library's code is loaded there,
// held until the process ends).  In host code `scratch` names a host-side
// stand-in, not the device array: host code only ever uses the per-device
// address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** p) {
    static std::mutex mu;
    static void* addr[64] = {nullptr};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (addr[dev] == nullptr) {
        void* a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));   // with this device current
        if (e != hipSuccess) return e;
        if (a == nullptr) return hipErrorInvalidSymbol;
        addr[dev] = a;
    }
    *p = addr[dev];
    return hipSuccess;
}

// lbf_beamform: the fast workers where they apply, the generic ones
// otherwise; the staging of a whole block comes from the stream-ordered pool.
hipError_t launch_beamform(const BlockDesc& d, hipStream_t st) {
    if (!needs_staging(d)) return launch_beamform_direct(d, st);
    const size_t bytes = (size_t)d.C * staging_channel_bytes(d);
    void* stage = nullptr;
    hipError_t e = staging_alloc(&stage, bytes, st);
    if (e != hipSuccess) return e;
    e = launch_beamform_staged(d, stage, bytes, st);
    const hipError_t ef = hipFreeAsync(stage, st);
    return e != hipSuccess ? e : ef;
}

}  // namespace lbf
