// bf_batch.hip -- persistent launches over the work items of several blocks
// (Section 7 of Mol & Romein: independent observations processed in parallel
// while resources allow).  The blocks are grouped by worker variant (input
// type, product, K-steps, beam streams); one persistent launch per variant
// present pulls that group's items from a device counter.  Each item runs
// exactly the worker lbf_beamform would run for it, so every block's result is
// bitwise the same alone or in a batch.  A kernel holding every variant at
// once would carry the register needs of the largest and spill; one variant per
// launch keeps the registers of the single-block kernels.  Blocks outside the
// fast path (more than 64 stations, t_int other than 16, channel integration,
// complex float input) are rare in a batch and run through their own launches
// on the same stream.
#include "bf_common.h"
#include "bf_workers.h"

namespace lbf {

struct BatchArgs {
    BlockDesc blk[kMaxBatch];
    int item_start[kMaxBatch + 1];   // prefix sums of items per block
    int nbg[kMaxBatch];
    int n;
};
static_assert(sizeof(BatchArgs) <= 4096, "kernel argument block");

// Items of t_int = 16 Stokes blocks (the common integration) run the fast
// workers; everything else in a batch runs the generic ones.
__host__ __device__ inline bool batch_fast(const BlockDesc& d) {
    return fast_path(d) && d.t_int == 16 && d.xtype != XT_CF32;
}

// variant index of a fast block: ((xtype, product), K-steps 4..8, streams 1, 2, 4)
constexpr int kBatchVariants = 2 * 2 * 5 * 3;
inline int batch_variant(const BlockDesc& d) {
    const int ik = fast_h_ksteps(d.S) - 4;
    const int xp = (d.xtype == XT_CI8 ? 0 : 2) + (d.product == PR_I ? 0 : 1);
    const int ns = fast_h_streams(d);
    return (xp * 5 + ik) * 3 + (ns == 1 ? 0 : ns == 2 ? 1 : 2);
}

template <int XT, int CT, int PR, int NK, int NS>
__global__ __launch_bounds__(kThreadsH) void bf_batch_kernel(BatchArgs a, int* counter) {
    __shared__ __attribute__((aligned(16))) uint32_t at[NS * 2 * kATileWords];
    __shared__ int next;
    const int total = a.item_start[a.n];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        if (it >= total) break;     // every work group leaves once the list is exhausted
        int j = 0;
        while (j + 1 < a.n && a.item_start[j + 1] <= it) ++j;
        item_h_fast<XT, CT, PR, 16, NK, NS>(a.blk[j], it - a.item_start[j], a.nbg[j], at);
    }
}

__global__ void fill_int_kernel(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One persistent launch of variant <XT, CT, PR, NK, NS>: one resident work
// group per slot the hardware offers; the queue, not the grid, spreads the
// uneven items.
template <int XT, int CT, int PR, int NK, int NS>
hipError_t launch_batch_k(const BatchArgs& a, int* counter, hipStream_t st) {
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bf_batch_kernel<XT, CT, PR, NK, NS>, kThreadsH, 0);
    if (per_cu < 1) per_cu = 1;
    const int total = a.item_start[a.n];
    const int slots = cus * per_cu;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, st, counter, 1, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bf_batch_kernel<XT, CT, PR, NK, NS>), dim3(total < slots ? total : slots), dim3(kThreadsH), 0,
                       st, a, counter);
    return hipGetLastError();
}

template <int XT, int CT, int PR, int NK>
hipError_t launch_batch_nk(int v, const BatchArgs& a, int* counter, hipStream_t st) {
    switch (v % 3) {
        case 0: return launch_batch_k<XT, CT, PR, NK, 1>(a, counter, st);
        case 1: return launch_batch_k<XT, CT, PR, NK, 2>(a, counter, st);
        default: return launch_batch_k<XT, CT, PR, NK, 4>(a, counter, st);
    }
}

template <int XT, int CT, int PR>
hipError_t launch_batch_pr(int v, const BatchArgs& a, int* counter, hipStream_t st) {
    switch (v % 15 / 3) {
        case 0: return launch_batch_nk<XT, CT, PR, 4>(v, a, counter, st);
        case 1: return launch_batch_nk<XT, CT, PR, 5>(v, a, counter, st);
        case 2: return launch_batch_nk<XT, CT, PR, 6>(v, a, counter, st);
        case 3: return launch_batch_nk<XT, CT, PR, 7>(v, a, counter, st);
        default: return launch_batch_nk<XT, CT, PR, 8>(v, a, counter, st);
    }
}

template <int CT>
hipError_t launch_batch_variant(int v, const BatchArgs& a, int* counter, hipStream_t st) {
    switch (v / 15) {
        case 0: return launch_batch_pr<XT_CI8, CT, PR_I>(v, a, counter, st);
        case 1: return launch_batch_pr<XT_CI8, CT, PR_IQUV>(v, a, counter, st);
        case 2: return launch_batch_pr<XT_CI16, CT, PR_I>(v, a, counter, st);
        default: return launch_batch_pr<XT_CI16, CT, PR_IQUV>(v, a, counter, st);
    }
}

// One group of batch-kernel blocks; block idx[g] forms its Stokes products
// channel-major in stage[g], then they are reordered into its final order.
static hipError_t run_batch_group(const BlockDesc* blks, const int* idx, int n, char* const* stage, int* d_counter,
                                  hipStream_t st) {
    BatchArgs a;
    a.n = 0;
    a.item_start[0] = 0;
    int entry_src[kMaxBatch];
    for (int g = 0; g < n; ++g) {
        const BlockDesc& b = blks[idx[g]];
        // a beam tail of at most 128 beams becomes an entry of its own while
        // the argument block has room (it holds kMaxBatch entries)
        BlockDesc part[2];
        int np = split_fast_h(b, part);
        if (a.n + np + (n - 1 - g) > kMaxBatch) np = 1, part[0] = b;
        for (int p = 0; p < np; ++p) {
            entry_src[a.n] = g;
            a.blk[a.n++] = part[p];
        }
    }
    for (int j = 0; j < a.n; ++j) {
        a.blk[j].out = stage[entry_src[j]];
        a.blk[j].order = 1;
        a.blk[j].ld_row = staging_ld(a.blk[j].B, a.blk[j].product == PR_IQUV ? 4 : 1);
        int nbg;
        const int items = block_items_fast_h(a.blk[j], &nbg);
        a.nbg[j] = nbg;
        a.item_start[j + 1] = a.item_start[j] + items;
    }
    // one launch per variant present, in variant order, on the same stream;
    // the counter is reset before each
    hipError_t e = hipSuccess;
    for (int v = 0; v < kBatchVariants && e == hipSuccess; ++v) {
        BatchArgs g;
        g.n = 0;
        g.item_start[0] = 0;
        for (int j = 0; j < a.n; ++j) {
            if (batch_variant(a.blk[j]) != v) continue;
            g.blk[g.n] = a.blk[j];
            g.nbg[g.n] = a.nbg[j];
            g.item_start[g.n + 1] = g.item_start[g.n] + (a.item_start[j + 1] - a.item_start[j]);
            g.n++;
        }
        if (g.n == 0) continue;
        e = a.blk[0].ctype == CT_F16 ? launch_batch_variant<CT_F16>(v, g, d_counter, st)
                                     : launch_batch_variant<CT_BF16>(v, g, d_counter, st);
    }
    for (int g = 0; g < n && e == hipSuccess; ++g) {
        const BlockDesc& b = blks[idx[g]];
        const int K = b.product == PR_IQUV ? 4 : 1;
        e = launch_stage_to_beam_major((const float*)stage[g], b.C, b.T / b.t_int, b.B * K, staging_ld(b.B, K),
                                       (float*)b.out, (size_t)b.C, st);
    }
    return e;
}

static size_t staging_block_bytes(const BlockDesc& b) {
    return ((size_t)b.C * staging_channel_bytes(b) + 255) & ~(size_t)255;
}

hipError_t launch_beamform_batch(const BlockDesc* blks, int n, int* d_counter, void* const* stage, const size_t* cap,
                                 hipStream_t st) {
    int idx[kMaxBatch], nb = 0;
    char* sp[kMaxBatch];
    size_t total = 0;
    for (int j = 0; j < n; ++j) {
        const bool fits = stage == nullptr || (stage[j] != nullptr && staging_block_bytes(blks[j]) <= cap[j]);
        if (batch_fast(blks[j]) && fits) {
            sp[nb] = stage ? (char*)stage[j] : nullptr;
            idx[nb++] = j;
            total += staging_block_bytes(blks[j]);
            continue;
        }
        // outside the batch kernel's path, or staging that holds only part of
        // the block's channels: its own launches
        const hipError_t e = stage ? launch_beamform_staged(blks[j], stage[j], cap[j], st) : launch_beamform(blks[j], st);
        if (e != hipSuccess) return e;
    }
    if (nb == 0) return hipSuccess;
    if (stage != nullptr) return run_batch_group(blks, idx, nb, sp, d_counter, st);
    // staging of the whole batch from the stream-ordered pool
    char* pool = nullptr;
    hipError_t e = staging_alloc((void**)&pool, total, st);
    if (e != hipSuccess) return e;
    size_t o = 0;
    for (int g = 0; g < nb; ++g) {
        sp[g] = pool + o;
        o += staging_block_bytes(blks[idx[g]]);
    }
    e = run_batch_group(blks, idx, nb, sp, d_counter, st);
    const hipError_t ef = hipFreeAsync(pool, st);
    return e != hipSuccess ? e : ef;
}

}  // namespace lbf
