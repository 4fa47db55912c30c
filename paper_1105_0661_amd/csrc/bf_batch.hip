// bf_batch.hip -- one persistent launch over the work items of several
// blocks (Section 7 of Mol & Romein: independent observations processed in
// parallel while resources allow).  Work groups pull items from a device
// counter; each item runs exactly the worker lbf_beamform would run for it,
// so every block's result is bitwise the same alone or in a batch.  Blocks
// outside the fast path (more than 64 stations, t_int other than 16, channel
// integration, complex float input) are rare in a batch and run through their
// own launches on the same stream.
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
__host__ __device__ inline bool batch_fast(const BlockDesc& d) { return fast_path(d) && d.t_int == 16; }

template <int XT, int CT, int PR>
LBF_INLINE void batch_item_fast(const BlockDesc& d, int item, int nbg, uint32_t* at) {
    const int nk = fast_h_ksteps(d.S);
    if (fast_h_streams(d) == 1) {
        if (nk == 4) item_h_fast<XT, CT, PR, 16, 4, 1>(d, item, nbg, at);
        else if (nk == 6) item_h_fast<XT, CT, PR, 16, 6, 1>(d, item, nbg, at);
        else item_h_fast<XT, CT, PR, 16, 8, 1>(d, item, nbg, at);
    } else {
        if (nk == 4) item_h_fast<XT, CT, PR, 16, 4, 2>(d, item, nbg, at);
        else if (nk == 6) item_h_fast<XT, CT, PR, 16, 6, 2>(d, item, nbg, at);
        else item_h_fast<XT, CT, PR, 16, 8, 2>(d, item, nbg, at);
    }
}

template <int CT>
__global__ __launch_bounds__(kThreadsH) void bf_batch_kernel(BatchArgs a, int* counter) {
    __shared__ __attribute__((aligned(16))) uint32_t at[2 * 2 * kATileWords];
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
        const BlockDesc& d = a.blk[j];
        const int item = it - a.item_start[j];
        if (d.xtype == XT_CI8) {
            if (d.product == PR_I) batch_item_fast<XT_CI8, CT, PR_I>(d, item, a.nbg[j], at);
            else batch_item_fast<XT_CI8, CT, PR_IQUV>(d, item, a.nbg[j], at);
        } else {
            if (d.product == PR_I) batch_item_fast<XT_CI16, CT, PR_I>(d, item, a.nbg[j], at);
            else batch_item_fast<XT_CI16, CT, PR_IQUV>(d, item, a.nbg[j], at);
        }
    }
}

__global__ void fill_int_kernel(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_beamform_batch(const BlockDesc* blks, int n, int* d_counter, hipStream_t st) {
    // blocks outside the batch kernel's path: their own launches
    BatchArgs a;
    a.n = 0;
    a.item_start[0] = 0;
    size_t stage_bytes = 0, stage_off[kMaxBatch];
    int src[kMaxBatch], nsrc = 0, entry_src[kMaxBatch];
    for (int j = 0; j < n; ++j) {
        if (!batch_fast(blks[j])) {
            const hipError_t e = launch_beamform(blks[j], st);
            if (e != hipSuccess) return e;
            continue;
        }
        const int K = blks[j].product == PR_IQUV ? 4 : 1;
        stage_off[nsrc] = stage_bytes;
        stage_bytes += ((size_t)blks[j].C * (blks[j].T / blks[j].t_int) * staging_ld(blks[j].B, K) * sizeof(float) +
                        255) & ~(size_t)255;
        src[nsrc] = j;
        // a beam tail of at most 128 beams becomes an entry of its own while
        // the argument block has room (it holds kMaxBatch entries)
        BlockDesc part[2];
        int np = split_fast_h(blks[j], part);
        if (a.n + np + (n - 1 - j) > kMaxBatch) np = 1, part[0] = blks[j];
        for (int p = 0; p < np; ++p) {
            entry_src[a.n] = nsrc;
            a.blk[a.n++] = part[p];
        }
        nsrc++;
    }
    if (a.n == 0) return hipSuccess;
    // Stokes go to channel-major staging first (as in lbf_beamform), then to
    // the beam-major outputs
    char* stage = nullptr;
    hipError_t e = staging_alloc((void**)&stage, stage_bytes, st);
    if (e != hipSuccess) return e;
    for (int j = 0; j < a.n; ++j) {
        a.blk[j].out = stage + stage_off[entry_src[j]];
        a.blk[j].order = 1;
        a.blk[j].ld_row = staging_ld(a.blk[j].B, a.blk[j].product == PR_IQUV ? 4 : 1);
        int nbg;
        const int items = block_items_fast_h(a.blk[j], &nbg);
        a.nbg[j] = nbg;
        a.item_start[j + 1] = a.item_start[j] + items;
    }
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, st, d_counter, 1, 0);
    e = hipGetLastError();
    if (e == hipSuccess) {
        // one resident work group per slot the hardware offers: the queue, not
        // the grid, spreads the uneven items
        int dev = 0, cus = 256, per_cu = 1;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (a.blk[0].ctype == CT_F16)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bf_batch_kernel<CT_F16>, kThreadsH, 0);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bf_batch_kernel<CT_BF16>, kThreadsH, 0);
        if (per_cu < 1) per_cu = 1;
        const int total = a.item_start[a.n];
        const int slots = cus * per_cu;
        const int grid = total < slots ? total : slots;
        if (a.blk[0].ctype == CT_F16)
            hipLaunchKernelGGL(bf_batch_kernel<CT_F16>, dim3(grid), dim3(kThreadsH), 0, st, a, d_counter);
        else
            hipLaunchKernelGGL(bf_batch_kernel<CT_BF16>, dim3(grid), dim3(kThreadsH), 0, st, a, d_counter);
        e = hipGetLastError();
    }
    for (int j = 0; j < nsrc && e == hipSuccess; ++j) {
        const BlockDesc& b = blks[src[j]];
        const int K = b.product == PR_IQUV ? 4 : 1;
        e = launch_stage_to_beam_major((const float*)(stage + stage_off[j]), b.C, b.T / b.t_int, b.B * K,
                                       staging_ld(b.B, K), (float*)b.out, st);
    }
    const hipError_t ef = hipFreeAsync(stage, st);
    return e != hipSuccess ? e : ef;
}

}  // namespace lbf
