// lbf_launch.h -- host-side launchers of the lbf kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include "lbf_device.h"

namespace lbf {

constexpr int kMaxBatch = 32;   // equals LBF_MAX_BATCH in include/lbf.h

// Set the calling thread's lbf_last_error() text; returns code.
int set_error(int code, const char* fmt, ...);

hipError_t launch_weights(const double* pos, int S, const double* dir, int B, double rx, double ry, double rz,
                          const double* delay, const double* freq, int C, int wtype, void* w, double* tau,
                          hipStream_t st);
hipError_t launch_beamform(const BlockDesc& d, hipStream_t st);
// Staging (channel-major Stokes of the fast workers before the reorder):
// whether a block needs it, its bytes per channel, and a launch through a
// caller-provided buffer of cap bytes (passes of staging_chunk(d, cap)
// channels; hipErrorInvalidValue if not one channel fits).
bool needs_staging(const BlockDesc& d);
// The block's incoherent beam is formed by its contraction: the fast FP16/BF16
// worker with several sample streams (items of at most 128 beams, HBM-bound).  With more
// beams that worker is bound by MFMA and VALU work, and a separate read of
// the samples costs less than the extra work in every item (measured).
bool fuses_incoherent(const BlockDesc& d);
// 1, 2 or 4: sample streams of every FP16/BF16 fast work item; 0: the
// measured tile table (set by lbf_set_tile_streams)
extern std::atomic<int> g_tile_streams_override;
size_t staging_channel_bytes(const BlockDesc& d);
int staging_chunk(const BlockDesc& d, size_t cap);
hipError_t launch_beamform_staged(const BlockDesc& d, void* stage, size_t cap, hipStream_t st);
// staging [c][m][ldb] of C2 channels -> out[b][m][c'] (rows of ldo), c' = c / F,
// each output the sum over its F channels in channel order
hipError_t launch_stage_sum_to_beam_major(const float* stage, int C2, int M, int B, int ldb, int F, float* out,
                                          size_t ldo, hipStream_t st);
// staging [c][m][ldb] of C2 channels -> out[c'][m][B] (dense rows), the same sums
hipError_t launch_stage_sum_channels(const float* stage, int C2, int M, int B, int ldb, int F, float* out,
                                     hipStream_t st);
hipError_t launch_beamform_direct(const BlockDesc& d, hipStream_t st);   // blocks that need no staging
// The fixed staging array of lbf_beamform_noalloc on the current device: its
// device address (looked up once per device, with that device current).
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
hipError_t noalloc_scratch(void** p);
hipError_t launch_beamform_generic(const BlockDesc& d, hipStream_t st);
hipError_t launch_fast_f32(const BlockDesc& d, hipStream_t st);
hipError_t launch_fast_f16(const BlockDesc& d, hipStream_t st);
hipError_t launch_fast_bf16(const BlockDesc& d, hipStream_t st);
// stage == nullptr: staging from the stream-ordered pool; else block j has
// cap[j] bytes of caller staging at stage[j] (blocks whose staging holds all
// their channels share the persistent launches, the others run alone in
// channel passes; stage[j] may be NULL for a block that needs none)
hipError_t launch_beamform_batch(const BlockDesc* blks, int n, int* d_counter, void* const* stage, const size_t* cap,
                                 hipStream_t st);
hipError_t staging_alloc(void** p, size_t bytes, hipStream_t st);
// Host-side walk of the fast workers' accesses of a block as lbf_beamform (or,
// channel_major, lbf_beamform_channel_major) launches them, staging passes of
// cap bytes (0: whole block) included: 0 when every access is good, 1 with a
// message on the first bad one, 2 when the staging holds less than one
// channel (bf_addr_check.cpp).
int check_block_addressing(const BlockDesc& d, bool channel_major, size_t cap, int threads, uint64_t* accesses,
                           char* msg, size_t msglen);
hipError_t launch_stokes(const float* y, int B, int C, int T, int product, int t_int, int f_int, float* s,
                         hipStream_t st);
hipError_t launch_transpose(const void* in, int C2, int B, int T2, int K, int elem_bytes, void* out,
                            hipStream_t st);
hipError_t launch_probe(int kind, int iters, const void* src, void* dst, size_t bytes, double* work, hipStream_t st);
hipError_t launch_stage_to_beam_major(const float* stage, int C2, int M, int B, int ldb, float* out, size_t ldo,
                                      hipStream_t st);
hipError_t launch_incoherent(const void* x, int xtype, int S, int C, int T, int product, int t_int, int f_int,
                             float* out, hipStream_t st);
// superstation groups: member station indices of group g are mem[off[g] .. off[g + 1])
constexpr int kSsMaxGroups = 64, kSsMaxMembers = 256;
struct SsGroups {
    int G;
    int off[kSsMaxGroups + 1];
    int mem[kSsMaxMembers];
};
hipError_t launch_superstation(const void* x, int xtype, int S, int C, int T, const float* w, const SsGroups& gr,
                               float* out, hipStream_t st);
constexpr int kChTile = 2048;   // channeliser: subband samples per polarisation in one work group's tile
hipError_t launch_channelize(const void* x, int xtype, int S, int NSB, int Tin, int Tsb, int nch, const int* shift,
                             float* out, hipStream_t st);
hipError_t launch_dedisperse(const void* y, int C, int B, int T, int n_fft, const void* chirp, void* out,
                             hipStream_t st);
hipError_t launch_dedisperse_stokes(const void* y, int C, int B, int T, int n_fft, const void* chirp, int product,
                                    int t_int, float* s, hipStream_t st);

}  // namespace lbf
