// lbf_launch.h -- host-side launchers of the lbf kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include "lbf_device.h"

namespace lbf {

constexpr int kMaxBatch = 32;   // equals LBF_MAX_BATCH in include/lbf.h

// Set the calling thread's lbf_last_error() text; returns code.
int set_error(int code, const char* fmt, ...);

hipError_t launch_weights(const double* pos, int S, const double* dir, int B, double rx, double ry, double rz,
                          const double* freq, int C, int wtype, void* w, double* tau, hipStream_t st);
hipError_t launch_beamform(const BlockDesc& d, hipStream_t st);
hipError_t launch_beamform_generic(const BlockDesc& d, hipStream_t st);
hipError_t launch_fast_f32(const BlockDesc& d, hipStream_t st);
hipError_t launch_fast_f16(const BlockDesc& d, hipStream_t st);
hipError_t launch_fast_bf16(const BlockDesc& d, hipStream_t st);
hipError_t launch_beamform_batch(const BlockDesc* blks, int n, int* d_counter, hipStream_t st);
hipError_t staging_alloc(void** p, size_t bytes, hipStream_t st);
hipError_t launch_stokes(const float* y, int B, int C, int T, int product, int t_int, int f_int, float* s,
                         hipStream_t st);
hipError_t launch_transpose(const void* in, int C2, int B, int T2, int K, int elem_bytes, void* out,
                            hipStream_t st);
hipError_t launch_probe(int kind, int iters, const void* src, void* dst, size_t bytes, double* work, hipStream_t st);
hipError_t launch_stage_to_beam_major(const float* stage, int C2, int M, int B, int ldb, float* out, hipStream_t st);
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

}  // namespace lbf
