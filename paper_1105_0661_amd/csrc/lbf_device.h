// lbf_device.h -- device-side types and helpers shared by the lbf kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbf {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef char charx4 __attribute__((ext_vector_type(4)));

enum { XT_CI8 = 0, XT_CI16 = 1, XT_CF32 = 2 };
enum { CT_F32 = 0, CT_F16 = 1, CT_BF16 = 2 };
enum { PR_VOLT = 0, PR_I = 1, PR_IQUV = 4 };

constexpr int kWave = 64;
constexpr int kTile = 32;            // MFMA 32x32 output tile: 32 samples x 32 beams
constexpr int kXcds = 8;             // MI355X: 8 XCDs, blocks dispatched round-robin
constexpr int kCusPerXcd = 32;

// One beam-forming block as the kernels see it (mirrors lbf_block).
struct BlockDesc {
    const void* x;      // [S][C][T][2] complex
    const void* w;      // [C][B][S] complex
    void* out;          // voltages [C][B][T][2] cf32, or Stokes [B][K][T'][C'] f32
    int S, C, T, B;
    int xtype, ctype, product;
    int t_int, f_int;
    int order;          // Stokes: 0 = [B][K][T'][C'] (beam-major), 1 = [C'][T'][B][K] (channel-major)
    int b0, b1;         // beams [b0, b1) taken by the fast FP16/BF16 worker (0, B for a whole block)
    int ld_row;         // Stokes order 1: floats per [C'][T'] row of [B][K] values (>= B*K)
    int c0, nc;         // fast workers: channels [c0, c0 + nc) (0, C for a whole block); their output
                        // holds channel c at index c - c0
    float* inc;         // FP16/BF16 fast worker, Stokes: also the incoherent beam [K][T'][C], or NULL
    int ns_force;       // FP16/BF16 fast worker: sample streams per item forced for this call (1, 2, 4),
                        // or 0 for the tile table; read once when the call starts
};

// ---------------------------------------------------------------------------
// sample loads: one time sample of one station, both polarisations
// (Xre, Xim, Yre, Yim) as floats.  Indices are checked by the caller.
// ---------------------------------------------------------------------------
template <int XT> struct Sample;

template <> struct Sample<XT_CI8> {
    static constexpr int bytes = 4;
    __device__ static inline floatx4 load(const void* base, size_t idx) {
        const int v = __builtin_nontemporal_load(reinterpret_cast<const int*>(base) + idx);
        floatx4 r;
        r[0] = (float)(int8_t)(v & 0xff);
        r[1] = (float)(int8_t)((v >> 8) & 0xff);
        r[2] = (float)(int8_t)((v >> 16) & 0xff);
        r[3] = (float)(int8_t)((v >> 24) & 0xff);
        return r;
    }
};

template <> struct Sample<XT_CI16> {
    static constexpr int bytes = 8;
    __device__ static inline floatx4 load(const void* base, size_t idx) {
        const shortx4 v = reinterpret_cast<const shortx4*>(base)[idx];
        floatx4 r;
        r[0] = (float)v[0];
        r[1] = (float)v[1];
        r[2] = (float)v[2];
        r[3] = (float)v[3];
        return r;
    }
};

template <> struct Sample<XT_CF32> {
    static constexpr int bytes = 16;
    __device__ static inline floatx4 load(const void* base, size_t idx) {
        return reinterpret_cast<const floatx4*>(base)[idx];
    }
};

// ---------------------------------------------------------------------------
// FP64 -> narrow conversions with a single round-to-nearest-even: round to
// odd into float, then the hardware's RNE conversion to f16 or bf16.  Going
// through float with round-to-odd keeps one rounding: float carries 24
// significand bits, at least 2 more than f16 (11) or bf16 (8).
// ---------------------------------------------------------------------------
// Round-to-odd from the round-to-nearest result f: when d is not exact in
// float it lies strictly between two neighbouring floats, one of them odd
// (in the bit pattern) -- the round-to-odd result.  f is one of the two; if f
// is even, the odd one is the neighbour on d's side, one bit pattern step
// away.  For finite d of at most float range (weights have |d| <= 1).
__device__ inline float f64_to_f32_round_odd(double d) {
    const float f = (float)d;
    const uint32_t u = __float_as_uint(f);
    const bool step = (double)f != d && (u & 1u) == 0u;
    const uint32_t toward_zero = __builtin_fabs((double)f) > __builtin_fabs(d) ? 0xffffffffu : 1u;
    return __uint_as_float(step ? u + toward_zero : u);
}

// ---------------------------------------------------------------------------
// Sample-to-row map inside a 32-sample MFMA tile.  The 32x32 result of a
// 32x32xK MFMA leaves, in lane (h = lane/32, col = lane%32), accumulator
// element e at row (e/4)*8 + h*4 + e%4.  Feeding A-row r with sample
//   t(r) = ((r >> 2) & 1) * 16 + (r >> 3) * 4 + (r & 3)
// gives lane half h the 16 consecutive samples 16h .. 16h+15 in element
// order, so integrations over up to 16 samples stay inside one lane.
// ---------------------------------------------------------------------------
__host__ __device__ inline int tile_row_sample(int r) {
    return ((r >> 2) & 1) * 16 + (r >> 3) * 4 + (r & 3);
}

// Block index remap so that the blocks resident at the same time on one XCD
// (blocks are dispatched round-robin over the 8 XCDs) work on adjacent items:
// their beam-major stores then land in the same cache lines of that XCD's L2.
__device__ inline int xcd_remap(int i, int n) {
    constexpr int R = kXcds * kCusPerXcd;
    const int full = (n / R) * R;
    if (i >= full) return i;
    const int round = i / R, j = i % R;
    return round * R + (j % kXcds) * kCusPerXcd + j / kXcds;
}

}  // namespace lbf
