/*
 * lbf.h -- C ABI of an MI355X-native tied-array beam former.
 *
 * The operations follow Mol & Romein, "The LOFAR Beam Former: Implementation
 * and Performance Analysis" (arxiv 1105.0661).  Section numbers below refer to
 * that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are DEVICE pointers owned by the caller.  The library
 *    never frees them and never keeps them after the work queued on `stream`
 *    has completed.  Other pointers are host pointers, read before the call
 *    returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every compute call is asynchronous on that stream: results are ready
 *    once the caller synchronises the stream.
 *  - Every call returns an lbf_status.  On a non-zero status nothing has been
 *    queued and no output has been written; lbf_last_error() returns a text for
 *    the calling thread.  No call aborts, throws or prints.
 *  - Complex values are stored as interleaved (re, im) pairs.
 *  - Symbols: S stations, B tied-array beams, C channels, T time samples per
 *    channel, 2 polarisations (X, Y), K Stokes parameters (1: I, 4: IQUV),
 *    t_int / f_int integration factors, T' = T / t_int, C' = C / f_int.
 */
#ifndef LBF_H
#define LBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBF_OK = 0,
    LBF_E_INVAL = -1,        /* malformed argument (size, NULL, divisibility)     */
    LBF_E_UNSUPPORTED = -2,  /* valid but not implemented (e.g. type combination) */
    LBF_E_NOMEM = -3,        /* does not fit the memory the caller provided       */
    LBF_E_HIP = -4,          /* the HIP runtime reported an error                 */
    LBF_E_BUSY = -5,         /* a bounded queue is full; retry later              */
    LBF_E_NOTFOUND = -6      /* unknown ticket / handle                           */
} lbf_status;

/* station sample type (Section 3: dual-polarisation complex 16-bit samples;
 * 8-bit station mode and complex float32 are also accepted) */
typedef enum { LBF_CI8 = 0, LBF_CI16 = 1, LBF_CF32 = 2 } lbf_input_t;

/* operand type of the weighted sum; accumulation is always FP32 */
typedef enum { LBF_F32 = 0, LBF_F16 = 1, LBF_BF16 = 2 } lbf_compute_t;

/* data product (Section 3: complex voltages, Stokes IQUV, Stokes I) */
typedef enum { LBF_VOLTAGES = 0, LBF_STOKES_I = 1, LBF_STOKES_IQUV = 4 } lbf_product_t;

/* Thread-local text describing the last non-zero status of this thread. */
const char* lbf_last_error(void);

/* Library version string, e.g. "lbf 1.0 gfx950". */
const char* lbf_version(void);

/*
 * Geometric delays and complex weights (Section 3; Section 4.3: each beam's
 * weights depend on the station location, the channel frequency and the beam
 * coordinates), with the sub-sample part of delay compensation (Section 3:
 * once the station series are shifted against each other by whole samples,
 * e.g. by lbf_channelize, the delay that remains is removed by a phase
 * rotation of each sample, which the weights carry):
 *
 *   tau[b][s] = p_s . (u_b - u_ref) / c0 - delta_s   (u_ref = 0 if ref_dir NULL,
 *                                                     delta_s = 0 if d_station_delay NULL)
 *   w[c][b][s] = exp(-2 pi i (m - rint(m))),  m = f_c * tau[b][s]
 *
 * Computed in FP64 on the device, then rounded once (round-to-nearest-even)
 * to the weight type.
 *   d_station_xyz   [S][3] f64, metres (local East-North-Up frame)
 *   d_beam_dir      [B][3] f64, unit direction vectors
 *   ref_dir         HOST [3] f64 or NULL
 *   d_station_delay [S] f64 seconds or NULL: each station's residual delay
 *                   (positive when its signal arrives late); the weight then
 *                   advances that station's phase by 2 pi f_c delta_s.  Exact
 *                   as the residual after a whole-sample shift when the
 *                   subbands are centred on whole multiples of the subband
 *                   sample rate, as a station's polyphase filter bank forms them
 *   d_freq_hz       [C] f64, the channels' sky frequencies
 *   d_w             [C][B][S] complex of wtype (complex f32: 8 bytes; complex
 *                   f16 / bf16: 4 bytes per weight)
 *   d_tau           [B][S] f64 seconds (including -delta_s), or NULL
 * Errors: LBF_E_INVAL for sizes < 1, NULL d_* inputs/outputs, unknown wtype,
 * B*S above 2^30 or C above 2097120.
 */
int lbf_compute_weights(const double* d_station_xyz, int S, const double* d_beam_dir, int B,
                        const double* ref_dir, const double* d_station_delay, const double* d_freq_hz, int C,
                        int wtype, void* d_w, double* d_tau, void* stream);

/*
 * One beam-forming block (Section 4.3): per channel, the weighted complex
 * sum of all station signals into every tied-array beam,
 *   y[c][b][t][p] = sum_s w[c][b][s] x[s][c][t][p],
 * followed for the Stokes products by Stokes detection (Section 4.5),
 * integration over t_int samples and f_int adjacent channels (Section 5.1)
 * and the per-beam, per-Stokes final order (Section 4.6).
 */
typedef struct {
    const void* d_x;   /* [S][C][T][2] complex of xtype                              */
    int xtype;         /* lbf_input_t                                                */
    int S, C, T;
    const void* d_w;   /* [C][B][S] complex of ctype (from lbf_compute_weights)      */
    int ctype;         /* lbf_compute_t: operand type of the contraction             */
    int B;
    int product;       /* lbf_product_t                                              */
    int t_int, f_int;  /* Stokes only: T % t_int == 0, C % f_int == 0; voltages: 1,1 */
    void* d_out;       /* VOLTAGES: complex f32 [C][B][T][2];
                          STOKES:   f32 [B][K][T'][C'] (beam-major final order)       */
} lbf_block;

/*
 * Run one block.  The Stokes products are fused: detection and integration
 * happen in the epilogue of the contraction kernel.  Blocks of at most 64
 * stations with t_int <= 16 (the fast workers) form them channel-major in a
 * staging buffer taken from the device's stream-ordered memory pool, then
 * reorder them into the final order: the same two steps as
 * lbf_beamform_channel_major + lbf_beam_major.  With channel integration
 * (f_int a power of two up to 64) the fast workers stage each channel
 * integrated in time, and the reorder sums each group of f_int channels in
 * channel order.  Other blocks store the final order from the epilogue
 * directly.
 * Errors: LBF_E_INVAL (sizes < 1, NULL pointers, T % t_int, C % f_int,
 * t_int/f_int != 1 for voltages, unknown enums); LBF_E_UNSUPPORTED for a Stokes
 * block whose t_int is not a power of two (use lbf_beamform with VOLTAGES,
 * then lbf_stokes, which accepts any divisor).
 */
int lbf_beamform(const lbf_block* blk, void* stream);

/*
 * lbf_beamform together with the incoherent beam of the same block (Section
 * 3: the station powers summed unweighted, a product formed beside the
 * tied-array beams from the same station data), d_inc laid out as
 * lbf_incoherent's output, f32 [K][T'][C'].  Blocks of at most 128 beams on
 * the FP16/BF16 fast worker (HBM-bound) read the station samples once: the
 * work items of their beam group form the incoherent beam from the sample
 * tile they stage, in FP32 from the operand-type samples (equal to
 * lbf_incoherent up to FP32 rounding when the operand type holds the samples
 * exactly: complex int8, int16 up to 2048 in FP16 and up to 256 in BF16).
 * Other blocks, whose contraction is bound by MFMA work, run lbf_beamform and
 * then lbf_incoherent.  d_out equals lbf_beamform's output bit for bit.
 * Errors: as lbf_beamform; LBF_E_INVAL for voltages, a NULL d_inc or one that
 * overlaps the samples or the output.
 */
int lbf_beamform_incoherent(const lbf_block* blk, float* d_inc, void* stream);

/*
 * lbf_beamform for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result bit for bit, but no call to hipMalloc, hipFree or any other
 * allocating routine.  The Stokes staging (the fast workers' channel-major
 * products before the reorder) comes from a fixed array of
 * LBF_NOALLOC_SCRATCH_BYTES that the library holds in device memory, one per
 * GPU it runs on, until the process ends; a block whose staging is larger
 * runs through it in passes of as many channels as fit.  Every call on one
 * GPU uses that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  Nothing in the
 * array needs to start at any value.
 * Errors: as lbf_beamform; LBF_E_NOMEM when one channel's staging
 * (T' x B x K floats, rows padded to a multiple of 32), times f_int with
 * channel integration on the fast workers, exceeds the array.
 */
#define LBF_NOALLOC_SCRATCH_BYTES (64ull << 20)
int lbf_beamform_noalloc(const lbf_block* blk, void* stream);

/*
 * The same block with the Stokes products left channel-major, the order in
 * which they are formed (each channel's beams together, Section 4.3), before
 * the reorder into the final order (Section 4.6):
 *   d_out  STOKES: f32 [C'][T'][B][K] (each beam's K parameters together, then
 *          the beams);  VOLTAGES: as lbf_beamform.
 * lbf_beam_major of this output equals lbf_beamform's output bit for bit.
 * With channel integration on the fast workers the per-channel products go
 * through staging from the stream-ordered pool, and the f_int channel sums
 * (in channel order, as lbf_beamform's) are written from it.
 * Errors: as lbf_beamform.
 */
int lbf_beamform_channel_major(const lbf_block* blk, void* stream);

/*
 * Reorder channel-major Stokes into the final per-beam order (Section 4.6):
 *   out[b][k][t][c] = in[c][t][b][k],   in f32 [C2][T2][B][K], out f32 [B][K][T2][C2].
 * K = 1 or 4.  in and out must not overlap.  Exact (a permutation).
 * Errors: LBF_E_INVAL for sizes < 1, K not 1 or 4, NULL or overlapping buffers.
 */
int lbf_beam_major(const float* d_in, int C2, int K, int T2, int B, float* d_out, void* stream);

/*
 * Several independent blocks (Section 7: independent observations processed
 * in parallel).  Blocks are grouped by worker variant (input type, product,
 * station count class, beam width); each group runs as ONE launch of a
 * persistent kernel that pulls (block, item) work items from a device queue,
 * so the items of all blocks of a group share the machine.  Blocks outside
 * the batch kernels' path (t_int other than 16, channel integration, more
 * than 64 stations) run through their own launches.  All launches go to
 * `stream`.  Each block's result is bitwise identical to lbf_beamform on that
 * block alone.  All blocks must be Stokes products with one ctype, F16 or
 * BF16.  n <= LBF_MAX_BATCH.  Each call takes the next of 1024 work counters
 * of its device, busy until the call's launches end: calls on one stream are
 * ordered and never collide, but no more than 1024 calls may be outstanding
 * at once on one device across different streams.
 * Errors: as lbf_beamform, per block; LBF_E_INVAL if n < 1 or n > LBF_MAX_BATCH;
 * LBF_E_UNSUPPORTED for voltages, F32 operands or mixed ctypes.
 */
#define LBF_MAX_BATCH 32
int lbf_beamform_batch(const lbf_block* blks, int n, void* stream);

/*
 * Stokes detection + integration of complex voltages (the unfused path,
 * Section 4.5):  I = |X|^2 + |Y|^2, Q = |X|^2 - |Y|^2, U = 2 Re(X conj Y),
 * V = 2 Im(X conj Y), summed over t_int samples and f_int channels.
 *   d_y  complex f32 [C][B][T][2]
 *   d_s  f32 [C'][B][T'][K]    (K = product: 1 or 4)
 * Any t_int dividing T and f_int dividing C is accepted.
 */
int lbf_stokes(const float* d_y, int B, int C, int T, int product, int t_int, int f_int,
               float* d_s, void* stream);

/*
 * Reorder into the final per-beam order (Section 4.6):
 *   out[b][k][t][c] = in[c][b][t][k]
 * for elements of elem_bytes = 4 (f32 Stokes) or 8 (complex f32 voltages,
 * with K = 2 polarisations).  in and out must not overlap.
 */
int lbf_transpose(const void* d_in, int C2, int B, int T2, int K, int elem_bytes, void* d_out,
                  void* stream);

/*
 * Incoherent beam (Section 3): unweighted accumulation of the station powers,
 *   inc[k][t'][c'] = sum over the t_int x f_int group of sum_s Stokes_k(x_s),
 * laid out like one beam of the Stokes product.
 *   d_x [S][C][T][2] complex of xtype;  d_out f32 [K][T'][C']
 */
int lbf_incoherent(const void* d_x, int xtype, int S, int C, int T, int product, int t_int,
                   int f_int, float* d_out, void* stream);

/*
 * Superstation beam forming (Section 4.2: a simplified beam former that
 * combines several stations as if they were one):
 *   out[g][c][t][p] = sum over members s of group g of w[c][s] x[s][c][t][p]
 * summed in member order in FP32.  The members of group g are
 * members[offsets[g] .. offsets[g+1]) (host arrays, offsets[0] = 0, not
 * decreasing; a station may belong to several groups).
 *   d_x   [S][C][T][2] complex of xtype, 16-byte aligned
 *   d_w   complex f32 [C][S] (e.g. lbf_compute_weights with one direction),
 *         or NULL for unit weights
 *   d_out complex f32 [G][C][T][2]: the station-sample layout, so it is a
 *         CF32 input of lbf_beamform with G stations; must not overlap d_x or d_w
 * Errors: LBF_E_INVAL for sizes < 1, an unknown xtype, G outside 1..64, more
 * than 256 members, a member outside 0..S-1, a malformed offsets array, NULL,
 * misaligned or overlapping buffers.
 */
int lbf_superstation(const void* d_x, int xtype, int S, int C, int T, const float* d_w, int G, const int* offsets,
                     const int* members, float* d_out, void* stream);

/*
 * Channeliser (Section 4.2: an FFT divides each subband into channels), with
 * the sample-granularity part of delay compensation (Section 3: station
 * series are shifted against each other by whole samples; the sub-sample part
 * is in the beam former's weights).  Station s contributes the window of T_sb
 * samples that starts d_shift[s] samples into its row (samples outside
 * [0, T_in) read as zero; NULL d_shift: no shift).  Every station's and
 * polarisation's window is cut into consecutive groups of nch samples; the
 * FFT of a group (forward sign exp(-2 pi i j k / nch), no window function, no
 * scaling) gives one sample of each of the subband's nch channels, lowest
 * frequency first: channel q is FFT bin (q + nch/2) mod nch.
 *   d_x     [S][NSB][T_in][2] complex of xtype (re, im interleaved), 16-byte aligned
 *   d_shift device int32 [S] (any values) or NULL
 *   d_out   complex f32 [S][NSB nch][T_sb / nch][2], the layout lbf_beamform
 *           takes as CF32 input (C = NSB nch, T = T_sb / nch); must not
 *           overlap d_x or d_shift
 * nch is a power of two from 2 to 256; T_sb must be a multiple of nch.
 * Errors: LBF_E_INVAL for sizes < 1, an unsupported nch, T_sb not a multiple
 * of nch, an unknown xtype, NULL, misaligned or overlapping buffers, or a grid
 * of more than 2^31 - 1 work groups.
 */
int lbf_channelize(const void* d_x, int xtype, int S, int NSB, int T_in, int T_sb, int nch, const int* d_shift,
                   float* d_out, void* stream);

/*
 * Channel-level dedispersion (Section 4.4): each polarisation's beam voltages
 * are cut into blocks of n_fft consecutive samples; each block is Fourier
 * transformed (forward sign exp(-2 pi i j k / n_fft)), multiplied bin by bin
 * with its channel's precomputed chirp weights, and transformed back with a
 * 1/n_fft factor, so all-one weights return the input.
 *   d_y     complex f32 [C][B][T][2]   (lbf_beamform VOLTAGES layout)
 *   d_chirp complex f32 [C][n_fft]     (bin k at index k; the same for every beam)
 *   d_out   complex f32 [C][B][T][2];  may equal d_y (in place), must not
 *           otherwise overlap it
 * n_fft is 8, 64, 512 or 4096 (the paper's 3 Hz subchannels of a 12 kHz
 * channel); T must be a multiple of n_fft.  Device buffers, caller-owned,
 * 16-byte aligned.  The chirp is read only.
 * Errors: LBF_E_INVAL for sizes < 1, an unsupported n_fft, T not a multiple
 * of n_fft, NULL, misaligned or partly overlapping buffers, or more than
 * 2^31 - 1 blocks (C B T / n_fft).
 */
int lbf_dedisperse(const void* d_y, int C, int B, int T, int n_fft, const void* d_chirp, void* d_out,
                   void* stream);

/*
 * Channel-level dedispersion (Section 4.4) followed by Stokes detection
 * (Section 4.5) and integration over t_int consecutive samples, in one pass:
 * the dedispersed voltages stay on chip.  Equals lbf_dedisperse and then
 * lbf_stokes (f_int = 1) up to FP32 rounding.
 *   d_y     complex f32 [C][B][T][2];  d_chirp complex f32 [C][n_fft]
 *   d_s     f32 [C][B][T'][K], T' = T / t_int (the layout of lbf_stokes;
 *           lbf_transpose gives the final order); must not overlap d_y or d_chirp
 * n_fft as lbf_dedisperse; product STOKES_I or STOKES_IQUV; t_int a power of
 * two up to min(n_fft, 64 max(1, n_fft / 256)) (1024 at n_fft = 4096).
 * Errors: LBF_E_INVAL for sizes < 1, an unsupported n_fft, product or t_int,
 * T not a multiple of n_fft, NULL, misaligned or overlapping buffers, or more
 * than 2^31 - 1 blocks.
 */
int lbf_dedisperse_stokes(const void* d_y, int C, int B, int T, int n_fft, const void* d_chirp, int product,
                          int t_int, float* d_s, void* stream);

/*
 * Peak probes, for reporting the kernels' rooflines against what this device
 * sustains beside the datasheet figures (not part of the beam former).
 *   kind 0: a register-only loop of MFMA 32x32x16 f16 (the FP16 contraction's
 *           instruction), two 256-thread work groups per compute unit,
 *           `iters` iterations of 8 independent MFMAs per wave; *work = flop.
 *   kind 1: the same with MFMA 32x32x2 f32; *work = flop.
 *   kind 2: a 16-byte copy of `bytes` (rounded down to 16) from d_src to
 *           d_dst (device buffers, not overlapping); *work = bytes moved
 *           (read + write).
 *   kind 3: a 16-byte read stream of `bytes` (rounded down to 16) of d_src;
 *           *work = bytes read.  d_dst (at least 1024 bytes) takes at most a
 *           word per thread index, where the xor of a thread's data equals a
 *           fixed key.
 * d_dst must be a device buffer of at least 1024 bytes for kinds 0, 1 and 3
 * (kinds 0 and 1 never write it).  The caller times the call with events on `stream`.
 * Errors: LBF_E_INVAL for an unknown kind, iters < 1, NULL pointers or
 * bytes < 16 for a copy or a read.
 */
int lbf_probe(int kind, int iters, const void* d_src, void* d_dst, uint64_t bytes, double* work, void* stream);

/*
 * Host-side check of the fast workers' memory addressing (no device access,
 * not part of the beam former): walks every buffer access their kernels make
 * for this block -- weight, sample and output descriptors and every 32-bit
 * offset, with the kernels' own address arithmetic -- and returns LBF_OK when
 * every descriptor lies inside its buffer, no offset wraps and every store the
 * epilogue means to make lands inside its descriptor; otherwise LBF_E_INVAL
 * with the first offending access in lbf_last_error().  channel_major: as
 * lbf_beamform_channel_major, else as lbf_beamform, whose Stokes go through
 * staging of staging_cap bytes in channel passes (0: the whole block at once).
 * Blocks the fast workers do not take check as LBF_OK with no access.  The
 * buffers are sized from the block; its pointers are not dereferenced (any
 * non-NULL value).  threads: host threads for the walk (1..64).
 * *accesses (may be NULL) receives the number of accesses walked.
 */
int lbf_check_addressing(const lbf_block* blk, int channel_major, uint64_t staging_cap, int threads,
                         uint64_t* accesses);

/*
 * Tuning hook (not part of the beam former): the tile shape of the FP16/BF16
 * fast worker's work items -- 1, 2 or 4 sample streams, i.e. items of 256,
 * 128 or 64 beams -- comes from a table measured per input type, station
 * count and beam count (tiles.json, compiled into the library).  streams = 1,
 * 2 or 4 forces that shape for every later call in this process (complex f32
 * samples keep 1); 0 restores the table.  For the sweep that measures the
 * table; it changes only speed, never results.  Each call reads the setting
 * once, when it starts, so a call that runs on another thread meanwhile takes
 * the old setting or the new one throughout.
 * Errors: LBF_E_INVAL for other values.
 */
int lbf_set_tile_streams(int streams);

/* Bytes of each operand of a block (host arithmetic, no device access). */
typedef struct {
    uint64_t input_bytes, weight_bytes, output_bytes;
    double flops;          /* 8 flops per complex multiply-add, both polarisations */
    uint64_t staging_bytes;          /* Stokes staging lbf_beamform takes for the whole block
                                        (the channel-major products before the reorder, one row
                                        per channel before any channel sums); 0 if none        */
    uint64_t staging_channel_bytes;  /* the same for one channel (a channel pass needs f_int of
                                        them with channel integration)                        */
} lbf_block_sizes;
int lbf_block_footprint(const lbf_block* blk, lbf_block_sizes* out);

/* ------------------------------------------------------------------------ */
/* Streaming server (Section 4.1: the station stream is cut into blocks;
 * Section 7: independent observations run in parallel as long as resources
 * allow).  Jobs are queued on the host, admitted when their device footprint
 * fits the caller's arena and an in-flight slot is free, and run on a pool of
 * HIP streams; several admitted jobs are batched as in lbf_beamform_batch.
 * Weights are cached on the device per observation id.                     */

typedef struct lbf_server lbf_server;

typedef struct {
    void* d_arena;            /* caller-owned device memory the server sub-allocates */
    uint64_t arena_bytes;
    int max_inflight;         /* jobs on the device at once (>= 1)                  */
    int n_streams;            /* HIP streams in the pool (>= 1, default priority)   */
    int queue_capacity;       /* host queue bound (>= 1); submit returns BUSY beyond */
    int max_batch;            /* jobs fused per launch (1..LBF_MAX_BATCH)            */
    int device;               /* HIP device ordinal                                  */
    uint64_t staging_cap;     /* most arena bytes one job's Stokes staging takes (the
                                 fast workers' channel-major products before the
                                 reorder; a larger block runs in channel passes);
                                 0: 256 MiB.  Counted in the job's footprint.       */
} lbf_server_cfg;

typedef struct {
    uint64_t obs_id;          /* weight-cache key: same geometry and frequencies     */
    const double* station_xyz; int S;   /* HOST [S][3] f64, copied at submit         */
    const double* beam_dir; int B;      /* HOST [B][3] f64, copied at submit         */
    const double* ref_dir;              /* HOST [3] f64 or NULL                      */
    const double* station_delay;        /* HOST [S] f64 residual delays (s) or NULL,
                                           copied at submit; part of the observation's
                                           geometry (the weight-cache key)           */
    const double* freq_hz; int C;       /* HOST [C] f64, copied at submit            */
    const void* x; int xtype; int T;    /* station samples [S][C][T][2]              */
    int x_on_host;            /* 1: x is HOST memory, copied into the arena;
                                 0: x is device memory valid until the job is DONE  */
    int ctype, product, t_int, f_int;
    void* d_out;              /* caller-owned device output, layout as lbf_beamform  */
    uint64_t stream_id;       /* 0: an independent block.  Otherwise the blocks of one
                                 stream are consecutive in time and are run in
                                 submission order; integration periods may span
                                 blocks (T % t_int need not be 0): the samples of an
                                 incomplete period at the end of a block stay on the
                                 device and are prepended to the stream's next
                                 block, so d_out receives the periods completed in
                                 this block, [B][K][P][C'] with
                                 P = (carried + T) / t_int (lbf_job_status.periods);
                                 the result equals lbf_beamform on the stream's
                                 samples concatenated in time.  Stokes products,
                                 device-resident x only; S, C, xtype and t_int
                                 stay those of the stream.  Arena use: a tail of
                                 S*C*(t_int-1) samples while samples are carried,
                                 and, for a block that carries in or out, its
                                 S*C*P*t_int samples concatenated for the kernel.
                                 A stream that ends on a period boundary releases
                                 its tail and its id; a failed block fails every
                                 later block of its stream (use a new id).        */
} lbf_job;

typedef enum { LBF_JOB_QUEUED = 0, LBF_JOB_ADMITTED = 1, LBF_JOB_RUNNING = 2, LBF_JOB_DONE = 3,
               LBF_JOB_FAILED = 4 } lbf_job_state;

typedef struct {
    int state;                /* lbf_job_state                                         */
    int error;                /* lbf_status of a FAILED job                            */
    uint64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns;  /* steady clock, ns       */
    int batch_size;           /* jobs in the launch that ran this job                  */
    int periods;              /* integration periods written to d_out (T' of the block) */
} lbf_job_status;

/* Errors: LBF_E_INVAL for a malformed cfg; LBF_E_HIP if the device or streams
 * cannot be set up. */
int lbf_server_create(const lbf_server_cfg* cfg, lbf_server** out);

/* Non-blocking.  LBF_E_INVAL for a malformed job (or a stream block whose S, C,
 * xtype or t_int differ from its stream's), LBF_E_NOMEM if its footprint
 * (weights, host-sample staging, stream carry, Stokes staging) can never fit
 * the arena or one channel's Stokes staging exceeds staging_cap, LBF_E_BUSY if the host queue is full, LBF_E_HIP for a
 * block of a stream an earlier block of which failed. */
int lbf_server_submit(lbf_server* srv, const lbf_job* job, uint64_t* ticket);

/* LBF_E_NOTFOUND for an unknown ticket.  A DONE/FAILED ticket stays
 * queryable until lbf_server_release. */
int lbf_server_poll(lbf_server* srv, uint64_t ticket, lbf_job_status* st);

/* Block until the ticket is DONE or FAILED (or timeout_ms elapses: LBF_E_BUSY). */
int lbf_server_wait(lbf_server* srv, uint64_t ticket, int timeout_ms, lbf_job_status* st);

/* Forget a finished ticket. */
int lbf_server_release(lbf_server* srv, uint64_t ticket);

/* Drain all queued and running jobs, then free the server's own state (never
 * the caller's arena or outputs). */
int lbf_server_destroy(lbf_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* LBF_H */
