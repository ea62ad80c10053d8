/*
 * hot.h -- C ABI of the MI355X hologram solver for holographic optical tweezers.
 *
 * Method: S. Bianchi and R. Di Leonardo, "Real-time optical micro-manipulation
 * using optimized holograms generated on the GPU" (arXiv:0907.4027).
 *   Eq. 1  V_m   = (1/N) sum_j exp(i (phi_j - Delta_j^m))          field at trap m
 *   Eq. 2  Delta = z_m pi/(lambda f^2) (x_j^2 + y_j^2) + 2 pi/(lambda f) (x_j x_m + y_j y_m)
 *   Eq. 3  phi_j = arg sum_m w_m exp(i (Delta_j^m + theta_m))       (w_m = 1: random superposition)
 *   Section 3  e = sum_m |V_m|^2,  u = 1 - (max I - min I)/(max I + min I),  I_m = |V_m|^2
 *   Section 3 / Fig. 2  GSW: w_m <- w_m <|V|>/|V_m|, theta_m <- arg V_m, repeat.
 *
 * Conventions shared by every entry point
 *   Units      SI metres for pitch, wavelength, focal length and trap positions;
 *              phases in radians.
 *   Pixels     phase masks are row-major float arrays [ny][nx]; pixel j = r*nx + c
 *              sits at x = (c - (nx-1)/2) * pitch, y = (r - (ny-1)/2) * pitch
 *              (origin on the optical axis, every pixel counts, x along columns).
 *   Output     phases in [0, 2 pi] (float rounding can return 2 pi itself);
 *              V as interleaved (re, im) float pairs.
 *   Precision  FP32 on the device; per-trap coefficients are formed in FP64 on
 *              the host and rounded once.  Inside the iterative solvers the per-block
 *              trap sums of Eq. 1 are rounded to fixed point, 2^-30 in units of V
 *              (re and im as 32-bit integers packed into one 64-bit atomic add), so
 *              V does not depend on the order in which blocks finish and every run
 *              is bitwise reproducible; the rounding adds at most 2^-31 per block and
 *              component to V (2.4e-7 over the 512 blocks of a 512 x 512 mask).
 *   Ownership  the caller owns every buffer passed in and out.  "device" pointers
 *              are device memory on the context's GPU (e.g. torch data_ptr());
 *              "host" pointers are ordinary CPU memory.  The library allocates
 *              only inside the context and never frees caller memory.
 *   Ordering   all device work is enqueued on the context's stream.  A call that
 *              is given a host `stats` pointer synchronises that stream before it
 *              returns; otherwise it returns as soon as the work is enqueued.
 *   Errors     every int-returning call returns HOT_OK (0) or a negative code;
 *              hot_last_error() then describes the failure (thread-local).  All
 *              argument checks run on the host before any device work, so on an
 *              error no output has been touched.  HOT_EDEGENERATE (every |V_m| = 0
 *              during GSW/GS) is detected on the device and reported by the call
 *              that synchronises (a call with `stats`, or hot_sync()).
 *   Threads    a context may be used by one host thread at a time; calls that
 *              overlap on one context race.
 */
#ifndef HOT_H
#define HOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOT_ABI_VERSION 1
#define HOT_MAX_TRAPS 2048  /* per hologram */
#define HOT_MAX_SIDE 4096   /* nx, ny */
#define HOT_MAX_BATCH 4096  /* holograms per batched call */

typedef struct hot_ctx hot_ctx;

/* SLM pixel grid and optics (Section 3, Fig. 1: SLM in the back focal plane). */
typedef struct hot_slm {
  int32_t nx, ny;     /* columns (x) and rows (y), 1..HOT_MAX_SIDE */
  double pitch;       /* pixel pitch [m], > 0 */
  double wavelength;  /* lambda [m], > 0 */
  double focal;       /* effective focal length f [m], > 0 */
} hot_slm;

/* Per-iteration figures of merit (Section 3): efficiency e, uniformity u, and
 * sigma = std(I)/mean(I) with the population standard deviation. */
typedef struct hot_stats {
  float efficiency, uniformity, sigma;
} hot_stats;

enum hot_status {
  HOT_OK = 0,
  HOT_EINVAL = -1,      /* bad argument (null pointer, size or value out of range, non-finite) */
  HOT_ENOMEM = -2,      /* device or pinned-host allocation failed */
  HOT_EDEVICE = -3,     /* no usable GPU, or a HIP runtime call failed */
  HOT_EDEGENERATE = -4  /* GSW/GS met <|V|> = 0: the phase mask sends no light to any trap */
};

/* How the propagation phase Delta is obtained inside the two passes. */
enum hot_variant {
  HOT_ONTHEFLY = 0, /* Delta recomputed per (pixel, trap) with FP32 sin/cos (default) */
  HOT_STORED = 1,   /* exp(i Delta) precomputed once as a complex64 [M][N] matrix, then two GEMV-shaped passes */
  HOT_SEPARABLE = 2 /* exact factorisation of Eq. 2, exp(i Delta) = X_m(column) Y_m(row): both passes become
                       dense complex contractions on the FP32 matrix cores, fused into one kernel per
                       iteration, with O((nx+ny) M) tables; also used by the batched, Eq. 1 and adjoint calls */
};

/* ---- context ------------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  `stream` is the hipStream_t to enqueue on
 * (e.g. torch.cuda.current_stream().cuda_stream); NULL means the device's default
 * (null) stream, which is also torch's default stream.  Returns HOT_EDEVICE when no
 * GPU is present. */
int hot_create(hot_ctx** out, int device, void* stream);
int hot_destroy(hot_ctx* ctx);
/* Switch the stream later calls enqueue on (NULL: the default stream). */
int hot_set_stream(hot_ctx* ctx, void* stream);
/* Select HOT_ONTHEFLY, HOT_STORED or HOT_SEPARABLE for later calls (hot_rs, hot_gs, hot_gsw;
 * HOT_SEPARABLE also for hot_gsw_batched, hot_forward_V and hot_adjoint, which otherwise
 * use the on-the-fly kernels). */
int hot_set_variant(hot_ctx* ctx, int variant);
/* Launch-shape knobs (used by the autotuner; 0 restores the built-in choice, except
 * HOT_TUNE_GRAPHS).  They change how work is tiled or launched, never what is computed
 * beyond FP32 summation order. */
enum hot_tuning_key {
  HOT_TUNE_PIXELS_PER_LANE = 1, /* fused iteration kernel: pixels per lane, 1 or 2 */
  HOT_TUNE_TRAPS_PER_LANE = 2,  /* trap pass: traps each lane accumulates: 1..6 or 8 */
  HOT_TUNE_SEGMENT = 3,         /* pixels of a row per block, 64..1024, for the fused iteration kernel
                                   and the stand-alone trap pass (built-in: 256 pixels for the fused
                                   kernel on holograms of 64 traps or more, one at a time or in a
                                   batch whose 512-pixel grid would give fewer than four blocks per
                                   compute unit, else 512; 256 for the trap pass) */
  HOT_TUNE_SLICES = 4,          /* trap pass: at most this many pixel slices per wave, 1..16 */
  HOT_TUNE_GRAPHS = 5,          /* 1 (default): replay a captured hipGraph of a solve's launch
                                   sequence when shapes and buffers repeat; 0: launch eagerly */
  HOT_TUNE_SEP_WAVES = 6,       /* separable variant: tiles of 16 x 16 pixels per block (1, 2 or 4),
                                   one or two waves each (HOT_TUNE_SEP_SPLIT) */
  HOT_TUNE_SEP_CHUNK = 7,       /* separable variant: traps whose tables a block holds in LDS at
                                   once, a multiple of 16 (more are streamed in chunks of this size) */
  HOT_TUNE_ROWS = 8,            /* on-the-fly iteration kernel: rows per block, 1 or 2 (two rows share
                                   one GS/GSW update and one set of trap-sum additions; 256-thread
                                   rows only) */
  HOT_TUNE_SEP_SPLIT = 9,       /* separable iteration: waves per 16 x 16 tile, 1 or 2 (two take half
                                   of the traps each and add their pixel sums in a fixed order;
                                   default: two when the grid has at most one block per compute
                                   unit, else one) */
  HOT_TUNE_FRACT = 10           /* direct passes: 1 reduces every per-term phase argument to one period
                                   explicitly (one more instruction per term); 0 (default) does so
                                   only when an argument could leave the hardware sin/cos domain */
};
int hot_set_tuning(hot_ctx* ctx, int key, int value);

/* Wait for the context's stream; returns HOT_EDEGENERATE if a GSW/GS run enqueued
 * since the last synchronising call met <|V|> = 0 (and clears the flag). */
int hot_sync(hot_ctx* ctx);

/* Host-only check of a problem description (no device work, usable without a GPU):
 * slm fields, 1 <= M <= HOT_MAX_TRAPS, xyz finite (host M x 3), iters >= 0. */
int hot_check_problem(const hot_slm* slm, int32_t M, const double* xyz, int32_t iters);

/* ---- single hologram ---------------------------------------------------------------- */

/* Random superposition, Eq. 3 with w_m = 1 (Section 3; Section 4 "SR holograms").
 *   xyz     host, M x 3 trap positions (x_m, y_m, z_m) [m]
 *   theta0  host, M trap phases [rad]; NULL draws them from `seed` with SplitMix64
 *           (theta_m = 2 pi (z >> 40) 2^-24 for the m-th output z)
 *   phase   device, N = nx*ny floats, out: phi_j
 *   V       device, 2M floats, out: V_m of the mask (Eq. 1)
 *   stats   host, 1 entry or NULL */
int hot_rs(hot_ctx* ctx, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
           uint64_t seed, float* phase, float* V, hot_stats* stats);

/* Gerchberg-Saxton: GSW below without the weight update (w_m = 1 throughout).
 *   stats   host, iters+1 entries or NULL: entry k describes V of the k-th mask. */
int hot_gs(hot_ctx* ctx, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
           uint64_t seed, int32_t iters, float* phase, float* V, hot_stats* stats);

/* Weighted Gerchberg-Saxton (Section 3, Fig. 2), `iters` = K iterations:
 *   w = w0 (or 1), theta = theta0, phi = backward(w, theta);
 *   K times: V = forward(phi) -> stats[k]; w_m <- w_m <|V|>/|V_m|; theta_m <- arg V_m;
 *            phi = backward(w, theta);
 *   finally V = forward(phi) -> stats[K].
 *   w0         device, M floats or NULL (all 1): warm start
 *   w_out      device, M floats or NULL: the weights that produced the final phase
 *   theta_out  device, M floats or NULL: the trap phases that produced the final phase
 * Passing (theta_out, w_out) of a K1-iteration call back as (theta0, w0) and running K2
 * more iterations reproduces a single K1+K2 call bit for bit. */
int hot_gsw(hot_ctx* ctx, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
            uint64_t seed, int32_t iters, const float* w0, float* w_out, float* theta_out,
            float* phase, float* V, hot_stats* stats);

/* Allocation-free GSW, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as hot_gsw, computed by the same on-the-fly kernels (whatever the context's variant) and
 * launched eagerly; bit for bit the result of hot_gsw with the context's launch shape.  It calls
 * no hipMalloc, hipFree or other allocating routine: every device table, state, trap sum,
 * statistic and flag it needs lives in a fixed 1 MiB workspace per GPU (a file-scope device array
 * whose address hot_create looks up), and its host tables go through a pinned staging buffer that
 * hot_create allocates.  Limit: the workspace holds M traps and `iters` iterations when its six
 * regions, 32 M (coefficients) + 32 M (state) + 64 (descriptors) + 192 M (trap sums) +
 * 12 (iters + 1) (statistics) + 4 (flag) bytes, each rounded up to a multiple of 256, total at most
 * 1 MiB: 2048 traps with up to 43000 iterations, 100 traps with up to 85000; larger requests fail
 * with HOT_EINVAL before any device work.  HOT_EDEGENERATE is reported when `stats` is given.  Every call on one GPU shares that GPU's workspace, which keeps the last call's
 * contents (the call clears what must start at zero): calls that overlap on one GPU, from any
 * contexts or streams, race and must not be issued. */
int hot_gsw_noalloc(hot_ctx* ctx, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
                    uint64_t seed, int32_t iters, const float* w0, float* w_out, float* theta_out,
                    float* phase, float* V, hot_stats* stats);

/* ---- batches of holograms sharing one SLM ------------------------------------------- */

/* B independent GSW problems in one launch sequence.  Hologram b has M[b] traps; traps
 * are concatenated in order (offset_b = M[0] + ... + M[b-1], total T = sum M).
 *   M       host, B counts, each 1..HOT_MAX_TRAPS
 *   xyz     host, T x 3;  theta0 host, T [rad] (required)
 *   phase   device, B x N floats;  V device, 2T floats
 *   stats   host, B x (iters+1) entries (hologram-major) or NULL
 * Each hologram's result matches hot_gsw on that hologram alone within the parity tolerance, and
 * bit for bit when both runs use the same launch shape (hot_set_tuning): the launch shape is
 * otherwise chosen per launch, and with it the order of each block's floating-point trap sums. */
int hot_gsw_batched(hot_ctx* ctx, const hot_slm* slm, int32_t B, const int32_t* M, const double* xyz,
                    const double* theta0, int32_t iters, float* phase, float* V, hot_stats* stats);

/* Eq. 1 for B given masks: V of hologram b from phase[b] (device, B x N) -> V (device, 2T). */
int hot_forward_V(hot_ctx* ctx, const hot_slm* slm, int32_t B, const int32_t* M, const double* xyz,
                  const float* phase, float* V);

/* Adjoint of Eq. 1: for a real loss L(V) and G_m = dL/dRe V_m + i dL/dIm V_m (device, 2T),
 *   grad_phase[b][j] = dL/dphi_j = (1/N) Im( exp(-i phi_j) sum_m G_m exp(i Delta_j^m) ),
 * with Delta recomputed (never stored).  phase device B x N, grad_phase device B x N. */
int hot_adjoint(hot_ctx* ctx, const hot_slm* slm, int32_t B, const int32_t* M, const double* xyz,
                const float* phase, const float* G, float* grad_phase);

/* ---- SLM output ----------------------------------------------------------------------- */

/* 8-bit SLM frame (Section 5: each grey level maps linearly onto a phase from 0 to 2 pi):
 *   frame[j] = rint(phase[j] * 256 / (2 pi)) mod 256,
 * with the product taken in FP32 (FP32(256 / (2 pi)) times the FP32 phase, rounded to
 * nearest even), so a phase of 2 pi encodes as 0.  phase: device, n floats (radians, as
 * written by the solvers); frame: device, n bytes.  Asynchronous on the context's stream. */
int hot_encode_u8(hot_ctx* ctx, int64_t n, const float* phase, uint8_t* frame);

/* ---- diagnostics ---------------------------------------------------------------------- */

/* Measurement aid for benchmarks and profilers: for the single-hologram problem given,
 * launches four groups of kernels `reps` times each, back to back on the context's stream
 * (current variant and tuning), each group bracketed by HIP events, and writes the mean
 * device time per launch in milliseconds to
 *   ms[0]  one GSW iteration's main work (on-the-fly: the fused update + pixel pass + trap pass
 *          kernel, which also sums the trap pass into V's fixed-point accumulators; separable:
 *          the fused update + both passes on the matrix cores; stored: the pixel and trap
 *          pass kernels)
 *   ms[1]  the reduction into V (stored: of the per-block partials, once per iteration;
 *          on-the-fly and separable: of the fixed-point accumulators, once per solve)
 *   ms[2]  the pixel pass alone   ms[3]  the trap pass alone
 * phase (device, N floats) and V (device, 2M floats) are scratch outputs.  Synchronises
 * the stream. */
int hot_time_passes(hot_ctx* ctx, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
                    int32_t reps, float* phase, float* V, float* ms);

/* Ablation of the pixel pass's design choices (the paper's rules of Section 2, measured in its
 * Table 1, Section 4), for the random-superposition pass: Eq. 3 with w_m = 1 and theta0 (host, M
 * radians), written to `phase` (device, nx*ny floats).  `placement` says where each thread finds
 * the per-trap records: HOT_REC_LDS (staged in LDS, read as broadcasts), HOT_REC_SCALAR (read from
 * global memory through the scalar cache, one load per wave), HOT_REC_GLOBAL (read from global
 * memory by every lane); `mapping` how pixels map to a block of `block` threads (64 or 256):
 * HOT_MAP_LINEAR (consecutive pixels of a row) or HOT_MAP_SQUARE (a square tile, 8x8 or 16x16:
 * one more FMA per term, as the row varies inside a block).  Records are formed once per block in
 * FP64 (a small table the context holds), then the pass is launched `reps` times back to back;
 * ms[0] gets the mean device milliseconds per launch.  Synchronises the context's stream. */
enum hot_record_placement { HOT_REC_LDS = 0, HOT_REC_SCALAR = 1, HOT_REC_GLOBAL = 2 };
enum hot_pixel_mapping { HOT_MAP_LINEAR = 0, HOT_MAP_SQUARE = 1 };
int hot_pixel_pass_variant(hot_ctx* ctx, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
                           int placement, int mapping, int block, int32_t reps, float* phase, float* ms);

/* Measurement aid: issue rate of the FP32 vector pipes that bound the direct passes.  Launches
 * one block of 4 * waves_per_simd waves per compute unit (waves_per_simd 1, 2, 4 or 8), each wave
 * running `reps` repetitions (1..2^24) of an unrolled instruction stream of one kind:
 *   kind 0  FP32 FMA (128 per repetition, 8 independent chains)
 *   kind 1  hardware sin/cos (128 per repetition, 8 independent chains)
 *   kind 2  the term of the direct passes (16 per repetition): two FMAs form the phase
 *           (Eq. 2 in revolutions), sin and cos, two FMAs accumulate (plus one add per repetition)
 *   kind 3  FP32 matrix products 16x16x4, four independent accumulators per wave
 *   kind 4  FP32 matrix products 16x16x4, one accumulator (each product waits for the last)
 *   kind 5  FP32 matrix products 32x32x2, four independent accumulators per wave
 *   kind 6  kind 3's products with 64 hardware sin/cos beside them per 16 products (FLOPs of the
 *           products counted): whether the two pipes overlap
 * after a short warm-up launch.  Writes, to host `out` (6 doubles):
 *   out[0] operations per second: lane-level FMAs (kind 0), sin/cos (kind 1), terms (kind 2) or
 *          FLOPs (kinds 3-6),
 *          over the span from the first wave's start to the last wave's end (s_memrealtime,
 *          100 MHz); out[1] mean shader clock of the waves [Hz] (s_memtime cycles over the same
 *          waves' real time); out[2] that span [s]; out[3] the launch's duration by HIP events [s];
 *   out[4] mean shader cycles per wave; out[5] number of waves.
 * Synchronises the context's stream; uses a small device buffer held by the context. */
int hot_probe_issue(hot_ctx* ctx, int kind, int waves_per_simd, int64_t reps, double* out);

/* Measurement aid: device memory bandwidth.  Copies `bytes` (a positive multiple of 16) from
 * device `src` to device `dst` (not overlapping) `reps` times (1..1000) after one untimed copy,
 * with a kernel of 16-byte vector loads and stores.  Writes to host `out` (2 doubles): out[0]
 * bytes read plus bytes written per second, out[1] ms per copy (HIP events).  Synchronises. */
int hot_probe_copy(hot_ctx* ctx, const void* src, void* dst, int64_t bytes, int reps, double* out);

/* Message for the last non-OK return on this thread ("" if none). */
const char* hot_last_error(void);
int hot_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HOT_H */
