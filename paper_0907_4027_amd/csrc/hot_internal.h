// hot_internal.h -- device data layout and kernel launchers shared by hot_kernels.hip
// and hot_api.cpp (the C ABI).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hot {

// Phases inside the kernels are in revolutions (1 rev = 2 pi rad), which makes the
// reduction of a phase to one period exact (fract of an FP32 value is exact) and
// matches the input convention of the hardware sin/cos (sin(2 pi x)).
//
// Pixel coordinates are carried as exact integers:
//   U_c = 2c - (nx-1),  V_r = 2r - (ny-1)  (so x = U pitch / 2, y = V pitch / 2),
// and Eq. 2 divided by 2 pi becomes  Delta_rev = g (U^2 + V^2) + a U + b V  with
//   a = pitch x_m / (2 lambda f),  b = pitch y_m / (2 lambda f),  g = pitch^2 z_m / (8 lambda f^2).
// Since U and V are integers, a and b matter only modulo 1 (the host reduces them, exactly).
//
// Per-block reference.  A block of the direct passes covers pixels U = Uc + u of one row V, with
// Uc the (integer) centre of its pixels and u = U - Uc even; there
//   Delta_rev = g u^2 + a' u + K,   a' = a + 2 g Uc (mod 1/2),   K = g (Uc^2 + V^2) + a Uc + b V (mod 1).
// a' and K are formed once per (trap, block) in FP64 from the FP64 coefficients and rounded once
// to FP32, so the per-term FP32 argument g u^2 + a' u + K stays small (|u| <= the block's width
// in U units) and the pixel pass (Eq. 3) and the trap pass (Eq. 1) see the same a' and K.

// Per-trap constant coefficients, formed in FP64 on the host (a, b reduced to [-1/2, 1/2)).
struct alignas(16) TrapCoef {
  double a, b, g;  // revolutions per pixel-index unit, as above
  float gf;        // g rounded to FP32: the lens coefficient of the per-term argument
  float pad;
};
static_assert(sizeof(TrapCoef) == 32, "TrapCoef is two 16-byte words");

// Per-trap iteration state, rewritten on the device by the weight/phase update.
struct alignas(16) TrapState {
  float theta_rev;  // theta_m / (2 pi), FP32 product of theta_rad and FP32(1/(2 pi))
  float w;          // GSW weight
  float theta_rad;  // theta_m in radians (what the caller sees)
  float pad;
};

// Per-hologram launch description for batched problems (device array, one per hologram).
struct alignas(16) HoloDesc {
  int32_t m;      // traps in this hologram
  int32_t off;    // offset of its first trap in the concatenated tables
  int32_t g;      // trap pass: trap lanes per slice
  int32_t a;      // trap pass: slices per wave
  int32_t tpl;    // trap pass: traps per lane per chunk (the launch's TPL)
  int32_t pad0, pad1, pad2;
};

constexpr int kTplMax = 8;     // traps per lane in the trap pass: 1..6 or 8
constexpr int kBlock = 256;    // threads of the stand-alone pass kernels
constexpr int kMaxTraps = 2048;
constexpr int kSegMax = 512;   // pixels of a row per stand-alone trap-pass block
constexpr int kLdsMax = 160 * 1024;  // LDS of one compute unit (one block may use all of it)

// Spans: a block's row segment is referenced 256 pixels at a time (hot_kernels.hip), so the
// per-term |u| stays <= kSpan.  The trap pass keeps its pixels in LDS span by span, kSpanStride
// float4 per span (slices cover < len + 64 entries, plus the read-ahead).
constexpr int kSpan = 256;
constexpr int kSpanStride = kSpan + 64 + 4;
// Pixel-pass records: M records, then zeros up to a multiple of kTrapChunk plus one more chunk.
constexpr int kTrapChunk = 4;
__host__ __device__ constexpr int rec_pad(int m) { return (m + 2 * kTrapChunk - 1) / kTrapChunk * kTrapChunk; }
__host__ __device__ constexpr int k_stride(int mmax) { return (mmax + 3) / 4 * 4; }
// Dynamic LDS of the direct passes: per (row, span) pair rec_pad(mmax) float4 records and
// k_stride(mmax) floats K.
inline size_t refs_lds_bytes(int rows_spans, int mmax) {
  return (size_t)rows_spans * (16 * (size_t)rec_pad(mmax) + 4 * (size_t)k_stride(mmax));
}
// Static LDS of the fused iteration kernel and of the stand-alone trap pass.
inline size_t iter_static_lds(int nt, int q, int tpl, int rows) {
  const int hs = nt * q / kSpan, w = nt / 64;
  return (size_t)rows * hs * kSpanStride * 16 + (size_t)rows * w * 64 * tpl * 8 + 8 * (size_t)nt * rows / 64 * 4;
}
inline size_t forward_static_lds(int tpl, int hs) {
  return (size_t)hs * kSpanStride * 16 + (size_t)(kBlock / 64) * 64 * tpl * 8;
}
constexpr int kStoredPpl = 8;  // stored variant: pixels per lane of the trap pass
inline int stored_nblk(int n) { return (n + 64 * kStoredPpl - 1) / (64 * kStoredPpl); }

// Row-segment tiling of the trap pass (and of the fused iteration kernel).
struct FwdGeom {
  int nx, ny;
  int seg_w;  // pixels per row segment (block)
  int nseg;   // segments per row
  int nblk() const { return nseg * ny; }
};

// One fused iteration: (optional GS/GSW update) -> pixel pass -> trap pass, its sums added to acc_out.
// Direct path: each iteration launch adds its per-block trap sums, as 64-bit fixed point, into
// kAccRegions regions (one per XCD of an MI355X; waves of XCD x use region x & 7), laid out
// [region][trap], one 64-bit word per trap (re and im packed, pack_sum in hot_kernels.hip); three
// such buffers rotate over the iterations.
constexpr int kAccRegions = 8;

struct IterArgs {
  FwdGeom fg;
  int B = 1;
  int nt = 256, q = 1, tpl = 1;  // threads per row (256/512), pixels per lane (1/2), traps per lane
  int rows = 1;                  // rows per block: 1, or 2 (nt = 256 only)
  int mmax = 1;                  // most traps of any hologram of the launch (sizes the LDS)
  HoloDesc one{};                // B == 1: the hologram's descriptor (one.m > 0), passed by value
  bool fract = false;
  const TrapCoef* coef = nullptr;
  const HoloDesc* hd = nullptr;
  const TrapState* st_in = nullptr;
  TrapState* st_out = nullptr;
  const unsigned long long* acc_in = nullptr;  // sums of the previous mask (used if upd != 0; never null)
  unsigned long long* acc_out = nullptr;       // sums of this launch's mask (added to; cleared beforehand)
  unsigned long long* acc_zero = nullptr;      // cleared here for the launch after next
  int T = 0;                                   // traps of all holograms of the launch
  float acc_scale = 0.0f, acc_unscale = 0.0f;  // 2^s, and 2^-s / N (s = 30 - ceil(log2 N))
  float* stats = nullptr;
  int kstat = 0, stat_stride = 1;
  int upd = 0;                   // 0 none, 1 GS, 2 GSW
  int* flag = nullptr;
  float* phase = nullptr;  // the mask is written when not null
};

// ---- launchers (hot_kernels.hip); all enqueue on `s` and return hipError_t ----

hipError_t launch_iter(hipStream_t s, const IterArgs& a);

// V (2T floats, interleaved) from one buffer of the direct path's fixed-point sums.
hipError_t launch_collect(hipStream_t s, int T, const unsigned long long* acc, float unscale, float* V);
// End of a solve: V from the sums and its figures of merit into stats[b][kstat] (st: the final
// state, read but not changed), one block per hologram.
hipError_t launch_finish(hipStream_t s, int B, int T, const unsigned long long* acc, float unscale,
                         const HoloDesc* hd, const TrapState* st, float* V, float* stats, int kstat,
                         int stat_stride);

// Pixel pass alone (Eq. 3 with weights).  mode 0 writes the phase; mode 1 (adjoint) reads
// `phase` and G (2T floats, interleaved) and writes grad[b][j] = (1/N) Im(e^{-i phi_j} sum_m G_m e^{i Delta_j^m}).
hipError_t launch_backward(hipStream_t s, int nx, int ny, int B, bool fract, int q, const TrapCoef* coef,
                           const TrapState* st, const HoloDesc* hd, float* phase, int mode, const float* G,
                           float* grad);

// Trap pass alone: per-block partial sums of e^{i 2pi (phi - Delta)} -> partial[(off + m) * nblk + blk].
// `tpl` is the traps-per-lane count every hologram of the launch was laid out for.
hipError_t launch_forward(hipStream_t s, const FwdGeom& fg, int B, int mmax, int tpl, bool fract,
                          const TrapCoef* coef, const HoloDesc* hd, const float* phase, float2* partial);

// Fixed-order sum of the partials: V (interleaved re/im) = sum / N.
hipError_t launch_reduce(hipStream_t s, int B, int mmax, int nblk, float inv_n, const float2* partial,
                         const HoloDesc* hd, float* V);

// One block per hologram: stats[b][kstat] from V and, for mode 1 (GS) / 2 (GSW), the update st_in -> st_out.
hipError_t launch_update(hipStream_t s, int B, const float* V, const HoloDesc* hd, const TrapState* st_in,
                         TrapState* st_out, float* stats, int kstat, int stat_stride, int mode, int* flag);

// Stored-exp(i Delta) variant.
hipError_t launch_expdelta(hipStream_t s, int nx, int ny, int B, int mmax, const TrapCoef* coef,
                           const HoloDesc* hd, float2* A);
hipError_t launch_backward_stored(hipStream_t s, int n, int B, const float2* A, const TrapState* st,
                                  const HoloDesc* hd, float* phase, float2* E);
hipError_t launch_forward_stored(hipStream_t s, int n, int B, int mmax, const float2* A, const float2* E,
                                 const HoloDesc* hd, float2* partial);

// Separable reformulation on the matrix cores (any batch); the per-block tables of Eq. 2's two
// factors are computed in LDS from coef.
struct SepArgs {
  int mode = 0;  // 0 iteration, 1 trap pass from `phase`, 2 pixel pass, 3 adjoint (G in vin, grad out)
  int W = 4;     // tiles per block: a block covers 16 rows x 16 W columns
  int kh = 1;    // mode 0: waves per tile (1, or 2 taking half of the traps each)
  int B = 1, nx = 0, ny = 0, mmax = 0;
  int one_m = 0, one_off = 0;  // B == 1: the hologram's trap count and offset, passed by value
  int sc = 16;   // traps per LDS super-chunk (multiple of 16); sep_lds_bytes(W, sc, mmax, kh) <= kSepLdsMax
  const TrapCoef* coef = nullptr;
  const HoloDesc* hd = nullptr;
  const TrapState* st_in = nullptr;
  TrapState* st_out = nullptr;
  const float* vin = nullptr;  // G (mode 3), interleaved
  // mode 0: rotating fixed-point trap sums, as for the direct iteration kernel
  const unsigned long long* acc_in = nullptr;
  unsigned long long* acc_out = nullptr;
  unsigned long long* acc_zero = nullptr;
  int T = 0;
  float acc_scale = 0.0f, acc_unscale = 0.0f;
  float* stats = nullptr;
  int kstat = 0, stat_stride = 1;
  int upd = 0;  // mode 0: 0 none, 1 GS, 2 GSW
  int* flag = nullptr;
  float inv_n = 0.0f;
  float* phase = nullptr;  // mode 0: written when non-null; modes 1, 3: read; mode 2: written
  float* grad = nullptr;
  float2* partial = nullptr;  // mode 1: [T][nblk()]
  int gx() const { return (nx + 16 * W - 1) / (16 * W); }
  int gy() const { return (ny + 15) / 16; }
  int nblk() const { return gx() * gy(); }
};
hipError_t launch_sep(hipStream_t s, const SepArgs& a);
// dynamic LDS of a separable launch: per-trap coefficients (32 B) and weights (8 B), the tables of
// sc traps for the block's 16 W columns and 16 rows (plain and weighted), W kh per-wave trap sums,
// and with kh = 2 the waves' partial pixel sums (2 KB per wave)
constexpr int kSepLdsMax = 160 * 1024 - 1024;
inline size_t sep_lds_bytes(int W, int sc, int mmax, int kh = 1) {
  const size_t mp = (size_t)(mmax + 15) / 16 * 16;
  return 40 * mp + 8 * (size_t)(sc + 2) * (16 * W + 32) + 8 * (size_t)W * kh * sc + (kh == 2 ? 2048 * (size_t)W * kh : 0);
}

// Micro-benchmarks (hot_probes.hip): issue-rate probe of kind 0 (FMA), 1 (sin/cos) or 2 (the
// direct passes' term: 4 FMA + sin + cos); every wave writes {shader clock, shader clock,
// real-time clock, real-time clock} at its start and end to stamps[4 wave .. 4 wave + 3].
int probe_ops_per_rep(int kind);
hipError_t launch_probe(hipStream_t s, int kind, int blocks, int threads, long long reps, float seed, float* sink,
                        unsigned long long* stamps);
// Device copy of n16 16-byte words on `blocks` blocks of 256 threads.
hipError_t launch_probe_copy(hipStream_t s, const void* src, void* dst, size_t n16, int blocks);

// Table 1 ablation of the random-superposition pixel pass (placement 0 LDS, 1 scalar loads, 2 global
// per-lane loads; mapping 0 linear row segments, 1 square tiles; bs = 64 or 256 pixels per block).
int abl_blocks(int mapping, int bs, int nx, int ny);
hipError_t launch_abl_records(hipStream_t s, int mapping, int bs, int nx, int ny, int M, const TrapCoef* coef,
                              const TrapState* st, float4* records);
hipError_t launch_abl_pixel(hipStream_t s, int placement, int mapping, int bs, int nx, int ny, int M,
                            const float4* records, float* phase);

// 8-bit SLM frame encoding.
hipError_t launch_encode_u8(hipStream_t s, const float* phase, uint8_t* frame, int64_t n);

// The fixed device workspace of the allocation-free entry point (hot_scratch.hip): its size, and
// its device address on `device` (which must be the current device).
constexpr size_t kScratchBytes = size_t(1) << 20;
hipError_t scratch_address(int device, void** out);

// Small helpers.
hipError_t launch_fill_u32(hipStream_t s, unsigned* p, unsigned v, int n);
// dst <- src, n16 16-byte words (src: device memory or the device mapping of pinned host memory).
hipError_t launch_copy16(hipStream_t s, const void* src, void* dst, size_t n16);
hipError_t launch_export_state(hipStream_t s, const TrapState* st, int t, float* w_out, float* theta_out);
hipError_t launch_import_w(hipStream_t s, const float* w0, TrapState* st, int t);

}  // namespace hot
