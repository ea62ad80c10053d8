// hot_kernels.hip -- CDNA4 (gfx950) kernels of the phase-only hologram solver.
//
// Method: Bianchi & Di Leonardo, arXiv:0907.4027.  Two passes per iteration:
//   pixel (backward) pass, Eq. 3 with weights:  phi_j = arg sum_m w_m e^{i(Delta_j^m + theta_m)}
//   trap (forward) pass, Eq. 1:                 V_m   = (1/N) sum_j e^{i(phi_j - Delta_j^m)}
// with Delta from Eq. 2 recomputed for every (pixel, trap) pair, and between them the
// GSW update of Section 3 (w_m <- w_m <|V|>/|V_m|, theta_m <- arg V_m).
//
// The paper runs one thread per pixel in both passes and sums Eq. 1 with a tree of
// shared-memory reduction kernels.  Here one kernel per iteration does, for one row
// segment of the SLM: the weight/phase update (recomputed identically by every block
// from the previous V, so no grid-wide synchronisation is needed), the pixel pass with
// one lane per pixel, and -- with the fresh phases handed over through LDS -- the trap
// pass with traps on lanes and pixels in a loop, so each lane accumulates its own V_m
// over a slice of pixels and no per-trap cross-lane reduction is needed.  Each block adds
// its per-trap sums as exact fixed-point integers to accumulators that the next launch
// reads, so V does not depend on the order of the blocks and no reduction kernel runs
// between iterations.
//
// All phases are in revolutions (see hot_internal.h).  sin/cos are the hardware
// V_SIN_F32 / V_COS_F32, which take revolutions; their domain is |x| < 256, and the
// host switches on an explicit fract() (exact in FP32) when a grid could leave it.
#include "hot_internal.h"

#include <algorithm>
#include <type_traits>

namespace hot {

namespace {

constexpr float kInv2Pi = 0.159154943091895336f;  // FP32(1 / (2 pi))
constexpr float kTwoPi = 6.28318530717958648f;    // FP32(2 pi)

// Holograms of at least this many traps run the iteration kernels' update and pixel pass at a
// higher wave priority than their trap pass (measured: 768^2 x 49 traps 21.9 -> 20.2 us per
// iteration, 512^2 x 100 16.6 -> 15.2 us; 768^2 x 25 14.6 -> 15.5 us, 1024 x 768 x 8 7.4 -> 9.7 us).
constexpr int kPriorityTraps = 40;

// The XCD (accelerator complex die) the wave runs on: hardware register XCC_ID, bits 3:0.
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & 15; }

template <bool FRACT>
__device__ __forceinline__ float to_period(float t) {
  if constexpr (FRACT) return __builtin_amdgcn_fractf(t);
  return t;
}

// Wave-wide reductions.  DPP steps combine lanes inside each row of 16 (xor 1, xor 2, then the
// half-row and row mirrors), after which every lane of a row holds the row result; the four
// row results are then read from lanes 0, 16, 32, 48 and combined in that order, so the
// result is the same, deterministic value in every lane.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float rows_of(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return (rows_of(v, 0) + rows_of(v, 16)) + (rows_of(v, 32) + rows_of(v, 48));
}
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x141>(v));
  v = fmaxf(v, dpp<0x140>(v));
  return fmaxf(fmaxf(rows_of(v, 0), rows_of(v, 16)), fmaxf(rows_of(v, 32), rows_of(v, 48)));
}
__device__ __forceinline__ float wave_min(float v) {
  v = fminf(v, dpp<0xB1>(v));
  v = fminf(v, dpp<0x4E>(v));
  v = fminf(v, dpp<0x141>(v));
  v = fminf(v, dpp<0x140>(v));
  return fminf(fminf(rows_of(v, 0), rows_of(v, 16)), fminf(rows_of(v, 32), rows_of(v, 48)));
}

// A caller's phase [rad] in revolutions, reduced to [0, 1] (1 is the same angle as 0): product and
// reduction in FP64, so a mask far outside [0, 2 pi) (an optimiser's drifting phase, say) loses
// nothing beyond its own FP32 rounding and stays inside the hardware sin/cos domain.  Once per pixel.
__device__ __forceinline__ float caller_phase_rev(float ph) {
  const double t = (double)ph * 0.15915494309189533577;  // 1 / (2 pi)
  return (float)(t - __builtin_floor(t));
}

__device__ __forceinline__ float wrap_phase(float ph) { return ph < 0.0f ? ph + kTwoPi : ph; }

// arg(x + i y) in [0, 2pi] (arg 0 = 0).  The octant is folded onto t = min(|x|,|y|) / max(|x|,|y|)
// in [0, 1], where atan t = t P(t^2) with P of degree 7: coefficients from a Lawson-weighted
// least-squares (near-minimax) fit to atan on [0, 1], max error 4e-8 in exact arithmetic and
// 1.4e-7 rad evaluated in FP32; the reciprocal adds at most 1.2e-7.  Then the octant and the
// quadrant are undone.
__device__ __forceinline__ float phase_of(float y, float x) {
  const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
  const float mx = __builtin_fmaxf(ax, ay), mn = __builtin_fminf(ax, ay);
  const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float s = t * t;
  float p = -4.054570390e-03f;
  p = __builtin_fmaf(p, s, 2.186296944e-02f);
  p = __builtin_fmaf(p, s, -5.591234356e-02f);
  p = __builtin_fmaf(p, s, 9.642198569e-02f);
  p = __builtin_fmaf(p, s, -1.390863004e-01f);
  p = __builtin_fmaf(p, s, 1.994656575e-01f);
  p = __builtin_fmaf(p, s, -3.332986079e-01f);
  p = __builtin_fmaf(p, s, 9.999993356e-01f);
  float r = p * t;
  if (ay > ax) r = 1.57079632679489662f - r;
  if (x < 0.0f) r = 3.14159265358979324f - r;
  if (y < 0.0f) r = kTwoPi - r;
  return r;
}

// Block-wide (NT threads) sums of a and b, max of c, min of d; every thread gets the
// results.  Waves reduce with wave_sum/max/min, lane 0 of each wave publishes to `sh`
// (4 * (NT / 64) floats, not reused by the caller), one barrier, then every thread combines
// the wave results in wave order.
template <int NT>
__device__ __forceinline__ void block_reduce(float* sh, float& a, float& b, float& c, float& d) {
  constexpr int W = NT / 64;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_max(c);
  d = wave_min(d);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[wave] = a;
    sh[W + wave] = b;
    sh[2 * W + wave] = c;
    sh[3 * W + wave] = d;
  }
  __syncthreads();
  a = sh[0];
  b = sh[W];
  c = sh[2 * W];
  d = sh[3 * W];
  for (int w = 1; w < W; ++w) {
    a += sh[w];
    b += sh[W + w];
    c = fmaxf(c, sh[2 * W + w]);
    d = fminf(d, sh[3 * W + w]);
  }
}

// Block-wide sum of a (every thread gets it), combined in wave order as in block_reduce.
template <int NT>
__device__ __forceinline__ void block_sum(float* sh, float& a) {
  constexpr int W = NT / 64;
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  a = sh[0];
  for (int w = 1; w < W; ++w) a += sh[w];
}

// V of trap k (local index) of a hologram: from an interleaved (re, im) array ...
struct VArray {
  const float* __restrict__ V;
  int off;
  __device__ float2 operator()(int k) const { return make_float2(V[2 * (off + k)], V[2 * (off + k) + 1]); }
};
// ... or from the fixed-point sums of the fused kernels: kAccRegions regions of T 64-bit words.
// A block adds its sum (re, im) of a trap as one word, pack_sum: re and im are rounded to
// integers in units of 1/scale, and the word is the 64-bit two's-complement value
// re + 2^32 im.  Words add like integers, so a sum of words is R + 2^32 I with R, I the sums of
// the parts; as long as |R| < 2^31 (the host picks scale so that any sum of N unit-modulus terms
// stays within 2^30), R is the low 32 bits read as signed, and I the high 32 bits plus one if R
// is negative.  V = (R, I) * unscale.
__device__ __forceinline__ unsigned long long pack_sum(float2 v, float scale) {
  const int re = (int)__builtin_rintf(v.x * scale), im = (int)__builtin_rintf(v.y * scale);
  return (unsigned long long)(long long)re + ((unsigned long long)(unsigned)im << 32);
}
static_assert(kAccRegions == 8, "VAcc sums eight regions");
struct VAcc {
  const unsigned long long* __restrict__ acc;
  int T, off;
  float unscale;
  // the eight words of trap k (loads only: nothing waits for them here) ...
  __device__ void load(int k, unsigned long long (&w8)[kAccRegions]) const {
#pragma unroll
    for (int r = 0; r < kAccRegions; ++r) w8[r] = acc[(size_t)r * T + off + k];
  }
  // ... and V from them: a tree of adds (exact, so the order is free), three dependent steps
  // instead of seven
  __device__ float2 sum(const unsigned long long (&w8)[kAccRegions]) const {
    const unsigned long long w = ((w8[0] + w8[1]) + (w8[2] + w8[3])) + ((w8[4] + w8[5]) + (w8[6] + w8[7]));
    const int re = (int)(unsigned)w;
    const int im = (int)((unsigned)(w >> 32) - (unsigned)(re >> 31));
    return make_float2((float)re * unscale, (float)im * unscale);
  }
  __device__ float2 operator()(int k) const {
    unsigned long long w8[kAccRegions];
    load(k, w8);
    return sum(w8);
  }
};

// Section 3 figures of merit and the GS/GSW update for one hologram, computed by one
// block from V (vmem(k) for its M traps) and the current state.
//   stats_row (3 floats) if non-null: e = sum I, u = 1 - (max-min)/(max+min), sigma = std(I)/mean(I)
//   mode 0: no update; 1 (GS): theta_m <- arg V_m; 2 (GSW): also w_m <- w_m <|V|>/|V_m|
// emit(m, state) is called once per trap m, by the thread that owns it.  <|V|> = 0 leaves
// the state unchanged and raises *flag (if non-null).  With PRE, trap threadIdx.x's V and state
// come from vpre / spre (loaded earlier by the caller) instead of memory.  |V_m|, <|V|> and the
// weight factor use the hardware square root and reciprocal (about 1 ulp each): this sits on the
// critical path at the start of every iteration launch.
template <int NT, class VGet, class Emit, bool PRE = false>
__device__ void update_traps(VGet vmem, const TrapState* __restrict__ st_in, int off, int M, int mode, float* sh,
                             float* stats_row, int* flag, Emit emit, float2 vpre = make_float2(0.0f, 0.0f),
                             TrapState spre = TrapState{}) {
  auto getv = [&](int k) {
    if (PRE && k == (int)threadIdx.x) return vpre;
    return vmem(k);
  };
  // PRE: the modulus of the thread's own V, its reciprocal and arg V do not need <|V|>; they are
  // formed here, so that their latency overlaps the block-wide sum instead of following it
  float own_amp = 0.0f, own_rcp = 0.0f, own_th = 0.0f;
  if (PRE && mode != 0 && (int)threadIdx.x < M) {
    own_amp = __builtin_amdgcn_sqrtf(vpre.x * vpre.x + vpre.y * vpre.y);
    own_rcp = __builtin_amdgcn_rcpf(own_amp);
    own_th = phase_of(vpre.y, vpre.x);
  }
  float sa = 0.0f, si = 0.0f, mx = -1.0f, mn = 3.0e38f;
  for (int k = threadIdx.x; k < M; k += NT) {
    const float2 v = getv(k);
    const float vr = v.x, vi = v.y;
    const float I = vr * vr + vi * vi;
    sa += __builtin_amdgcn_sqrtf(I);
    si += I;
    mx = fmaxf(mx, I);
    mn = fminf(mn, I);
  }
  if (stats_row) {
    block_reduce<NT>(sh, sa, si, mx, mn);
  } else {
    block_sum<NT>(sh, sa);  // the update needs only <|V|>
  }
  const float mean_abs = sa * __builtin_amdgcn_rcpf((float)M);
  if (stats_row) {
    const float mu = si / (float)M;
    float var = 0.0f, z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
    for (int k = threadIdx.x; k < M; k += NT) {
      const float2 v = getv(k);
      const float vr = v.x, vi = v.y;
      const float dI = vr * vr + vi * vi - mu;
      var += dI * dI;
    }
    block_reduce<NT>(sh + 4 * (NT / 64), var, z0, z1, z2);
    var /= (float)M;
    if (threadIdx.x == 0) {
      stats_row[0] = si;
      stats_row[1] = (mx + mn) > 0.0f ? 1.0f - (mx - mn) / (mx + mn) : 0.0f;
      stats_row[2] = mu > 0.0f ? sqrtf(var) / mu : 0.0f;
    }
  }
  const bool degenerate = mode != 0 && !(mean_abs > 0.0f);
  if (degenerate && flag && threadIdx.x == 0) *flag = 1;
  const float floor_abs = 1e-12f * mean_abs;
  for (int k = threadIdx.x; k < M; k += NT) {
    TrapState s = (PRE && k == (int)threadIdx.x) ? spre : st_in[off + k];
    if (mode != 0 && !degenerate) {
      float amp, rcp_amp, th;  // |V_m|, its reciprocal, arg V_m in [0, 2pi]
      if (PRE && k == (int)threadIdx.x) {
        amp = own_amp;
        rcp_amp = own_rcp;
        th = own_th;
      } else {
        const float2 v = getv(k);
        amp = __builtin_amdgcn_sqrtf(v.x * v.x + v.y * v.y);
        rcp_amp = __builtin_amdgcn_rcpf(amp);
        th = phase_of(v.y, v.x);
      }
      const bool tiny = amp < floor_abs;
      if (mode == 2) s.w *= mean_abs * (tiny ? __builtin_amdgcn_rcpf(floor_abs) : rcp_amp);
      if (!tiny) {
        s.theta_rad = th > 3.14159265358979324f ? th - kTwoPi : th;  // kept in (-pi, pi]
        s.theta_rev = s.theta_rad * kInv2Pi;
      }
    }
    emit(k, s);
  }
}

// Pixel-pass terms for Q pixels of one lane: S += w_m e^{i 2pi (g u^2 + a' u + C_m)} over all
// traps, u = U - Uc the lane's pixel relative to the block's reference (hot_internal.h).  Per
// term: 2 FMA, sin, cos, 2 FMA.  The per-trap record {a', g, C_m, w_m} (C_m = K + theta_rev:
// everything constant over the block's pixels) is an LDS broadcast, and the
// records of the next kTrapChunk traps are loaded while the current ones are used.  Only LDS
// loads are in flight here, so the in-order LDS counter lets the compiler wait for exactly
// the records it needs (a scalar load in the loop would force a wait for all of them).
// `rec` holds M records followed by zero records up to round_up(M, kTrapChunk) + kTrapChunk
// (w = 0: they add nothing).
// (kTrapChunk and rec_pad are in hot_internal.h.)

template <int Q, bool FRACT>
__device__ __forceinline__ void pixel_chunk(const float4* c, const float* U, const float* U2, float* sr, float* si) {
#pragma unroll
  for (int i = 0; i < kTrapChunk; ++i) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float t = to_period<FRACT>(__builtin_fmaf(c[i].y, U2[q], __builtin_fmaf(c[i].x, U[q], c[i].z)));
      const float sn = __builtin_amdgcn_sinf(t), cs = __builtin_amdgcn_cosf(t);
      sr[q] = __builtin_fmaf(c[i].w, cs, sr[q]);
      si[q] = __builtin_fmaf(c[i].w, sn, si[q]);
    }
  }
}

// Two record buffers alternate: one chunk is summed while the next one is read.  The offset of
// each read is hidden from the optimiser (an empty asm on the uniform counter); otherwise it
// proves that a chunk equals the one read a step earlier and reloads it where it is used,
// waiting on LDS each step.  Full double steps run while 8 traps remain, then at most two
// chunks.  Every read stays below rec_pad(M) (the loop reads up to m0 + 11 with m0 + 8 <= M).
template <int Q, bool FRACT>
__device__ __forceinline__ void pixel_terms(const float4* rec, int M, const float* U, const float* U2, float* sr,
                                            float* si) {
  float4 ra[kTrapChunk], rb[kTrapChunk];
#pragma unroll
  for (int i = 0; i < kTrapChunk; ++i) ra[i] = rec[i];
  int m0 = 0;
  for (; m0 + 2 * kTrapChunk <= M; m0 += 2 * kTrapChunk) {
    int nb = m0 + kTrapChunk;
    asm volatile("" : "+s"(nb));
#pragma unroll
    for (int i = 0; i < kTrapChunk; ++i) rb[i] = rec[nb + i];
    __builtin_amdgcn_sched_barrier(0);
    pixel_chunk<Q, FRACT>(ra, U, U2, sr, si);
    int na = m0 + 2 * kTrapChunk;
    asm volatile("" : "+s"(na));
#pragma unroll
    for (int i = 0; i < kTrapChunk; ++i) ra[i] = rec[na + i];
    __builtin_amdgcn_sched_barrier(0);
    pixel_chunk<Q, FRACT>(rb, U, U2, sr, si);
  }
  if (m0 < M) {
    if (m0 + kTrapChunk < M) {
#pragma unroll
      for (int i = 0; i < kTrapChunk; ++i) rb[i] = rec[m0 + kTrapChunk + i];
    }
    pixel_chunk<Q, FRACT>(ra, U, U2, sr, si);
    if (m0 + kTrapChunk < M) pixel_chunk<Q, FRACT>(rb, U, U2, sr, si);
  }
}

// The block reference of a trap (hot_internal.h): a' = a + 2 g Uc reduced mod 1/2 (u is even) and
// K = g (Uc^2 + V^2) + a Uc + b V reduced mod 1, both in FP64 (exact to ~1e-16 rev: the products
// of the coefficients with these integers are exact, each sum rounds once), then rounded to FP32.
__device__ __forceinline__ float block_slope(const TrapCoef& c, double Uc) {
  double ap = __builtin_fma(2.0 * c.g, Uc, c.a);
  ap -= 0.5 * __builtin_rint(2.0 * ap);
  return (float)ap;
}
__device__ __forceinline__ float block_const(const TrapCoef& c, double Uc, double V) {
  const double k = __builtin_fma(c.g, __builtin_fma(Uc, Uc, V * V), __builtin_fma(c.a, Uc, c.b * V));
  return (float)(k - __builtin_floor(k));
}
// Centre of a block's pixels [c0, c0 + len): Uc of the column c0 + (len - 1) / 2.
__device__ __forceinline__ int centre_col(int c0, int len) { return c0 + (max(len, 1) - 1) / 2; }

// Pixel-pass record of trap m: {a', g, K + theta_rev, w}; records past M are zero (w = 0).
__device__ __forceinline__ void stage_record(float4* rec, int m, float ap, float gf, float k, float theta_rev,
                                             float w) {
  rec[m] = make_float4(ap, gf, k + theta_rev, w);
}
template <int NT>
__device__ __forceinline__ void pad_records(float4* rec, int M) {
  for (int m = M + (int)threadIdx.x; m < rec_pad(M); m += NT) rec[m] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Spans.  The pixels of a row segment are referenced span by span: span h holds the pixels
// [kSpan h, kSpan (h + 1)) of the segment, with its own centre Uc_h, slope a'_h and constant K_h
// (hot_internal.h), so |u| <= kSpan in the per-term argument whatever the segment's width.  The
// trap pass's pixels sit in LDS span by span, kSpanStride entries per span (zero-padded).
// (kSpan, kSpanStride and the LDS sizes are in hot_internal.h.)

// Trap pass over one row segment (per half of a block with ROWS = 2) whose pixels
// (phi_rev, u, u^2, mask) sit span by span in LDS `pxh` (len real entries).  The W waves of a half
// share the HS spans, WS = W / HS waves per span; each wave is split into A slices of G lanes;
// lane (slice s, position l) owns traps l, l+G, ..., l+(TPL-1)G of a chunk and loops over the
// pixels of its slice:
//   t = phi - a'_m u - g_m u^2               2 VALU
//   sin t, cos t                             2 transcendental
//   acc += mask (cos t, sin t)              2 VALU
// with a'_m and g_m the coefficients of its span's records.  The slice partials of each trap are
// then summed in slice order through LDS `red`, span by span; the span constant K_m of Eq. 2 is
// left out of the pixel sums: each span's sum is turned by e^{-i 2pi K_m} once, by the thread that
// sums its slices, and store(m, sum) gets the block's sum over its spans and rows.  Slots past M
// take trap M - 1's coefficients (always a valid read, and the arguments stay in the sin/cos
// domain); their sums are never written out.
template <int TPL>
struct LaneCoef {
  float na[TPL], ng[TPL];
};
template <int TPL>
__device__ __forceinline__ LaneCoef<TPL> lane_coef(const float4* rec, int M, int G, int k0) {
  const int lane = threadIdx.x & 63;
  const int tl = lane - lane / G * G;
  LaneCoef<TPL> lc;
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const float4 r = rec[min(k0 + tl + k * G, M - 1)];
    lc.na[k] = -r.x;
    lc.ng[k] = -r.y;
  }
  return lc;
}

template <int W, int HS, int TPL, bool FRACT, int ROWS, class Store>
__device__ __forceinline__ void trap_pass_block(const float4* rec, int rp, const float* kt, int mp, int M, int G,
                                                int A, const float4* pxh, int len, float2* red, Store store) {
  static_assert(W % HS == 0, "whole waves per span");
  constexpr int NB = ROWS * W * 64, WS = W / HS;
  const int half = (int)threadIdx.x / (W * 64);
  const int wave = ((int)threadIdx.x >> 6) - half * W, lane = threadIdx.x & 63;
  const int s = lane / G, tl = lane - s * G;
  const bool active = s < A;
  const int h = wave / WS, lw = wave - h * WS;  // the wave's span, and its place among the span's waves
  const int lh = min(max(len - kSpan * h, 0), kSpan);
  const int SA = WS * A;  // slices per span
  const int slen = (lh + SA - 1) / SA;
  const float4* mine = pxh + h * kSpanStride + (lw * A + min(s, A - 1)) * slen;
  const float4* rech = rec + (half * HS + h) * rp;
  const int nslot = G * TPL;
  for (int k0 = 0; k0 < M; k0 += nslot) {
    const LaneCoef<TPL> lc = lane_coef<TPL>(rech, M, G, k0);
    float na[TPL], ng[TPL], accr[TPL], acci[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      na[k] = lc.na[k];
      ng[k] = lc.ng[k];
      accr[k] = 0.0f;
      acci[k] = 0.0f;
    }
    // Two pixels per half step, from two register pairs that alternate: one pair is summed while
    // the next is read (offsets hidden from the optimiser as in the pixel pass).  Full double
    // steps run while 4 pixels remain, then the last 1-3 pixels one pair and one single at a
    // time.  Reads reach at most mine[slen + 1], inside the span's region (SA slen + 2 entries).
    auto term1 = [&](const float4& p0) {
#pragma unroll
      for (int k = 0; k < TPL; ++k) {
        const float ta = to_period<FRACT>(__builtin_fmaf(ng[k], p0.z, __builtin_fmaf(na[k], p0.y, p0.x)));
        accr[k] = __builtin_fmaf(p0.w, __builtin_amdgcn_cosf(ta), accr[k]);
        acci[k] = __builtin_fmaf(p0.w, __builtin_amdgcn_sinf(ta), acci[k]);
      }
    };
    auto terms = [&](const float4& p0, const float4& p1) {
#pragma unroll
      for (int k = 0; k < TPL; ++k) {
        const float ta = to_period<FRACT>(__builtin_fmaf(ng[k], p0.z, __builtin_fmaf(na[k], p0.y, p0.x)));
        const float tb = to_period<FRACT>(__builtin_fmaf(ng[k], p1.z, __builtin_fmaf(na[k], p1.y, p1.x)));
        accr[k] = __builtin_fmaf(p0.w, __builtin_amdgcn_cosf(ta), accr[k]);
        acci[k] = __builtin_fmaf(p0.w, __builtin_amdgcn_sinf(ta), acci[k]);
        accr[k] = __builtin_fmaf(p1.w, __builtin_amdgcn_cosf(tb), accr[k]);
        acci[k] = __builtin_fmaf(p1.w, __builtin_amdgcn_sinf(tb), acci[k]);
      }
    };
    float4 pa = mine[0], pb = mine[1], pc, pd;
    int j = 0;
    for (; j + 4 <= slen; j += 4) {
      int nc = j + 2;
      asm volatile("" : "+s"(nc));
      pc = mine[nc];
      pd = mine[nc + 1];
      __builtin_amdgcn_sched_barrier(0);
      terms(pa, pb);
      int na2 = j + 4;
      asm volatile("" : "+s"(na2));
      pa = mine[na2];
      pb = mine[na2 + 1];
      __builtin_amdgcn_sched_barrier(0);
      terms(pc, pd);
    }
    const int rest = slen - j;  // 0..3 pixels left, pa and pb already read
    if (rest >= 2) {
      if (rest == 3) pc = mine[j + 2];
      terms(pa, pb);
      if (rest == 3) term1(pc);
    } else if (rest == 1) {
      term1(pa);
    }
    __syncthreads();  // red[] is free: its readers of the previous chunk are done
    if (active) {
#pragma unroll
      for (int k = 0; k < TPL; ++k)
        red[(half * W * A + wave * A + s) * nslot + tl + k * G] = make_float2(accr[k], acci[k]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nslot; i += NB) {
      const int m = k0 + i;
      if (m < M) {
        float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int hr = 0; hr < ROWS * HS; ++hr) {  // (row half, span) pairs
          const float kh = kt[hr * mp + m];
          // the span's slices in order; the reads go out in groups so that their latencies overlap
          const float2* rp2 = red + hr * SA * nslot + i;
          float sr = 0.0f, si = 0.0f;
          int s2 = 0;
          for (; s2 + 8 <= SA; s2 += 8) {
            float2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = rp2[(s2 + u) * nslot];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              sr += v[u].x;
              si += v[u].y;
            }
          }
          if (s2 + 4 <= SA) {
            float2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = rp2[(s2 + u) * nslot];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              sr += v[u].x;
              si += v[u].y;
            }
            s2 += 4;
          }
          for (; s2 < SA; ++s2) {
            sr += rp2[s2 * nslot].x;
            si += rp2[s2 * nslot].y;
          }
          const float cs = __builtin_amdgcn_cosf(kh), sn = __builtin_amdgcn_sinf(kh);
          acc.x += __builtin_fmaf(sr, cs, si * sn);  // (sr + i si) e^{-i 2pi K}
          acc.y += __builtin_fmaf(si, cs, -sr * sn);
        }
        store(m, acc);
      }
    }
  }
}

// Stage the records and K of trap m for the block's spans of a row segment starting at column
// cbeg with lseg pixels, for its ROWS rows (row coordinate of row hr: Vb + 2 hr).  First the span
// references of the trap, a' per span and K per (row, span) pair (geometry only: they do not depend
// on the iteration's state) ...
template <int HS, int ROWS>
struct SpanRefs {
  float ap[HS], k[ROWS * HS];
};
template <int HS, int ROWS>
__device__ __forceinline__ SpanRefs<HS, ROWS> span_refs(const TrapCoef& c, int nx, int cbeg, int lseg, int Vb) {
  SpanRefs<HS, ROWS> r;
#pragma unroll
  for (int h = 0; h < HS; ++h) {
    const int cc = centre_col(cbeg + kSpan * h, min(max(lseg - kSpan * h, 1), kSpan));
    const double Uc = (double)(2 * cc - (nx - 1));
    r.ap[h] = block_slope(c, Uc);
#pragma unroll
    for (int hr = 0; hr < ROWS; ++hr) r.k[hr * HS + h] = block_const(c, Uc, (double)(Vb + 2 * hr));
  }
  return r;
}
// ... and its records and K from them, with the state's theta and w.
template <int HS, int ROWS>
__device__ __forceinline__ void stage_refs(float4* rec, int rp, float* kt, int mp, int m, const SpanRefs<HS, ROWS>& r,
                                           float gf, float theta_rev, float w) {
#pragma unroll
  for (int h = 0; h < HS; ++h) {
#pragma unroll
    for (int hr = 0; hr < ROWS; ++hr) {
      stage_record(rec + (hr * HS + h) * rp, m, r.ap[h], gf, r.k[hr * HS + h], theta_rev, w);
      kt[(hr * HS + h) * mp + m] = r.k[hr * HS + h];
    }
  }
}
template <int HS, int ROWS>
__device__ __forceinline__ void stage_spans(float4* rec, int rp, float* kt, int mp, int m, const TrapCoef& c, int nx,
                                            int cbeg, int lseg, int Vb, float theta_rev, float w) {
  stage_refs<HS, ROWS>(rec, rp, kt, mp, m, span_refs<HS, ROWS>(c, nx, cbeg, lseg, Vb), c.gf, theta_rev, w);
}

// ------------------------------------------------------------------ fused iteration kernel
//
// Grid (nseg, ceil(ny / ROWS), B), ROWS * NT threads.  Each half of NT threads passes over one row
// segment (seg_w <= NT * Q pixels, HS = NT Q / kSpan spans) of row ROWS * blockIdx.y + half; both
// halves share the update and add one sum per trap (ROWS = 2 halves the update work and the
// atomic adds per row).
//   upd = 0: use st_in as is;  1/2: GS/GSW update from V of the previous mask and st_in,
//   recomputed by every block; block (0, 0, b) also writes the new state to st_out and the
//   figures of merit of that V to stats[b][kstat].
//   V is not a separate array: the previous launch added each block's trap sums to acc_in as
//   fixed-point words (pack_sum: re and im in one 64-bit atomic add), one region per XCD (the
//   XCC_ID of the adding wave) so that the atomics of different XCDs do not contend; integer
//   sums do not depend on the order of the adds, so the result is deterministic.  This launch
//   adds its own sums to acc_out, and block (0, 0, b) clears hologram b's part of acc_zero for the
//   launch after next.  acc_in is read even when upd == 0 (it must be a valid buffer; the values
//   are then unused).
//   one.m > 0: a single hologram whose descriptor comes by value, so no global load waits for it.
//   The arguments reach the waves by scalar loads: the compiler preloads leading arguments into
//   SGPRs only up to the first aggregate, and the descriptor leads the list.  Passing its fields
//   as scalars instead, so that the first 14 SGPRs of arguments are preloaded, measured 0.5-1 %
//   slower in same-box A/B runs, as did reordering the arguments: the time these loads take is
//   not what sets the prologue's length, and the code layout moves the launch by that much.
//   Writes the phase (radians) when `phase` is not null (the host passes it for the last mask only).
//   Dynamic LDS: refs_lds_bytes(ROWS * HS, mmax) for records and K (mmax >= every hologram's M).
template <int NT, int Q, int TPL, bool FRACT, int ROWS>
__global__ void __launch_bounds__(NT * ROWS)
k_iter(HoloDesc one, const TrapCoef* __restrict__ coef, const TrapState* __restrict__ st_in,
       const unsigned long long* __restrict__ acc_in, const HoloDesc* __restrict__ hd,
       TrapState* __restrict__ st_out, unsigned long long* __restrict__ acc_out,
       unsigned long long* __restrict__ acc_zero, int T, float scale, float unscale,
       float* __restrict__ stats, int kstat, int stat_stride, int upd, int* __restrict__ flag, int nx, int ny,
       int seg_w, int mmax, float* __restrict__ phase) {
  constexpr int W = NT / 64;           // waves per half
  constexpr int NB = NT * ROWS;        // threads of the block
  constexpr int HS = NT * Q / kSpan;   // spans per segment
  static_assert(HS >= 1 && NT * Q == HS * kSpan, "segments of whole spans");
  __shared__ float4 pxs[ROWS * HS * kSpanStride];
  __shared__ float2 red[ROWS * W * 64 * TPL];  // slice partials of both halves
  __shared__ float sh[8 * NB / 64];
  extern __shared__ float4 refs[];
  const int rp = rec_pad(mmax), mp = k_stride(mmax);
  float* kts = reinterpret_cast<float*>(refs + ROWS * HS * rp);
  const int b = blockIdx.z, sg = blockIdx.x;
  const int half = ROWS == 1 ? 0 : (int)threadIdx.x / NT, tid = (int)threadIdx.x - half * NT;
  const int r = blockIdx.y * ROWS + half;
  const HoloDesc d = one.m > 0 ? one : hd[b];
  const int M = d.m, off = d.off, G = d.g, A = d.a;
  const TrapCoef* __restrict__ cf = coef + off;
  float4* px = pxs + half * HS * kSpanStride;
  const bool lead = sg == 0 && blockIdx.y == 0;
  const VAcc vacc{acc_in, T, off, unscale};
  const int cbeg = sg * seg_w, lseg = min(nx, cbeg + seg_w) - cbeg;
  const int Vb = 2 * (int)(blockIdx.y * ROWS) - (ny - 1);

  // Every read of the block's own trap data is issued here, so the update waits for one memory
  // round trip: threads past M in a wave that holds traps read trap M - 1 and ignore it; waves
  // whose first thread is past M hold no trap and read nothing.  The coefficients go first: they
  // stay in the L2 from launch to launch and return about a thousand cycles before the
  // accumulators (rewritten by the previous launch, so read from beyond the L2), and loads return
  // in order, so the trap's span references (FP64) are formed while the accumulators are in flight.
  //
  // Wave priority (holograms of kPriorityTraps traps or more): the update and the pixel pass run
  // at priority 1, the trap pass at 0.  The blocks sharing a compute unit otherwise finish in age
  // order (the oldest wave's instructions issue first), and the youngest block's trap pass is left
  // to run alone, one wave per SIMD, at the end of the launch; with the trap passes yielding to
  // the pixel passes, the younger blocks catch up while the older ones take their trap passes,
  // and the unit's blocks reach the trap pass, and the end, closer together.  With fewer traps
  // the trap pass is short and holding it back costs more than the tail saves.
  if (M >= kPriorityTraps) __builtin_amdgcn_s_setprio(1);
  const int tm = min((int)threadIdx.x, M - 1);
  TrapCoef c_first = {0.0, 0.0, 0.0, 0.0f, 0.0f};
  TrapState s_first = {0.0f, 0.0f, 0.0f, 0.0f};
  float2 v_first = make_float2(0.0f, 0.0f);
  SpanRefs<HS, ROWS> r_first = {};
  if (__builtin_amdgcn_readfirstlane((int)threadIdx.x & ~63) < M) {
    c_first = cf[tm];
    asm volatile("" ::: "memory");  // (keeps the loads below after this one)
    s_first = st_in[off + tm];
    v_first = vacc(tm);
    r_first = span_refs<HS, ROWS>(c_first, nx, cbeg, lseg, Vb);
    __builtin_amdgcn_sched_barrier(0);  // all of it before the first use of the accumulators
  }
  if (lead) {
    for (int i = threadIdx.x; i < kAccRegions * M; i += NB) {
      const int g = i / M;
      acc_zero[(size_t)g * T + off + (i - g * M)] = 0ull;
    }
  }
  auto coef_of = [&](int m) { return m == (int)threadIdx.x ? c_first : cf[m]; };
  auto stage = [&](int m, const TrapCoef& c, const TrapState& s) {
    if (m == (int)threadIdx.x) {
      stage_refs<HS, ROWS>(refs, rp, kts, mp, m, r_first, c.gf, s.theta_rev, s.w);
    } else {
      stage_spans<HS, ROWS>(refs, rp, kts, mp, m, c, nx, cbeg, lseg, Vb, s.theta_rev, s.w);
    }
  };
  for (int hs = 0; hs < ROWS * HS; ++hs) pad_records<NB>(refs + hs * rp, M);  // (no trap's record)
  if (upd == 0) {
    for (int m = threadIdx.x; m < M; m += NB) stage(m, coef_of(m), m == (int)threadIdx.x ? s_first : st_in[off + m]);
  } else {
    auto emit = [&](int m, const TrapState& s) {
      if (lead) st_out[off + m] = s;
      stage(m, coef_of(m), s);
    };
    update_traps<NB, VAcc, decltype(emit), true>(vacc, st_in, off, M, upd, sh,
                                                 lead ? stats + 3 * ((size_t)b * stat_stride + kstat) : nullptr,
                                                 lead ? flag : nullptr, emit, v_first, s_first);
  }
  __syncthreads();

  // pixel pass: pixel q of the lane is pixel i = Q tid + q of the segment (adjacent pixels, so the
  // Q pixels of a lane and the 64 Q pixels of a wave lie in one span), at u = 2 (column - the
  // span's centre); one record stream per wave
  const int len = r < ny ? lseg : 0;  // a missing last row has no pixels
  const int h0 = Q * tid / kSpan;
  const int cc0 = centre_col(cbeg + kSpan * h0, min(max(lseg - kSpan * h0, 1), kSpan));
  float u[Q], u2[Q], sr[Q], si[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    u[q] = (float)(2 * (cbeg + Q * tid + q - cc0));
    u2[q] = u[q] * u[q];
    sr[q] = 0.0f;
    si[q] = 0.0f;
  }
  pixel_terms<Q, FRACT>(refs + (half * HS + h0) * rp, M, u, u2, sr, si);
  float* __restrict__ prow = phase ? phase + (size_t)b * nx * ny + (size_t)r * nx + cbeg : nullptr;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = Q * tid + q;
    float4* slot = px + h0 * kSpanStride + (i - kSpan * h0);
    if (i < len) {
      const float ph = phase_of(si[q], sr[q]);
      if (prow) prow[i] = ph;
      *slot = make_float4(ph * kInv2Pi, u[q], u2[q], 1.0f);
    } else {
      *slot = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
  for (int i = tid; i < HS * (kSpanStride - kSpan); i += NT) {  // each span's padding
    const int h = i / (kSpanStride - kSpan);
    px[h * kSpanStride + kSpan + (i - h * (kSpanStride - kSpan))] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  __syncthreads();
  unsigned long long* __restrict__ mine = acc_out + (size_t)(xcc_id() & (kAccRegions - 1)) * T + off;
  auto add_sum = [&](int m, float2 v) {
    __hip_atomic_fetch_add(mine + m, pack_sum(v, scale), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  __builtin_amdgcn_s_setprio(0);
  trap_pass_block<W, HS, TPL, FRACT, ROWS>(refs, rp, kts, mp, M, G, A, px, len, red, add_sum);
}

// ------------------------------------------------------------------ stand-alone passes
//
// Pixel pass alone.  MODE 0 writes phase = arg S in [0, 2pi].  MODE 1 is the adjoint of
// Eq. 1: with w e^{i theta} := G_m = dL/dRe V_m + i dL/dIm V_m it writes
// grad[j] = (1/N) Im(e^{-i phi_j} S_j) for the given phase.  A block covers kBlock Q <= kSpan
// pixels of a row: one span.
template <int Q, bool FRACT, int MODE>
__global__ void __launch_bounds__(kBlock)
k_backward(const TrapCoef* __restrict__ coef, const TrapState* __restrict__ st, const HoloDesc* __restrict__ hd,
           int nx, int ny, float* __restrict__ phase, const float* __restrict__ G, float* __restrict__ grad,
           float inv_n) {
  static_assert(kBlock * Q <= kSpan, "one span per block");
  __shared__ float4 rec[rec_pad(kMaxTraps)];
  const int b = blockIdx.z, r = blockIdx.y;
  const int M = hd[b].m, off = hd[b].off;
  const TrapCoef* __restrict__ cf = coef + off;
  // the block's pixels: columns [c0, c0 + kBlock Q) of row r, referenced to their centre
  const int c0 = blockIdx.x * (kBlock * Q);
  const int cc = centre_col(c0, min(nx, c0 + kBlock * Q) - c0);
  const double Uc = (double)(2 * cc - (nx - 1)), Vr = (double)(2 * r - (ny - 1));
  for (int m = threadIdx.x; m < M; m += kBlock) {
    float th, w;
    if constexpr (MODE == 0) {
      const TrapState s = st[off + m];
      th = s.theta_rev;
      w = s.w;
    } else {
      const float gr = G[2 * (off + m)], gi = G[2 * (off + m) + 1];
      w = sqrtf(gr * gr + gi * gi);
      th = atan2f(gi, gr) * kInv2Pi;
    }
    const TrapCoef c = cf[m];
    stage_record(rec, m, block_slope(c, Uc), c.gf, block_const(c, Uc, Vr), th, w);
  }
  pad_records<kBlock>(rec, M);
  __syncthreads();
  const int cbase = c0 + threadIdx.x;
  float u[Q], u2[Q], sr[Q], si[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    u[q] = (float)(2 * (cbase + q * kBlock - cc));
    u2[q] = u[q] * u[q];
    sr[q] = 0.0f;
    si[q] = 0.0f;
  }
  pixel_terms<Q, FRACT>(rec, M, u, u2, sr, si);
  const size_t rowbase = (size_t)b * nx * ny + (size_t)r * nx;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = cbase + q * kBlock;
    if (c < nx) {
      if constexpr (MODE == 0) {
        phase[rowbase + c] = phase_of(si[q], sr[q]);
      } else {
        float sp, cp;
        sincosf(phase[rowbase + c], &sp, &cp);
        grad[rowbase + c] = (si[q] * cp - sr[q] * sp) * inv_n;
      }
    }
  }
}

// Trap pass alone on a given phase mask: block = one row segment of HS spans, kBlock threads.
// Dynamic LDS: refs_lds_bytes(HS, mmax).
template <int TPL, bool FRACT, int HS>
__global__ void __launch_bounds__(kBlock)
k_forward(const TrapCoef* __restrict__ coef, const HoloDesc* __restrict__ hd, const float* __restrict__ phase,
          int nx, int ny, int seg_w, int nseg, int mmax, float2* __restrict__ partial) {
  constexpr int W = kBlock / 64;
  __shared__ float4 px[HS * kSpanStride];
  __shared__ float2 red[W * 64 * TPL];
  extern __shared__ float4 refs[];
  const int rp = rec_pad(mmax), mp = k_stride(mmax);
  float* kts = reinterpret_cast<float*>(refs + HS * rp);
  const int b = blockIdx.z, r = blockIdx.y, sg = blockIdx.x;
  const int M = hd[b].m, G = hd[b].g, A = hd[b].a, off = hd[b].off;
  const TrapCoef* __restrict__ cf = coef + off;
  const int cbeg = sg * seg_w;
  const int len = min(nx, cbeg + seg_w) - cbeg;
  for (int m = threadIdx.x; m < M; m += kBlock)
    stage_spans<HS, 1>(refs, rp, kts, mp, m, cf[m], nx, cbeg, len, 2 * r - (ny - 1), 0.0f, 0.0f);
  const float* __restrict__ ph = phase + (size_t)b * nx * ny + (size_t)r * nx + cbeg;
  for (int i = threadIdx.x; i < HS * kSpanStride; i += kBlock) {
    const int h = i / kSpanStride, l = i - h * kSpanStride, c = kSpan * h + l;  // pixel c of the segment
    if (l < kSpan && c < len) {
      const int cc = centre_col(cbeg + kSpan * h, min(len - kSpan * h, kSpan));
      const float u = (float)(2 * (cbeg + c - cc));
      // any phase the caller passes, in revolutions within one period
      px[i] = make_float4(caller_phase_rev(ph[c]), u, u * u, 1.0f);
    } else {
      px[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
  __syncthreads();
  const int nblk = ny * nseg;
  float2* __restrict__ out = partial + (size_t)off * nblk + r * nseg + sg;
  trap_pass_block<W, HS, TPL, FRACT, 1>(refs, rp, kts, mp, M, G, A, px, len, red,
                                        [&](int m, float2 v) { out[(size_t)m * nblk] = v; });
}

// ------------------------------------------------------------------ reduce, update, finalize
//
// Grid (ceil(Mmax / 4), B), 256 threads: wave w of block x sums trap m = 4x + w over the
// nblk partials (lanes take every 64th block, then a butterfly; fixed order) -> V_m = sum / N.
__global__ void __launch_bounds__(256)
k_reduce(const float2* __restrict__ partial, const HoloDesc* __restrict__ hd, int nblk, float inv_n,
         float* __restrict__ V) {
  const int b = blockIdx.y;
  const int M = hd[b].m, off = hd[b].off;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (m >= M) return;
  const float2* __restrict__ p = partial + (size_t)(off + m) * nblk;
  float sr = 0.0f, si = 0.0f;
  for (int k = lane; k < nblk; k += 64) {
    const float2 v = p[k];
    sr += v.x;
    si += v.y;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    V[2 * (off + m)] = sr * inv_n;
    V[2 * (off + m) + 1] = si * inv_n;
  }
}

// V of all T traps from the fixed-point region sums of the direct path (one thread per trap).
__global__ void __launch_bounds__(256)
k_collect(const unsigned long long* __restrict__ acc, int T, float unscale, float* __restrict__ V) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= T) return;
  const float2 v = VAcc{acc, T, 0, unscale}(t);
  V[2 * t] = v.x;
  V[2 * t + 1] = v.y;
}

// End of a solve on the fixed-point path, one block per hologram: V of its traps from the sums
// (written to V) and their figures of merit into stats[b][kstat].
__global__ void __launch_bounds__(256)
k_finish(const unsigned long long* __restrict__ acc, int T, float unscale, const HoloDesc* __restrict__ hd,
         const TrapState* __restrict__ st, float* __restrict__ V, float* __restrict__ stats, int kstat,
         int stat_stride) {
  __shared__ float sh[8 * 4];
  const int b = blockIdx.x;
  const int M = hd[b].m, off = hd[b].off;
  const VAcc vacc{acc, T, off, unscale};
  for (int m = threadIdx.x; m < M; m += 256) {
    const float2 v = vacc(m);
    V[2 * (off + m)] = v.x;
    V[2 * (off + m) + 1] = v.y;
  }
  update_traps<256>(vacc, st, off, M, 0, sh, stats + 3 * ((size_t)b * stat_stride + kstat), nullptr,
                    [](int, const TrapState&) {});
}

// One block per hologram: figures of merit of V into stats[b][kstat] and, for mode 1/2,
// the GS/GSW update st_in -> st_out (st_out may equal st_in).
__global__ void __launch_bounds__(256)
k_update(const float* __restrict__ V, const HoloDesc* __restrict__ hd, const TrapState* st_in, TrapState* st_out,
         float* __restrict__ stats, int kstat, int stat_stride, int mode, int* __restrict__ flag) {
  __shared__ float sh[8 * 4];
  const int b = blockIdx.x;
  const int M = hd[b].m, off = hd[b].off;
  update_traps<256>(VArray{V, off}, st_in, off, M, mode, sh, stats + 3 * ((size_t)b * stat_stride + kstat), flag,
                    [&](int m, const TrapState& s) {
                      if (mode != 0) st_out[off + m] = s;
                    });
}

// ------------------------------------------------------------------ stored exp(i Delta) variant

// A[m][j] = exp(i 2pi Delta_rev): the argument is formed exactly in FP64 and reduced to one period
// before the FP32 sin/cos (a one-time table, so the FP64 work is cheap).
__global__ void __launch_bounds__(kBlock)
k_expdelta(const TrapCoef* __restrict__ coef, const HoloDesc* __restrict__ hd, int nx, int ny, float2* __restrict__ A) {
  const int b = blockIdx.z, m = blockIdx.y;
  const int M = hd[b].m, off = hd[b].off;
  if (m >= M) return;
  const int n = nx * ny;
  const TrapCoef c = coef[off + m];
  float2* __restrict__ row = A + (size_t)(off + m) * n;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
    const int r = j / nx, col = j - r * nx;
    const double U = (double)(2 * col - (nx - 1)), Vr = (double)(2 * r - (ny - 1));
    const double d = __builtin_fma(c.g, __builtin_fma(U, U, Vr * Vr), __builtin_fma(c.a, U, c.b * Vr));
    const float t = (float)(d - __builtin_floor(d));
    row[j] = make_float2(__builtin_amdgcn_cosf(t), __builtin_amdgcn_sinf(t));
  }
}

// S_j = sum_m (w e^{i theta})_m A[m][j]; phase = arg S, E_j = e^{i phase} for the forward pass.
__global__ void __launch_bounds__(kBlock)
k_backward_stored(const float2* __restrict__ A, const TrapState* __restrict__ st, const HoloDesc* __restrict__ hd,
                  int n, float* __restrict__ phase, float2* __restrict__ E) {
  __shared__ float2 cm[kMaxTraps];
  const int b = blockIdx.y;
  const int M = hd[b].m, off = hd[b].off;
  for (int m = threadIdx.x; m < M; m += kBlock) {
    const TrapState s = st[off + m];
    const float t = __builtin_amdgcn_fractf(s.theta_rev);
    cm[m] = make_float2(s.w * __builtin_amdgcn_cosf(t), s.w * __builtin_amdgcn_sinf(t));
  }
  __syncthreads();
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  const float2* __restrict__ col = A + (size_t)off * n + j;
  float sr = 0.0f, si = 0.0f;
#pragma unroll 16
  for (int m = 0; m < M; ++m) {
    const float2 v = col[(size_t)m * n];
    const float2 k = cm[m];
    sr = __builtin_fmaf(k.x, v.x, __builtin_fmaf(-k.y, v.y, sr));
    si = __builtin_fmaf(k.x, v.y, __builtin_fmaf(k.y, v.x, si));
  }
  const float ph = phase_of(si, sr);
  phase[(size_t)b * n + j] = ph;
  const float pr = ph * kInv2Pi;
  E[(size_t)b * n + j] = make_float2(__builtin_amdgcn_cosf(pr), __builtin_amdgcn_sinf(pr));
}

// Per wave: 64 * PPL pixels (PPL per lane, kept in registers); for each trap of its group the
// wave sums conj(A[m][j]) E_j over its pixels and writes one partial per (trap, wave).  Grid x =
// pixel blocks x tg trap groups: a hologram's traps are split into tg contiguous groups so that
// enough waves stream A at once to keep HBM busy (each (trap, pixel block) is still one wave).
template <int PPL>
__global__ void __launch_bounds__(kBlock)
k_forward_stored(const float2* __restrict__ A, const float2* __restrict__ E, const HoloDesc* __restrict__ hd, int n,
                 int tg, float2* __restrict__ partial) {
  const int b = blockIdx.y;
  const int M = hd[b].m, off = hd[b].off;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nblk = (n + 64 * PPL - 1) / (64 * PPL);
  const int nbx = (nblk + 3) / 4;
  const int grp = (int)blockIdx.x / nbx;
  const int blk = ((int)blockIdx.x - grp * nbx) * 4 + wave;
  const int mg = (M + tg - 1) / tg;
  const int m0 = grp * mg, m1 = min(M, m0 + mg);
  if (blk >= nblk || m0 >= m1) return;
  const int j0 = blk * 64 * PPL + lane;
  float er[PPL], ei[PPL];
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const int j = j0 + p * 64;
    const float2 e = j < n ? E[(size_t)b * n + j] : make_float2(0.0f, 0.0f);
    er[p] = e.x;
    ei[p] = e.y;
  }
  for (int m = m0; m < m1; ++m) {
    const float2* __restrict__ row = A + (size_t)(off + m) * n;
    float sr = 0.0f, si = 0.0f;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const int j = j0 + p * 64;
      const float2 v = j < n ? row[j] : make_float2(0.0f, 0.0f);
      sr = __builtin_fmaf(v.x, er[p], __builtin_fmaf(v.y, ei[p], sr));  // Re(conj(v) e)
      si = __builtin_fmaf(v.x, ei[p], __builtin_fmaf(-v.y, er[p], si)); // Im(conj(v) e)
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) partial[(size_t)(off + m) * nblk + blk] = make_float2(sr, si);
  }
}

// ------------------------------------------------------------------ separable reformulation (matrix cores)
//
// Eq. 2 separates per trap: Delta_rev = (g U^2 + a U) + (g V^2 + b V), so
//   e^{i 2pi Delta_j^m} = X_m(c) Y_m(r),  X_m(c) = e^{i 2pi (g U_c^2 + a U_c)},  Y_m(r) = e^{i 2pi (g V_r^2 + b V_r)}.
// With the trap weights c_m = w_m e^{i theta_m} the two passes become dense complex contractions:
//   pixel pass (Eq. 3)  S[r][c] = sum_m (c_m Y_m(r)) X_m(c),          phi = arg S
//   trap pass (Eq. 1)   T[r][m] = sum_c e^{i phi[r][c]} conj X_m(c),  V_m = (1/N) sum_r conj Y_m(r) T[r][m]
// of the same size as the direct sums, with the N*M transcendentals of Eq. 2 replaced by
// per-block tables of the two factors.  Both run on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32), each complex product as four real MFMAs.
//
// MFMA 16x16x4 operands: lane l = i + 16 k holds A[i][k] and B[k][i]; result D[i][j] is in
// lane j + 16 (i / 4), register i % 4.
//
// A block owns 16 rows x 16 W columns of the SLM, one wave per 16 x 16 tile (or, in the
// iteration, two waves per tile that split the traps, so that two waves share each SIMD):
//   pixel pass  D = X^T (columns x traps) . (c Y) (traps x rows); lane (j, g) ends with the
//               four pixels (row0 + j, col0 + 4 g + v), v = 0..3, in its four registers
//   epilogue    E = S / |S| = e^{i phase} of those pixels, kept in registers (and the phase,
//               arg S, where it is wanted)
//   trap pass   D = E (rows x columns) . conj X^T (columns x traps), the lane's four E values
//               taken as its four k-steps (the column sum runs in that permuted order, and the
//               B operand reads follow it), so E never leaves the registers; each lane then
//               folds its four rows against conj Y, and the four lane groups are combined.
// The block's tables X_m(c) (its 16 W columns) and Y_m(r), c_m Y_m(r) (its 16 rows) are
// computed into LDS from the per-trap coefficients, trap index fastest, for super-chunks of
// `sc` traps: (16 W + 16) sc sin/cos pairs per block, against 2 x 16 x 16 W x sc complex
// products of the passes.  In the pixel pass lane group g takes traps base + g nk + i at
// k-step i (i < nk), so each lane's operands are consecutive in LDS.  Every block
// recomputes the GS/GSW update from the previous V, as the direct kernel does.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float2 trap_weight(const TrapState& s) {
  return make_float2(s.w * __builtin_amdgcn_cosf(s.theta_rev), s.w * __builtin_amdgcn_sinf(s.theta_rev));
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Pixel pass operands of NK k-steps: xr -> X[column][traps], yr -> (c Y)[row][traps], NK
// consecutive complex entries each (16-byte aligned when NK is even).
template <int NK>
struct PixelOps {
  float2 x[NK], y[NK];
  __device__ __forceinline__ void load(const float2* xr, const float2* yr) {
    if constexpr (NK % 2 == 0) {
#pragma unroll
      for (int i = 0; i < NK; i += 2) {
        const float4 a = *reinterpret_cast<const float4*>(xr + i), c = *reinterpret_cast<const float4*>(yr + i);
        x[i] = make_float2(a.x, a.y);
        x[i + 1] = make_float2(a.z, a.w);
        y[i] = make_float2(c.x, c.y);
        y[i + 1] = make_float2(c.z, c.w);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NK; ++i) {
        x[i] = xr[i];
        y[i] = yr[i];
      }
    }
  }
  __device__ __forceinline__ void mma(f32x4& sre, f32x4& sim) const {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      sre = mfma16(x[i].x, y[i].x, sre);
      sre = mfma16(x[i].y, -y[i].y, sre);
      sim = mfma16(x[i].x, y[i].y, sim);
      sim = mfma16(x[i].y, y[i].x, sim);
    }
  }
};

template <int NK>
__device__ __forceinline__ void pixel_tail(const float2* xr, const float2* yr, f32x4& sre, f32x4& sim) {
  PixelOps<NK> o;
  o.load(xr, yr);
  o.mma(sre, sim);
}

// Sum over the four lane groups (lanes li, li + 16, li + 32, li + 48), the same value in every
// lane: (R0 + R1) + (R2 + R3) in rows 0 and 1, (R2 + R3) + (R0 + R1) in rows 2 and 3.
__device__ __forceinline__ float sum_lane_groups(float v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}

// Trap pass for NTL consecutive tiles of 16 traps: xc -> X[column 4g][trap li] (columns xs apart),
// yc -> Y[row 4g][trap li] (rows xs apart); tile t's trap sums over this wave's pixels go to
// out[16 t] from the lanes of group 0.  The tiles' MFMAs are interleaved, so one tile's folding
// and lane-group sums overlap the products of the others.
template <int NTL>
__device__ __forceinline__ void trap_tiles(const float2* xc, const float2* yc, int xs, const float* er,
                                           const float* ei, int g, float2* out) {
  float2 x[NTL][4], y[NTL][4];
#pragma unroll
  for (int t = 0; t < NTL; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      x[t][v] = xc[16 * t + v * xs];
      y[t][v] = yc[16 * t + v * xs];
    }
  }
  f32x4 tre[NTL], tim[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) {
    tre[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    tim[t] = tre[t];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
      tre[t] = mfma16(er[v], x[t][v].x, tre[t]);
      tre[t] = mfma16(ei[v], x[t][v].y, tre[t]);
      tim[t] = mfma16(ei[v], x[t][v].x, tim[t]);
      tim[t] = mfma16(er[v], -x[t][v].y, tim[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NTL; ++t) {
    float pr = 0.0f, pi = 0.0f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      pr = __builtin_fmaf(y[t][v].x, tre[t][v], __builtin_fmaf(y[t][v].y, tim[t][v], pr));   // Re(conj(y) t)
      pi = __builtin_fmaf(y[t][v].x, tim[t][v], __builtin_fmaf(-y[t][v].y, tre[t][v], pi));  // Im(conj(y) t)
    }
    pr = sum_lane_groups(pr);
    pi = sum_lane_groups(pi);
    if (g == 0) out[16 * t] = make_float2(pr, pi);
  }
}

// MODE 0: one iteration: update, pixel pass, trap pass (phase written when non-null).  As in k_iter,
//   V of the previous mask is the sum of acc_in's per-XCD fixed-point regions, each trap's block
//   sum is added to acc_out's region of the adding wave's XCD, and block (0, 0, b) clears
//   hologram b's part of acc_zero; acc_in is read even when upd == 0 (a valid buffer).
// MODE 1: trap pass alone from the given phase (Eq. 1): per-block partials
// MODE 2: pixel pass alone from the given state (phase out)
// MODE 3: adjoint of Eq. 1: weights G_m (vin), grad[j] = (1/N) Im(e^{-i phi_j} S_j) for the given phase
// KH = 2 (MODE 0): two waves per tile, each taking half of the k-steps of the pixel pass and half
//   of the trap tiles of the trap pass; the two partial pixel sums meet in LDS and are added in
//   a fixed order (first half + second half), so both waves hold the same S, and the phase is
//   written by the first.  Twice the waves per SIMD, the same work.
// Grid (ceil(nx / 16 W), ceil(ny / 16), B), W KH waves per block; sc = traps per super-chunk (a
// multiple of 16); dynamic LDS sep_lds_bytes(W, sc, Mmax, KH).  At least two waves per SIMD
// (<= 256 registers per wave, AGPRs included): on large grids two blocks then share a compute unit.
template <int W, int MODE, int KH>
__global__ void __launch_bounds__(W * KH * 64, 2)
k_sep(const TrapCoef* __restrict__ coef, const TrapState* __restrict__ st_in,
      const unsigned long long* __restrict__ acc_in, int one_m, int one_off, int T, float unscale, int nx, int ny,
      int sc, int upd, const HoloDesc* __restrict__ hd, TrapState* __restrict__ st_out,
      const float* __restrict__ vin, float* __restrict__ stats, int kstat, int stat_stride, int* __restrict__ flag,
      float inv_n, float* __restrict__ phase, float* __restrict__ grad, float2* __restrict__ partial,
      unsigned long long* __restrict__ acc_out, unsigned long long* __restrict__ acc_zero, float scale) {
  static_assert(KH == 1 || (KH == 2 && MODE == 0), "trap halves are built for the iteration only");
  constexpr int NW = W * KH, NT = NW * 64, CW = 16 * W;
  constexpr bool kPixel = MODE != 1, kTrap = MODE <= 1;
  extern __shared__ float4 lds4[];
  __shared__ float sh[8 * NW];
  const int b = blockIdx.z;
  // one_m > 0: a single hologram whose trap count and offset come by value (preloaded into
  // SGPRs with the other leading arguments), so the first coefficient and state loads wait for no
  // load of the descriptor
  int M = one_m, off = one_off;
  if (one_m <= 0) {
    M = hd[b].m;
    off = hd[b].off;
  }
  const int Mp = (M + 15) & ~15;
  const int XS = sc + 2;  // row stride of the table copies (float2), skewed across banks
  TrapCoef* cf = reinterpret_cast<TrapCoef*>(lds4);     // [Mp] FP64 coefficients
  float2* cw = reinterpret_cast<float2*>(cf + Mp);       // [Mp] c_m
  float2* xt = cw + Mp;                                  // [CW][XS] X_m(c)
  float2* yt = xt + CW * XS;                             // [16][XS] Y_m(r)
  float2* ywt = yt + 16 * XS;                            // [16][XS] c_m Y_m(r)
  float2* red = ywt + 16 * XS;                           // [NW][sc] per-wave trap sums
  float4* sx = reinterpret_cast<float4*>(red + NW * sc);  // KH = 2: [NW][64][2] partial pixel sums

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int tw = wave % W, half = wave / W;  // the wave's tile, and its share of the traps
  const int row0 = blockIdx.y * 16, cb = blockIdx.x * CW;
  const int c0 = cb + tw * 16;
  const int r = row0 + li;
  const size_t pix0 = (size_t)b * nx * ny + (size_t)r * nx + c0 + 4 * g;  // pixel (r, c0 + 4 g)
  bool in[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) in[v] = r < ny && c0 + 4 * g + v < nx;
  float er[4], ei[4];

  // tables of traps [k0, k0 + n) into LDS.  Eq. 2's factors are formed about a reference column
  // (row) of each group of 16: for the group's columns c = c_t + i, i in [-8, 8) (c_t = the group's
  // first column + 8),
  //   X_m(c) = e^{i 2pi (K_t + s_t i + 4 g i^2)},  K_t = g U_t^2 + a U_t (mod 1),  s_t = 4 g U_t + 2 a (mod 1)
  // with U_t = 2 c_t - (nx - 1) (exact for integer i); K_t and s_t are formed in FP64 (exact to
  // ~1e-16 rev) once per trap and group, and each entry's argument, under 5 rev, in FP32.  Rows
  // likewise, one group per block.  Lane j keeps trap k0 + j's group constants in registers while
  // its wave fills its share of the group's entries: wave w takes columns 16 (w % W) + (w / W) 16 / KH
  // + [0, 16 / KH) (tables_x) or rows w, w + NW, ... (tables_y).  Columns past nx and rows past ny
  // get the formula's values (finite, small arguments; such pixels have E = 0), and traps past M
  // are left as the formula gives them (c_m = 0, partials never written), so none of them reach
  // V or the phase.
  static_assert(16 % NW == 0, "rows of a block split evenly over its waves");
  auto group_ref = [](double g, double lin, double X) {  // (K, s) about integer coordinate X
    const double k = __builtin_fma(g, X * X, lin * X);
    double sl = __builtin_fma(4.0 * g, X, 2.0 * lin);
    sl -= __builtin_rint(sl);
    return make_float2((float)(k - __builtin_floor(k)), (float)sl);
  };
  auto factor = [](float2 ks, float q, int i) {
    const float fi = (float)i;
    const float t = __builtin_fmaf(q, fi * fi, __builtin_fmaf(ks.y, fi, ks.x));
    return make_float2(__builtin_amdgcn_cosf(t), __builtin_amdgcn_sinf(t));
  };
  const int xg = wave % W, xsub = wave / W;  // the column group this wave fills, and its share of it
  // (the wave's first column within its group is a compile-time constant in each branch, so the
  // entries' offsets i and i^2 fold into the code)
  auto tables_x_from = [&](auto first, int k0, int n) {
    constexpr int F = decltype(first)::value;
    const double Ut = (double)(2 * (cb + 16 * xg + 8) - (nx - 1));
    float2* row = xt + (16 * xg + F) * XS;
    for (int j = lane; j < n; j += 64) {
      const TrapCoef k = cf[k0 + j];
      const float2 ks = group_ref(k.g, k.a, Ut);
      const float q = (float)(4.0 * k.g);
#pragma unroll
      for (int i = 0; i < 16 / KH; ++i) row[i * XS + j] = factor(ks, q, F + i - 8);
    }
  };
  auto tables_x = [&](int k0, int n) {
    if (KH == 1 || xsub == 0) {
      tables_x_from(std::integral_constant<int, 0>{}, k0, n);
    } else {
      tables_x_from(std::integral_constant<int, 16 / KH>{}, k0, n);
    }
  };
  auto tables_y = [&](int k0, int n, bool weighted) {
    const double Vt = (double)(2 * (row0 + 8) - (ny - 1));
    for (int j = lane; j < n; j += 64) {
      const TrapCoef k = cf[k0 + j];
      const float2 ks = group_ref(k.g, k.b, Vt);
      const float q = (float)(4.0 * k.g);
      const float2 w = weighted ? cw[k0 + j] : make_float2(0.0f, 0.0f);
#pragma unroll
      for (int i = 0; i < 16 / NW; ++i) {
        const int row = wave + i * NW;
        const float2 v = factor(ks, q, row - 8);
        yt[row * XS + j] = v;
        if (weighted) ywt[row * XS + j] = cmul(w, v);
      }
    }
  };
  const int nsc = (Mp + sc - 1) / sc;

  // per-trap coefficients into LDS.  Trap threadIdx.x's coefficients, V and state are loaded
  // first; the block then builds the first super-chunk's X table (which needs no weights) while
  // the update's inputs arrive, and only then does the GS/GSW update.
  const VAcc vacc{acc_in, T, off, unscale};
  const bool lead = blockIdx.x == 0 && blockIdx.y == 0;
  // the coefficients are loaded unconditionally (threads past M read trap M - 1; their copies are
  // never used as trap threadIdx.x), so the values stay in registers
  const int tm = min((int)threadIdx.x, M - 1);
  // wave priority (kPriorityTraps traps or more): the update, the tables and the pixel pass at 1,
  // the trap pass at 0, so that the blocks sharing a compute unit reach the trap pass, and the
  // end, closer together (as in k_iter)
  if (M >= kPriorityTraps) __builtin_amdgcn_s_setprio(1);
  const TrapCoef c_first = coef[off + tm];
  if ((int)threadIdx.x < Mp) cf[threadIdx.x] = (int)threadIdx.x < M ? c_first : TrapCoef{0.0, 0.0, 0.0, 0.0f, 0.0f};
  __builtin_amdgcn_sched_barrier(0);
  // The state and V's words are read once the coefficients are in (those stay in the L2 from
  // launch to launch and return about a thousand cycles before the accumulators, which the
  // previous launch rewrote), so the first X table is built while these are in flight; V is
  // summed only where the update needs it.
  TrapState s_first = {0.0f, 0.0f, 0.0f, 0.0f};
  unsigned long long w_first[kAccRegions] = {};
  if (kPixel && MODE != 3) {
    s_first = st_in[off + tm];
    if (MODE == 0) vacc.load(tm, w_first);  // (acc_in is valid even when upd == 0)
  }
  if (MODE == 0 && lead) {
    for (int i = threadIdx.x; i < kAccRegions * M; i += NT) {
      const int gi = i / M;
      acc_zero[(size_t)gi * T + off + (i - gi * M)] = 0ull;
    }
  }
  for (int m = NT + (int)threadIdx.x; m < Mp; m += NT) cf[m] = m < M ? coef[off + m] : TrapCoef{0.0, 0.0, 0.0, 0.0f, 0.0f};
  __syncthreads();
  if constexpr (kPixel) {
    tables_x(0, min(sc, Mp));
    if (MODE == 3) {
      for (int m = threadIdx.x; m < M; m += NT) cw[m] = make_float2(vin[2 * (off + m)], vin[2 * (off + m) + 1]);
    } else if (MODE == 2 || upd == 0) {
      for (int m = threadIdx.x; m < M; m += NT) cw[m] = trap_weight(m == (int)threadIdx.x ? s_first : st_in[off + m]);
    } else {
      auto emit = [&](int m, const TrapState& st) {
        if (lead) st_out[off + m] = st;
        cw[m] = trap_weight(st);
      };
#pragma unroll
      for (int r = 0; r < kAccRegions; ++r) asm volatile("" : "+v"(w_first[r]));  // (the sum stays here)
      const float2 v_first = vacc.sum(w_first);
      update_traps<NT, VAcc, decltype(emit), true>(vacc, st_in, off, M, upd, sh,
                                                   lead ? stats + 3 * ((size_t)b * stat_stride + kstat) : nullptr,
                                                   lead ? flag : nullptr, emit, v_first, s_first);
    }
    for (int m = M + (int)threadIdx.x; m < Mp; m += NT) cw[m] = make_float2(0.0f, 0.0f);
    __syncthreads();
  }

  if constexpr (kPixel) {
    // S^T[c][r] = sum_m X[m][c] (c_m Y[m][r])
    f32x4 sre = {0.0f, 0.0f, 0.0f, 0.0f}, sim = sre;
    const float2* xrow = xt + (tw * 16 + li) * XS;
    const float2* yrow = ywt + li * XS;
    for (int s = 0; s < nsc; ++s) {
      const int k0 = s * sc, n = min(sc, Mp - k0);
      if (s > 0) {
        __syncthreads();  // the previous super-chunk is no longer read
        tables_x(k0, n);
      }
      tables_y(k0, n, true);
      __syncthreads();
      int ksteps = (min(n, M - k0) + 3) / 4;  // traps past M add nothing: skip them
      const float2* xs0 = xrow;
      const float2* ys0 = yrow;
      if constexpr (KH == 2) {  // the first half takes k-steps [0, kh), the second [kh, ksteps)
        const int kh = (ksteps + 1) / 2;
        if (half == 1) {
          xs0 += 4 * kh;
          ys0 += 4 * kh;
        }
        ksteps = half == 0 ? kh : ksteps - kh;
      }
      const int nfull = ksteps / 8;  // groups of 32 traps, operands double-buffered
      PixelOps<8> ga, gb;
      if (nfull > 0) ga.load(xs0 + 8 * g, ys0 + 8 * g);
      int q = 0;
      for (; q + 2 <= nfull; q += 2) {
        gb.load(xs0 + 32 * (q + 1) + 8 * g, ys0 + 32 * (q + 1) + 8 * g);
        __builtin_amdgcn_sched_barrier(0);
        ga.mma(sre, sim);
        __builtin_amdgcn_sched_barrier(0);
        if (q + 2 < nfull) ga.load(xs0 + 32 * (q + 2) + 8 * g, ys0 + 32 * (q + 2) + 8 * g);
        __builtin_amdgcn_sched_barrier(0);
        gb.mma(sre, sim);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (q < nfull) ga.mma(sre, sim);
      const int base = 32 * nfull, nk = ksteps - 8 * nfull;
      const float2* xr = xs0 + base + nk * g;
      const float2* yr = ys0 + base + nk * g;
      switch (nk) {
        case 1: pixel_tail<1>(xr, yr, sre, sim); break;
        case 2: pixel_tail<2>(xr, yr, sre, sim); break;
        case 3: pixel_tail<3>(xr, yr, sre, sim); break;
        case 4: pixel_tail<4>(xr, yr, sre, sim); break;
        case 5: pixel_tail<5>(xr, yr, sre, sim); break;
        case 6: pixel_tail<6>(xr, yr, sre, sim); break;
        case 7: pixel_tail<7>(xr, yr, sre, sim); break;
        default: break;
      }
    }
    if constexpr (KH == 2) {
      sx[(wave * 64 + lane) * 2] = make_float4(sre[0], sre[1], sre[2], sre[3]);
      sx[(wave * 64 + lane) * 2 + 1] = make_float4(sim[0], sim[1], sim[2], sim[3]);
      __syncthreads();
      const float4 r0 = sx[(tw * 64 + lane) * 2], i0 = sx[(tw * 64 + lane) * 2 + 1];
      const float4 r1 = sx[((W + tw) * 64 + lane) * 2], i1 = sx[((W + tw) * 64 + lane) * 2 + 1];
      sre = f32x4{r0.x + r1.x, r0.y + r1.y, r0.z + r1.z, r0.w + r1.w};
      sim = f32x4{i0.x + i1.x, i0.y + i1.y, i0.z + i1.z, i0.w + i1.w};
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if constexpr (MODE == 3) {
        if (in[v]) {
          const float pr = caller_phase_rev(phase[pix0 + v]);
          grad[pix0 + v] =
              inv_n * (__builtin_amdgcn_cosf(pr) * sim[v] - __builtin_amdgcn_sinf(pr) * sre[v]);  // Im(e^{-i phi} S)
        }
      } else {
        if (phase != nullptr && in[v] && half == 0) phase[pix0 + v] = phase_of(sim[v], sre[v]);
        const float n2 = sre[v] * sre[v] + sim[v] * sim[v];
        float cr = 1.0f, ci = 0.0f;  // arg 0 = 0
        if (n2 >= 1.17549435e-38f) {
          const float inv = __builtin_amdgcn_rsqf(n2);
          cr = sre[v] * inv;
          ci = sim[v] * inv;
        } else if (n2 > 0.0f) {
          const float pr = atan2f(sim[v], sre[v]) * kInv2Pi;
          cr = __builtin_amdgcn_cosf(pr);
          ci = __builtin_amdgcn_sinf(pr);
        }
        er[v] = in[v] ? cr : 0.0f;
        ei[v] = in[v] ? ci : 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float pr = in[v] ? caller_phase_rev(phase[pix0 + v]) : 0.0f;
      er[v] = in[v] ? __builtin_amdgcn_cosf(pr) : 0.0f;
      ei[v] = in[v] ? __builtin_amdgcn_sinf(pr) : 0.0f;
    }
  }

  __builtin_amdgcn_s_setprio(0);
  if constexpr (kTrap) {
    // per tile of 16 traps: T^T[r][m] = sum_c E[r][c] conj X[m][c], then sum_r conj Y[m][r] T^T[r][m]
    const int nblk = gridDim.x * gridDim.y, blk = blockIdx.y * gridDim.x + blockIdx.x;
    // super-chunks in reverse order: the pixel pass's last one is still in LDS (tables X and Y),
    // so it is taken first and only the others are rebuilt.  Each trap's sum lies within one
    // super-chunk, so the order changes no result.
    const float2* xcol = xt + (tw * 16 + 4 * g) * XS + li;
    const float2* ycol = yt + (4 * g) * XS + li;
    for (int s = nsc - 1; s >= 0; --s) {
      const int k0 = s * sc, n = min(sc, Mp - k0);
      if (!kPixel || s < nsc - 1) {
        if (kPixel || s < nsc - 1) __syncthreads();  // the previous super-chunk is no longer read
        tables_x(k0, n);
        tables_y(k0, n, false);
        __syncthreads();
      }
      // KH = 2: the first half takes tiles [0, th) of 16 traps, the second [th, n / 16)
      const int th = KH == 2 ? (n / 16 + 1) / 2 : n / 16;
      int t = KH == 2 && half == 1 ? 16 * th : 0;
      const int tend = KH == 2 && half == 0 ? 16 * th : n;
      for (; t + 128 <= tend; t += 128) trap_tiles<8>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li);
      switch ((tend - t) / 16) {
        case 1: trap_tiles<1>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li); break;
        case 2: trap_tiles<2>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li); break;
        case 3: trap_tiles<3>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li); break;
        case 4: trap_tiles<4>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li); break;
        case 5: trap_tiles<5>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li); break;
        case 6: trap_tiles<6>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li); break;
        case 7: trap_tiles<7>(xcol + t, ycol + t, XS, er, ei, g, red + wave * sc + t + li); break;
        default: break;
      }
      __syncthreads();
      for (int m = threadIdx.x; m < n && k0 + m < M; m += NT) {
        const float2* rm = red + (KH == 2 && m >= 16 * th ? W * sc : 0) + m;  // the half that took m
        float2 acc = rm[0];
#pragma unroll
        for (int w = 1; w < W; ++w) {
          acc.x += rm[w * sc].x;
          acc.y += rm[w * sc].y;
        }
        if constexpr (MODE == 0) {
          __hip_atomic_fetch_add(acc_out + (size_t)(xcc_id() & (kAccRegions - 1)) * T + off + k0 + m,
                                 pack_sum(acc, scale), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          partial[(size_t)(off + k0 + m) * nblk + blk] = acc;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ Table 1 ablation: the pixel pass of random superposition
//
// The paper's design rules for its pixel-pass kernel (Section 2; Table 1, Section 4) vary where a
// thread finds the trap parameters and how pixels map to threads.  These kernels time the same
// choices on gfx950 for the random-superposition pass (Eq. 3 with w_m = 1):
//   placement  LDS (records staged into shared memory, read as broadcasts), SCALAR (read from global
//              memory through the scalar cache: one load per wave), GLOBAL (read from global memory by
//              every lane: vector loads of one address)
//   mapping    LINEAR (a block is BS consecutive pixels of a row) or SQUARE (a block is a sqrt(BS) x
//              sqrt(BS) tile of pixels)
// Records are formed once per block by k_abl_records, in FP64 about the block's centre: LINEAR
// {a', g, K + theta_rev, 0} with t = g u^2 + a' u + C (2 FMA), SQUARE {a', b', g, K + theta_rev} with
// t = g (u^2 + v^2) + a' u + b' v + C (3 FMA: the row is no longer constant within a block).
enum { kAblLds = 0, kAblScalar = 1, kAblGlobal = 2 };
enum { kAblLinear = 0, kAblSquare = 1 };

template <int MAP>
__device__ __forceinline__ void abl_block(int blk, int nx, int ny, int BS, int& c0, int& r0, int& cw, int& rh) {
  if constexpr (MAP == kAblLinear) {
    const int nxb = (nx + BS - 1) / BS;
    r0 = blk / nxb;
    c0 = (blk - r0 * nxb) * BS;
    cw = BS;
    rh = 1;
  } else {
    const int side = BS == 64 ? 8 : 16;
    const int nxb = (nx + side - 1) / side;
    r0 = (blk / nxb) * side;
    c0 = (blk - blk / nxb * nxb) * side;
    cw = side;
    rh = side;
  }
}

// One block per pixel block, threads over traps: records[blk][m].
template <int MAP>
__global__ void __launch_bounds__(256)
k_abl_records(const TrapCoef* __restrict__ coef, const TrapState* __restrict__ st, int M, int nx, int ny, int BS,
              float4* __restrict__ records) {
  const int blk = blockIdx.x;
  int c0, r0, cw, rh;
  abl_block<MAP>(blk, nx, ny, BS, c0, r0, cw, rh);
  const int cc = centre_col(c0, min(nx - c0, cw)), rc = r0 + (max(min(ny - r0, rh), 1) - 1) / 2;
  const double Uc = (double)(2 * cc - (nx - 1)), Vc = (double)(2 * rc - (ny - 1));
  for (int m = threadIdx.x; m < M; m += 256) {
    const TrapCoef c = coef[m];
    const float k = block_const(c, Uc, Vc) + st[m].theta_rev;
    float4 r;
    if constexpr (MAP == kAblLinear) {
      r = make_float4(block_slope(c, Uc), c.gf, k, 0.0f);
    } else {
      double bp = __builtin_fma(2.0 * c.g, Vc, c.b);  // b' = b + 2 g Vc, mod 1/2 (v is even)
      bp -= 0.5 * __builtin_rint(2.0 * bp);
      r = make_float4(block_slope(c, Uc), (float)bp, c.gf, k);
    }
    records[(size_t)blk * M + m] = r;
  }
}

template <int PLACE, int MAP, int BS>
__global__ void __launch_bounds__(BS)
k_abl_pixel(const float4* __restrict__ records, int M, int nx, int ny, float* __restrict__ phase) {
  __shared__ float4 lrec[PLACE == kAblLds ? kMaxTraps : 1];
  const int blk = blockIdx.x;
  int c0, r0, cw, rh;
  abl_block<MAP>(blk, nx, ny, BS, c0, r0, cw, rh);
  const float4* __restrict__ rec = records + (size_t)blk * M;
  if constexpr (PLACE == kAblLds) {
    for (int m = threadIdx.x; m < M; m += BS) lrec[m] = rec[m];
    __syncthreads();
  }
  const int c = c0 + (MAP == kAblLinear ? (int)threadIdx.x : (int)threadIdx.x % cw);
  const int r = r0 + (MAP == kAblLinear ? 0 : (int)threadIdx.x / cw);
  const int cc = centre_col(c0, min(nx - c0, cw)), rc = r0 + (max(min(ny - r0, rh), 1) - 1) / 2;
  const float u = (float)(2 * (c - cc)), v = (float)(2 * (r - rc));
  const float u2 = MAP == kAblLinear ? u * u : u * u + v * v;
  // a lane-varying zero: makes the GLOBAL placement's record address a per-lane (vector) address
  int z = 0;
  if constexpr (PLACE == kAblGlobal) asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  auto load = [&](int m) {
    if constexpr (PLACE == kAblLds) return lrec[m];
    if constexpr (PLACE == kAblScalar) return rec[__builtin_amdgcn_readfirstlane(m)];
    return rec[m + z];
  };
  float sr = 0.0f, si = 0.0f;
  auto term = [&](const float4& q) {
    float t;
    if constexpr (MAP == kAblLinear) {
      t = __builtin_fmaf(q.y, u2, __builtin_fmaf(q.x, u, q.z));
    } else {
      t = __builtin_fmaf(q.z, u2, __builtin_fmaf(q.x, u, __builtin_fmaf(q.y, v, q.w)));
    }
    sr += __builtin_amdgcn_cosf(t);
    si += __builtin_amdgcn_sinf(t);
  };
  // eight records in flight per step, alike for every placement
  int m = 0;
  for (; m + 8 <= M; m += 8) {
    float4 q[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = load(m + i);
#pragma unroll
    for (int i = 0; i < 8; ++i) term(q[i]);
  }
  for (; m < M; ++m) term(load(m));
  if (c < nx && r < ny) phase[(size_t)r * nx + c] = phase_of(si, sr);
}

// ------------------------------------------------------------------ helpers

// 8-bit SLM frame: grey level = rint(phase * 256 / (2 pi)) mod 256 (FP32 product, round to even).
__global__ void __launch_bounds__(256) k_encode_u8(const float* __restrict__ phase, uint8_t* __restrict__ frame,
                                                   int64_t n) {
  constexpr float kLevelsPerRad = 40.7436654315252059f;  // FP32(256 / (2 pi))
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int level = (int)__builtin_rintf(phase[i] * kLevelsPerRad);
    frame[i] = (uint8_t)(level & 255);
  }
}

// dst[i] = src[i] for n 16-byte words; src may be pinned host memory (read through its device
// mapping), dst device memory.
__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

__global__ void k_fill_u32(unsigned* p, unsigned v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_export_state(const TrapState* __restrict__ st, int t, float* w_out, float* theta_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < t) {
    if (w_out) w_out[i] = st[i].w;
    if (theta_out) theta_out[i] = st[i].theta_rad;
  }
}

__global__ void k_import_w(const float* __restrict__ w0, TrapState* __restrict__ st, int t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < t) st[i].w = w0[i];
}

// ------------------------------------------------------------------ template dispatch

template <int NT, int Q, int TPL, bool FRACT, int ROWS>
hipError_t iter_rows(hipStream_t s, const IterArgs& a) {
  constexpr int HS = NT * Q / kSpan;
  if (a.fg.seg_w > NT * Q || !a.acc_in || !a.acc_out || !a.acc_zero || a.T < 1 || a.mmax < 1) return hipErrorInvalidValue;
  const size_t dyn = refs_lds_bytes(ROWS * HS, a.mmax);
  if (dyn + iter_static_lds(NT, Q, TPL, ROWS) > (size_t)kLdsMax) return hipErrorInvalidValue;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_iter<NT, Q, TPL, FRACT, ROWS>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     kLdsMax - (int)iter_static_lds(NT, Q, TPL, ROWS));
  if (attr != hipSuccess) return attr;
  dim3 grid(a.fg.nseg, (a.fg.ny + ROWS - 1) / ROWS, a.B);
  hipLaunchKernelGGL((k_iter<NT, Q, TPL, FRACT, ROWS>), grid, dim3(NT * ROWS), dyn, s, a.B == 1 ? a.one : HoloDesc{},
                     a.coef, a.st_in, a.acc_in, a.hd, a.st_out, a.acc_out, a.acc_zero, a.T, a.acc_scale, a.acc_unscale,
                     a.stats, a.kstat, a.stat_stride, a.upd, a.flag, a.fg.nx, a.fg.ny, a.fg.seg_w, a.mmax, a.phase);
  return hipGetLastError();
}

template <int NT, int Q, int TPL, bool FRACT>
hipError_t iter_t(hipStream_t s, const IterArgs& a) {
  if constexpr (NT == 256) {
    if (a.rows == 2) return iter_rows<NT, Q, TPL, FRACT, 2>(s, a);
  }
  if (a.rows != 1) return hipErrorInvalidValue;
  return iter_rows<NT, Q, TPL, FRACT, 1>(s, a);
}

template <int NT, int Q, bool FRACT>
hipError_t iter_tpl(hipStream_t s, const IterArgs& a) {
  switch (a.tpl) {
    case 1: return iter_t<NT, Q, 1, FRACT>(s, a);
    case 2: return iter_t<NT, Q, 2, FRACT>(s, a);
    case 3: return iter_t<NT, Q, 3, FRACT>(s, a);
    case 4: return iter_t<NT, Q, 4, FRACT>(s, a);
    case 5: return iter_t<NT, Q, 5, FRACT>(s, a);
    case 6: return iter_t<NT, Q, 6, FRACT>(s, a);
    case 8: return iter_t<NT, Q, 8, FRACT>(s, a);
    default: return hipErrorInvalidValue;
  }
}

template <bool FRACT>
hipError_t iter_shape(hipStream_t s, const IterArgs& a) {
  if (a.nt == 256 && a.q == 1) return iter_tpl<256, 1, FRACT>(s, a);
  if (a.nt == 256 && a.q == 2) return iter_tpl<256, 2, FRACT>(s, a);
  if (a.nt == 512 && a.q == 1) return iter_tpl<512, 1, FRACT>(s, a);
  if (a.nt == 512 && a.q == 2) return iter_tpl<512, 2, FRACT>(s, a);
  return hipErrorInvalidValue;
}

template <int Q, bool FRACT, int MODE>
hipError_t backward_q(hipStream_t s, int nx, int ny, int B, const TrapCoef* coef, const TrapState* st,
                      const HoloDesc* hd, float* phase, const float* G, float* grad, float inv_n) {
  dim3 grid((nx + kBlock * Q - 1) / (kBlock * Q), ny, B);
  hipLaunchKernelGGL((k_backward<Q, FRACT, MODE>), grid, dim3(kBlock), 0, s, coef, st, hd, nx, ny, phase, G, grad,
                     inv_n);
  return hipGetLastError();
}

template <bool FRACT, int MODE>
hipError_t backward_sel(hipStream_t s, int q, int nx, int ny, int B, const TrapCoef* coef, const TrapState* st,
                        const HoloDesc* hd, float* phase, const float* G, float* grad, float inv_n) {
  // one pixel per lane: a block is one span (kBlock = kSpan pixels)
  if (q != 1) return hipErrorInvalidValue;
  return backward_q<1, FRACT, MODE>(s, nx, ny, B, coef, st, hd, phase, G, grad, inv_n);
}

template <int TPL, bool FRACT, int HS>
hipError_t forward_hs(hipStream_t s, const FwdGeom& fg, int B, int mmax, const TrapCoef* coef, const HoloDesc* hd,
                      const float* phase, float2* partial) {
  const size_t dyn = refs_lds_bytes(HS, mmax);
  if (dyn + forward_static_lds(TPL, HS) > (size_t)kLdsMax) return hipErrorInvalidValue;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_forward<TPL, FRACT, HS>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     kLdsMax - (int)forward_static_lds(TPL, HS));
  if (attr != hipSuccess) return attr;
  dim3 grid(fg.nseg, fg.ny, B);
  hipLaunchKernelGGL((k_forward<TPL, FRACT, HS>), grid, dim3(kBlock), dyn, s, coef, hd, phase, fg.nx, fg.ny, fg.seg_w,
                     fg.nseg, mmax, partial);
  return hipGetLastError();
}

template <int TPL>
hipError_t forward_t(hipStream_t s, const FwdGeom& fg, int B, int mmax, bool fract, const TrapCoef* coef,
                     const HoloDesc* hd, const float* phase, float2* partial) {
  const bool two = fg.seg_w > kSpan;
  if (fract)
    return two ? forward_hs<TPL, true, 2>(s, fg, B, mmax, coef, hd, phase, partial)
               : forward_hs<TPL, true, 1>(s, fg, B, mmax, coef, hd, phase, partial);
  return two ? forward_hs<TPL, false, 2>(s, fg, B, mmax, coef, hd, phase, partial)
             : forward_hs<TPL, false, 1>(s, fg, B, mmax, coef, hd, phase, partial);
}

}  // namespace

hipError_t launch_iter(hipStream_t s, const IterArgs& a) {
  return a.fract ? iter_shape<true>(s, a) : iter_shape<false>(s, a);
}

hipError_t launch_backward(hipStream_t s, int nx, int ny, int B, bool fract, int q, const TrapCoef* coef,
                           const TrapState* st, const HoloDesc* hd, float* phase, int mode, const float* G,
                           float* grad) {
  const float inv_n = 1.0f / ((float)nx * (float)ny);
  if (mode == 0)
    return fract ? backward_sel<true, 0>(s, q, nx, ny, B, coef, st, hd, phase, G, grad, inv_n)
                 : backward_sel<false, 0>(s, q, nx, ny, B, coef, st, hd, phase, G, grad, inv_n);
  return fract ? backward_sel<true, 1>(s, q, nx, ny, B, coef, st, hd, phase, G, grad, inv_n)
               : backward_sel<false, 1>(s, q, nx, ny, B, coef, st, hd, phase, G, grad, inv_n);
}

hipError_t launch_forward(hipStream_t s, const FwdGeom& fg, int B, int mmax, int tpl, bool fract,
                          const TrapCoef* coef, const HoloDesc* hd, const float* phase, float2* partial) {
  if (fg.seg_w > kSegMax || mmax < 1) return hipErrorInvalidValue;
  switch (tpl) {
    case 1: return forward_t<1>(s, fg, B, mmax, fract, coef, hd, phase, partial);
    case 2: return forward_t<2>(s, fg, B, mmax, fract, coef, hd, phase, partial);
    case 3: return forward_t<3>(s, fg, B, mmax, fract, coef, hd, phase, partial);
    case 4: return forward_t<4>(s, fg, B, mmax, fract, coef, hd, phase, partial);
    case 5: return forward_t<5>(s, fg, B, mmax, fract, coef, hd, phase, partial);
    case 6: return forward_t<6>(s, fg, B, mmax, fract, coef, hd, phase, partial);
    case 8: return forward_t<8>(s, fg, B, mmax, fract, coef, hd, phase, partial);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(hipStream_t s, int B, int mmax, int nblk, float inv_n, const float2* partial,
                         const HoloDesc* hd, float* V) {
  dim3 grid((mmax + 3) / 4, B);
  hipLaunchKernelGGL(k_reduce, grid, dim3(256), 0, s, partial, hd, nblk, inv_n, V);
  return hipGetLastError();
}

hipError_t launch_finish(hipStream_t s, int B, int T, const unsigned long long* acc, float unscale,
                         const HoloDesc* hd, const TrapState* st, float* V, float* stats, int kstat,
                         int stat_stride) {
  hipLaunchKernelGGL(k_finish, dim3(B), dim3(256), 0, s, acc, T, unscale, hd, st, V, stats,
                     kstat, stat_stride);
  return hipGetLastError();
}

hipError_t launch_collect(hipStream_t s, int T, const unsigned long long* acc, float unscale, float* V) {
  hipLaunchKernelGGL(k_collect, dim3((T + 255) / 256), dim3(256), 0, s, acc, T, unscale, V);
  return hipGetLastError();
}

hipError_t launch_update(hipStream_t s, int B, const float* V, const HoloDesc* hd, const TrapState* st_in,
                         TrapState* st_out, float* stats, int kstat, int stat_stride, int mode, int* flag) {
  hipLaunchKernelGGL(k_update, dim3(B), dim3(256), 0, s, V, hd, st_in, st_out, stats, kstat, stat_stride, mode, flag);
  return hipGetLastError();
}

hipError_t launch_expdelta(hipStream_t s, int nx, int ny, int B, int mmax, const TrapCoef* coef,
                           const HoloDesc* hd, float2* A) {
  const int n = nx * ny;
  dim3 grid(std::min((n + kBlock - 1) / kBlock, 1024), mmax, B);
  hipLaunchKernelGGL(k_expdelta, grid, dim3(kBlock), 0, s, coef, hd, nx, ny, A);
  return hipGetLastError();
}

hipError_t launch_backward_stored(hipStream_t s, int n, int B, const float2* A, const TrapState* st,
                                  const HoloDesc* hd, float* phase, float2* E) {
  dim3 grid((n + kBlock - 1) / kBlock, B);
  hipLaunchKernelGGL(k_backward_stored, grid, dim3(kBlock), 0, s, A, st, hd, n, phase, E);
  return hipGetLastError();
}

hipError_t launch_forward_stored(hipStream_t s, int n, int B, int mmax, const float2* A, const float2* E,
                                 const HoloDesc* hd, float2* partial) {
  const int nblk = stored_nblk(n);
  // trap groups: about 4096 waves in all (four per SIMD), at most one per trap
  const int tg = std::max(1, std::min({mmax, 16, (4096 + nblk * B - 1) / (nblk * B)}));
  dim3 grid((nblk + 3) / 4 * tg, B);
  hipLaunchKernelGGL(k_forward_stored<kStoredPpl>, grid, dim3(kBlock), 0, s, A, E, hd, n, tg, partial);
  return hipGetLastError();
}

template <int W, int MODE, int KH>
hipError_t sep_t(hipStream_t s, const SepArgs& a) {
  // raise the kernel's dynamic LDS limit once, to everything the static part leaves
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sep<W, MODE, KH>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, kSepLdsMax);
  if (attr != hipSuccess) return attr;
  const size_t lds = sep_lds_bytes(W, a.sc, a.mmax, KH);
  if (lds > (size_t)kSepLdsMax) return hipErrorInvalidValue;
  dim3 grid(a.gx(), a.gy(), a.B);
  if (MODE == 0 && (!a.acc_in || !a.acc_out || !a.acc_zero || a.T < 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sep<W, MODE, KH>), grid, dim3(W * KH * 64), lds, s, a.coef, a.st_in, a.acc_in,
                     a.B == 1 ? a.one_m : 0, a.B == 1 ? a.one_off : 0, a.T, a.acc_unscale, a.nx, a.ny, a.sc, a.upd,
                     a.hd, a.st_out, a.vin, a.stats, a.kstat, a.stat_stride, a.flag, a.inv_n, a.phase, a.grad,
                     a.partial, a.acc_out, a.acc_zero, a.acc_scale);
  return hipGetLastError();
}

template <int W>
hipError_t sep_mode(hipStream_t s, const SepArgs& a) {
  switch (a.mode) {
    case 0: return a.kh == 2 ? sep_t<W, 0, 2>(s, a) : sep_t<W, 0, 1>(s, a);
    case 1: return sep_t<W, 1, 1>(s, a);
    case 2: return sep_t<W, 2, 1>(s, a);
    case 3: return sep_t<W, 3, 1>(s, a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sep(hipStream_t s, const SepArgs& a) {
  if (a.W != 1 && a.W != 2 && a.W != 4) return hipErrorInvalidValue;
  if (a.kh != 1 && a.kh != 2) return hipErrorInvalidValue;
  if (a.nx < 1 || a.ny < 1 || a.mmax < 1 || a.mmax > kMaxTraps || a.sc < 16 || a.sc % 16 != 0)
    return hipErrorInvalidValue;
  switch (a.W) {
    case 1: return sep_mode<1>(s, a);
    case 2: return sep_mode<2>(s, a);
    default: return sep_mode<4>(s, a);
  }
}

int abl_blocks(int mapping, int bs, int nx, int ny) {
  if (mapping == kAblLinear) return ((nx + bs - 1) / bs) * ny;
  const int side = bs == 64 ? 8 : 16;
  return ((nx + side - 1) / side) * ((ny + side - 1) / side);
}

hipError_t launch_abl_records(hipStream_t s, int mapping, int bs, int nx, int ny, int M, const TrapCoef* coef,
                              const TrapState* st, float4* records) {
  const int nb = abl_blocks(mapping, bs, nx, ny);
  if (mapping == kAblLinear)
    hipLaunchKernelGGL(k_abl_records<kAblLinear>, dim3(nb), dim3(256), 0, s, coef, st, M, nx, ny, bs, records);
  else
    hipLaunchKernelGGL(k_abl_records<kAblSquare>, dim3(nb), dim3(256), 0, s, coef, st, M, nx, ny, bs, records);
  return hipGetLastError();
}

template <int PLACE, int MAP>
hipError_t abl_bs(hipStream_t s, int bs, int nx, int ny, int M, const float4* records, float* phase) {
  const int nb = abl_blocks(MAP, bs, nx, ny);
  if (bs == 64)
    hipLaunchKernelGGL((k_abl_pixel<PLACE, MAP, 64>), dim3(nb), dim3(64), 0, s, records, M, nx, ny, phase);
  else
    hipLaunchKernelGGL((k_abl_pixel<PLACE, MAP, 256>), dim3(nb), dim3(256), 0, s, records, M, nx, ny, phase);
  return hipGetLastError();
}

template <int PLACE>
hipError_t abl_map(hipStream_t s, int mapping, int bs, int nx, int ny, int M, const float4* records, float* phase) {
  return mapping == kAblLinear ? abl_bs<PLACE, kAblLinear>(s, bs, nx, ny, M, records, phase)
                               : abl_bs<PLACE, kAblSquare>(s, bs, nx, ny, M, records, phase);
}

hipError_t launch_abl_pixel(hipStream_t s, int placement, int mapping, int bs, int nx, int ny, int M,
                            const float4* records, float* phase) {
  if ((bs != 64 && bs != 256) || (mapping != kAblLinear && mapping != kAblSquare) || M < 1 || M > kMaxTraps)
    return hipErrorInvalidValue;
  switch (placement) {
    case kAblLds: return abl_map<kAblLds>(s, mapping, bs, nx, ny, M, records, phase);
    case kAblScalar: return abl_map<kAblScalar>(s, mapping, bs, nx, ny, M, records, phase);
    case kAblGlobal: return abl_map<kAblGlobal>(s, mapping, bs, nx, ny, M, records, phase);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_encode_u8(hipStream_t s, const float* phase, uint8_t* frame, int64_t n) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_encode_u8, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, phase, frame, n);
  return hipGetLastError();
}

hipError_t launch_copy16(hipStream_t s, const void* src, void* dst, size_t n16) {
  if (n16 == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n16 + 255) / 256, 1024);
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t s, unsigned* p, unsigned v, int n) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_export_state(hipStream_t s, const TrapState* st, int t, float* w_out, float* theta_out) {
  hipLaunchKernelGGL(k_export_state, dim3((t + 255) / 256), dim3(256), 0, s, st, t, w_out, theta_out);
  return hipGetLastError();
}

hipError_t launch_import_w(hipStream_t s, const float* w0, TrapState* st, int t) {
  hipLaunchKernelGGL(k_import_w, dim3((t + 255) / 256), dim3(256), 0, s, w0, st, t);
  return hipGetLastError();
}

}  // namespace hot
