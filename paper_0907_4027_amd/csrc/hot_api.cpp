// hot_api.cpp -- the C ABI declared in include/hot.h: argument checks, per-trap
// coefficients (FP64 -> FP32, Eq. 2 in revolutions), trap-pass tiling, device buffers,
// and the launch sequences of RS / GS / GSW (Section 3, Fig. 2), the batched solver,
// Eq. 1 on its own and its adjoint.
#include "hot.h"
#include "hot_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace hot;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(e_ == hipErrorOutOfMemory ? HOT_ENOMEM : HOT_EDEVICE, "%s failed: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                             \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Staging {
  void* host = nullptr;  // pinned host memory
  void* dev = nullptr;   // the same memory as the device addresses it
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

constexpr int kRing = 8;
// captured launch sequences kept per context (least recently used dropped first): enough for a
// batch of holograms solved one by one into their own output buffers
constexpr int kGraphCache = 128;
constexpr double kPi = 3.14159265358979323846;

}  // namespace

struct hot_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  int variant = HOT_ONTHEFLY;
  int tune_q = 0, tune_tpl = 0, tune_seg = 0, tune_amax = 0, tune_sepw = 0, tune_sepc = 0, tune_rows = 0;
  int tune_sepk = 0;
  int tune_fract = 0;
  int num_cu = 256;  // compute units of the device (launch-shape choices)
  int use_graphs = 1;
  // captured launch sequences of solve(), keyed by everything they bake in (shapes, pointers)
  struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  DevBuf coef, st, hd, partial, stats, flag, amat, efield;
  DevBuf probe;  // micro-benchmark sink and clock stamps
  DevBuf abl;    // per-block records of the pixel-pass ablation
  DevBuf acc;  // fused paths: 3 rotating buffers of fixed-point trap sums [kAccRegions][T] u64 (re + 2^32 im)
  Staging ring[kRing];
  int ring_pos = 0;
  int* flag_host = nullptr;  // pinned
  // allocation-free entry point: the device address of this GPU's fixed workspace, and a pinned
  // host buffer of the same size (its device mapping, and an event behind its last upload), all
  // set up by hot_create
  void* scratch = nullptr;
  char* na_host = nullptr;
  char* na_dev = nullptr;
  hipEvent_t na_ev = nullptr;
  bool na_pending = false;
  // identity of the trap tables now on the device (skips re-upload and stored-matrix rebuilds)
  std::vector<double> key;
  bool amat_valid = false;
  std::vector<TrapCoef> h_coef;
  std::vector<TrapState> h_st;
  std::vector<HoloDesc> h_hd;
};

namespace {

int set_dev(hot_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  return HOT_OK;
}

int ensure(hot_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes <= b.cap) return HOT_OK;
  if (b.p) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(HOT_ENOMEM, "device allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
  }
  b.cap = want;
  return HOT_OK;
}

// Asynchronous host-to-device copy through a ring of pinned staging buffers, so the
// caller's host arrays may be reused as soon as the call returns.  The copy is a kernel on the
// context's stream that reads the pinned buffer through its device mapping (the runtime's own
// copy of a few hundred bytes was measured to stall the stream for ~0.5 ms after some launch
// sequences); a slot is reused only after the event behind its copy has completed.  Sizes are
// multiples of 16 bytes (the tables are arrays of 16- and 32-byte records).
int upload(hot_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return HOT_OK;
  if (bytes % 16 != 0) return fail(HOT_EINVAL, "internal: upload of %zu bytes is not a multiple of 16", bytes);
  Staging& s = c->ring[c->ring_pos];
  c->ring_pos = (c->ring_pos + 1) % kRing;
  if (s.pending) {
    HIP_TRY(hipEventSynchronize(s.ev));
    s.pending = false;
  }
  if (s.cap < bytes) {
    if (s.host) HIP_TRY(hipHostFree(s.host));
    s.host = nullptr;
    s.dev = nullptr;
    s.cap = 0;
    size_t want = std::max<size_t>(bytes, 4096);
    hipError_t e = hipHostMalloc(&s.host, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(HOT_ENOMEM, "pinned host allocation of %zu bytes failed", want);
    }
    e = hipHostGetDevicePointer(&s.dev, s.host, 0);
    if (e != hipSuccess || !s.dev) {
      (void)hipGetLastError();
      (void)hipHostFree(s.host);
      s.host = nullptr;
      s.dev = nullptr;
      return fail(HOT_EDEVICE, "pinned staging buffer has no device mapping");
    }
    s.cap = want;
  }
  memcpy(s.host, src, bytes);
  HIP_TRY(launch_copy16(c->stream, s.dev, dst, bytes / 16));
  HIP_TRY(hipEventRecord(s.ev, c->stream));
  s.pending = true;
  return HOT_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_slm(const hot_slm* slm) {
  if (!slm) return fail(HOT_EINVAL, "slm is NULL");
  if (slm->nx < 1 || slm->ny < 1 || slm->nx > HOT_MAX_SIDE || slm->ny > HOT_MAX_SIDE)
    return fail(HOT_EINVAL, "grid %d x %d outside 1..%d", slm->nx, slm->ny, HOT_MAX_SIDE);
  if (!finite_pos(slm->pitch) || !finite_pos(slm->wavelength) || !finite_pos(slm->focal))
    return fail(HOT_EINVAL, "pitch, wavelength and focal length must be finite and > 0");
  return HOT_OK;
}

int check_traps(int32_t m, const double* xyz, const char* what) {
  if (m < 1 || m > HOT_MAX_TRAPS) return fail(HOT_EINVAL, "%s: trap count %d outside 1..%d", what, m, HOT_MAX_TRAPS);
  if (!xyz) return fail(HOT_EINVAL, "%s: xyz is NULL", what);
  for (int64_t i = 0; i < 3LL * m; ++i)
    if (!std::isfinite(xyz[i])) return fail(HOT_EINVAL, "%s: xyz[%lld] is not finite", what, (long long)i);
  return HOT_OK;
}

uint64_t splitmix64_next(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Trap-pass lane layout for a hologram of m traps on a row segment of len pixels, for a
// block of W waves and tpl traps per lane: each wave = a slices x g trap lanes.  Returns an
// estimate of the block's cycles: per chunk of g*tpl traps, every lane walks its slice
// (slen pixels x tpl terms x 36 issue cycles, or the LDS read when tpl is small), then the
// block syncs and sums the S = W*a slice partials of each trap.
double layout_cost(int m, int len, int W, int tpl, int amax_cap, int& g, int& a) {
  int amax = std::max(1, std::min(16, len / (8 * W)));
  if (amax_cap > 0) amax = std::min(amax, amax_cap);
  double best = 1e300;
  g = 64;
  a = 1;
  for (int gg = 1; gg <= 64; ++gg) {
    const int aa = std::min(64 / gg, amax);
    const int S = W * aa;
    const int slen = (len + S - 1) / S;
    const int chunks = (m + gg * tpl - 1) / (gg * tpl);
    const int outs_per_thread = (gg * tpl + 64 * W - 1) / (64 * W);
    const double step = std::max(36.0 * tpl, 32.0);
    const double cost = chunks * (slen * step + 500.0 + 12.0 * S * outs_per_thread);
    if (cost < best - 1e-9) {
      best = cost;
      g = gg;
      a = aa;
    }
  }
  return best;
}

const int kTplChoices[] = {1, 2, 3, 4, 5, 6, 8};

// One traps-per-lane count for the whole launch (it is a template parameter of the kernel):
// the one with the least summed cost over the holograms.
int choose_tpl(const int32_t* counts, int B, int len, int W, int amax_cap) {
  int best_t = 1;
  double best = 1e300;
  for (int t : kTplChoices) {
    double cost = 0.0;
    for (int b = 0; b < B; ++b) {
      int g, a;
      cost += layout_cost(counts[b], len, W, t, amax_cap, g, a);
    }
    if (cost < best) {
      best = cost;
      best_t = t;
    }
  }
  return best_t;
}

struct Plan {
  int B = 0, T = 0, mmax = 0, nx = 0, ny = 0, n = 0;
  bool fract = false;
  // fused iteration kernel: row segments of <= nt*q pixels, nt threads, q pixels per lane
  FwdGeom fg{};
  int nt = 256, q = 1, tpl = 1, rows = 1;
  // stand-alone trap pass (hot_forward_V): row segments of <= kSegMax pixels, kBlock threads
  FwdGeom fgf{};
  int tplf = 1;
  int nblk_stored = 0;
  // separable variant: blocks of 16 rows x 16 sep_w columns, sep_sc traps per LDS super-chunk
  int sep_w = 4, nblk_sep = 0, sep_sc = 16;
  int sep_kh = 1;  // waves per 16 x 16 tile in the separable iteration (2: each takes half of the traps)
  // fused paths' fixed point: scale 2^s with s = 30 - ceil(log2 N) (re and im as 32-bit integers in
  // one 64-bit word); every block sum and every trap's total has magnitude <= N, so no sum of the
  // scaled parts leaves +-2^30
  float acc_scale = 0.0f, acc_unscale = 0.0f;
  HoloDesc one{};  // the first hologram's fused-kernel descriptor (passed by value when B == 1)
};

FwdGeom row_segments(int nx, int ny, int segmax) {
  FwdGeom f;
  f.nx = nx;
  f.ny = ny;
  f.nseg = (nx + segmax - 1) / segmax;
  f.seg_w = (nx + f.nseg - 1) / f.nseg;
  return f;
}

// Build the coefficient, state and descriptor tables of a problem on the host, into coef_out [T],
// st_out [T] and hd_out [2B] (the fused kernel's layouts, then the stand-alone trap pass's).
int prepare_into(hot_ctx* c, const hot_slm* slm, int B, const int32_t* counts, const double* xyz,
                 const double* theta0, bool seeded, uint64_t seed, Plan& P, TrapCoef* coef_out, TrapState* st_out,
                 HoloDesc* hd_out) {
  P.B = B;
  P.nx = slm->nx;
  P.ny = slm->ny;
  P.n = slm->nx * slm->ny;
  {
    int lg = 0;
    while ((1LL << lg) < (long long)P.n) ++lg;
    // fixed-point trap sums (re and im packed into one 64-bit word): any sum of at most N
    // unit-modulus terms stays within 2^30 units of 2^-(30 - lg)
    P.acc_scale = (float)std::ldexp(1.0, 30 - lg);
    P.acc_unscale = (float)(std::ldexp(1.0, lg - 30) / (double)P.n);
  }
  P.T = 0;
  P.mmax = 0;
  for (int b = 0; b < B; ++b) {
    P.T += counts[b];
    P.mmax = std::max(P.mmax, (int)counts[b]);
  }
  // fused kernel shape
  {
    const int q = c->tune_q == 2 ? 2 : 1;
    int segmax = 512 * q;
    if (c->tune_seg > 0) {
      segmax = std::min(segmax, c->tune_seg);
    } else if (c->tune_q == 0 && P.mmax >= 64 &&
               (B == 1 || (int64_t)row_segments(slm->nx, slm->ny, 512).nseg * slm->ny * B < 4 * c->num_cu)) {
      // 256-pixel segments for a hologram of 64 traps or more (or a batch whose 512-pixel grid
      // would leave fewer than four blocks per compute unit): the blocks sharing a unit finish
      // close together, and twice the blocks shorten the last one's trap pass.  Measured per
      // iteration in situ, 256 against 512 pixels: 512^2 x 100 15.4 against 16.5 us, 1024^2 x 256
      // 110.1 against 111.2 us, 768^2 x 81 25.0 against 29.6 us; with fewer traps the update and
      // the trap sums, repeated by every block, cost more than the tail saves (768^2 x 9 19.8
      // against 15.0 us, 1024 x 768 x 8 13.5 against 10.5 us), and a batch of 16 holograms of
      // 4..256 traps at 512^2 runs 2 % faster on 512-pixel segments
      segmax = 256;
    }
    P.fg = row_segments(slm->nx, slm->ny, segmax);
    // two pixels per lane once a segment outgrows 256 pixels (measured faster than one pixel on
    // 512-thread blocks: the pixel pass reuses each trap record twice)
    P.q = (c->tune_q == 0 && P.fg.seg_w > 256) ? 2 : q;
    P.nt = P.fg.seg_w <= 256 * P.q ? 256 : 512;
    // one row per block: two rows sharing an update and one set of trap-sum additions were
    // measured slower (GSW 512^2 x 100: 18.8 against 18.0 us per iteration)
    P.rows = P.nt == 256 && c->tune_rows > 0 ? c->tune_rows : 1;
  }
  // stand-alone trap pass: one 256-pixel span per block by default (twice the blocks of 512-pixel
  // segments; measured 6-7 % faster at 512^2 with 64 or 100 traps, 2 % at 1024^2 x 256)
  P.fgf = row_segments(slm->nx, slm->ny, c->tune_seg > 0 ? std::min(c->tune_seg, kSegMax) : kSpan);
  P.nblk_stored = stored_nblk(P.n);
  {
    // separable: the widest block (most waves sharing one update and one sum per trap) that
    // still gives every compute unit a block
    const int rows = (slm->ny + 15) / 16;
    int w = c->tune_sepw;
    if (w == 0) {
      w = 1;
      for (int cand : {4, 2}) {
        const int cols = (slm->nx + 16 * cand - 1) / (16 * cand);
        if ((int64_t)cols * rows * B >= 256) {
          w = cand;
          break;
        }
      }
    }
    P.sep_w = w;
    P.nblk_sep = ((slm->nx + 16 * w - 1) / (16 * w)) * rows;
    // two waves per tile when the grid has at most one block per compute unit (one wave per
    // SIMD otherwise); a larger grid already has two resident blocks per unit, and the split
    // only adds the exchange of the pixel sums (measured slower there)
    P.sep_kh = c->tune_sepk > 0 ? c->tune_sepk : (int64_t)P.nblk_sep * B <= 256 ? 2 : 1;
    // traps per LDS super-chunk: all of them when they fit, with room for a second resident
    // block per compute unit when the grid has more blocks than compute units
    const int mp = (P.mmax + 15) / 16 * 16;
    const size_t row_bytes = sep_lds_bytes(w, 16, P.mmax, P.sep_kh) - sep_lds_bytes(w, 0, P.mmax, P.sep_kh);
    const size_t fixed = sep_lds_bytes(w, 0, P.mmax, P.sep_kh);
    int sc = 16;
    for (int bpc : {2, 1}) {
      // (a block of more than four waves already fills its compute unit's registers)
      if (bpc == 2 && ((int64_t)P.nblk_sep * B <= 256 || w * P.sep_kh > 4)) continue;
      const size_t budget = (size_t)kSepLdsMax / bpc;
      if (budget <= fixed + row_bytes) continue;
      sc = (int)std::min<size_t>(mp / 16, (budget - fixed) / row_bytes) * 16;
      // equal super-chunks (multiples of 16): no short last one, whose tables (the ones the
      // trap pass reuses) would leave most lanes idle
      const int nsc = (mp + sc - 1) / sc;
      sc = ((mp + nsc - 1) / nsc + 15) / 16 * 16;
      break;
    }
    if (c->tune_sepc > 0) sc = std::min(mp, c->tune_sepc);
    P.sep_sc = std::max(16, sc);
  }

  // Eq. 2 in revolutions per pixel-index unit (hot_internal.h), in FP64; a and b are reduced to
  // [-1/2, 1/2] (exact: U and V are integers, so a U and b V change by whole revolutions)
  const double lf = slm->wavelength * slm->focal;
  const double ca = slm->pitch / (2.0 * lf);
  const double cg = slm->pitch * slm->pitch / (8.0 * lf * slm->focal);
  double gmax = 0.0, amax = 0.0;
  uint64_t sm = seed;
  for (int t = 0; t < P.T; ++t) {
    const double x = xyz[3 * t], y = xyz[3 * t + 1], z = xyz[3 * t + 2];
    TrapCoef k;
    k.a = ca * x;
    k.a -= std::rint(k.a);
    k.b = ca * y;
    k.b -= std::rint(k.b);
    k.g = cg * z;
    k.gf = (float)k.g;
    k.pad = 0.0f;
    coef_out[t] = k;
    gmax = std::max(gmax, std::fabs(k.g));
    amax = std::max(amax, std::fabs(k.a) + 2.0 * std::fabs(k.g) * (slm->nx - 1));
    double th;
    if (seeded)
      th = 2.0 * kPi * (double)(splitmix64_next(sm) >> 40) * (1.0 / 16777216.0);
    else
      th = theta0[t];
    if (!std::isfinite(th)) return fail(HOT_EINVAL, "theta0[%d] is not finite", t);
    TrapState s;
    s.theta_rad = (float)th;
    s.theta_rev = s.theta_rad * 0.159154943091895336f;
    s.w = 1.0f;
    s.pad = 0.0f;
    st_out[t] = s;
  }
  // Largest per-term argument of the direct passes, |g u^2 + a' u + C| with |a'| <= min(1/4, |a| + 2|g| Uc)
  // (a' is reduced mod 1/2), |C| < 3/2 and |u| at most the widest block of any pass in U units (the
  // fused iteration, the stand-alone pixel pass of kBlock pixels and the stand-alone trap pass).
  // The hardware sin/cos take |x| < 256 rev; beyond a margin the passes reduce each argument
  // explicitly (fract, one more instruction per term), as they do when the tuning knob asks.
  const double umax = (double)std::max({P.fg.seg_w, P.fgf.seg_w, kBlock * 2});
  const double bound = gmax * umax * umax + std::min(0.25, amax) * umax + 2.5;
  P.fract = c->tune_fract == 1 || bound > 240.0;
  // the fused kernel's LDS (static part, plus records and K for every (row, span) pair) must fit a
  // compute unit; for very many traps the planner falls back to one row per block, then to
  // segments of at most 512 pixels
  auto iter_lds = [&]() {
    const int hs = P.nt * P.q / kSpan;
    return refs_lds_bytes(P.rows * hs, P.mmax) + iter_static_lds(P.nt, P.q, kTplMax, P.rows);
  };
  if (iter_lds() > (size_t)kLdsMax && P.rows == 2) P.rows = 1;
  if (iter_lds() > (size_t)kLdsMax && P.fg.seg_w > 512) {
    P.fg = row_segments(slm->nx, slm->ny, 512);
    P.q = P.fg.seg_w > 256 ? 2 : 1;
    P.nt = 256;
  }
  if (iter_lds() > (size_t)kLdsMax)
    return fail(HOT_EINVAL, "%d traps do not fit the iteration kernel's LDS with this launch shape", P.mmax);
  const int Wi = P.nt / 64, Wf = kBlock / 64;
  P.tpl = c->tune_tpl > 0 ? c->tune_tpl : choose_tpl(counts, B, P.fg.seg_w, Wi, c->tune_amax);
  P.tplf = c->tune_tpl > 0 ? c->tune_tpl : choose_tpl(counts, B, P.fgf.seg_w, Wf, c->tune_amax);
  int off = 0;
  for (int b = 0; b < B; ++b) {
    HoloDesc h{};
    h.m = counts[b];
    h.off = off;
    h.tpl = P.tpl;
    layout_cost(h.m, P.fg.seg_w, Wi, P.tpl, c->tune_amax, h.g, h.a);
    hd_out[b] = h;
    if (b == 0) P.one = h;
    h.tpl = P.tplf;
    layout_cost(h.m, P.fgf.seg_w, Wf, P.tplf, c->tune_amax, h.g, h.a);
    hd_out[B + b] = h;
    off += counts[b];
  }
  return HOT_OK;
}

int prepare(hot_ctx* c, const hot_slm* slm, int B, const int32_t* counts, const double* xyz, const double* theta0,
            bool seeded, uint64_t seed, Plan& P) {
  int64_t T = 0;
  for (int b = 0; b < B; ++b) T += counts[b];
  c->h_coef.resize(T);
  c->h_st.resize(T);
  c->h_hd.resize(2 * (size_t)B);
  return prepare_into(c, slm, B, counts, xyz, theta0, seeded, seed, P, c->h_coef.data(), c->h_st.data(),
                      c->h_hd.data());
}

// Device tables: coef [T], hd [2B] (fused-kernel layouts, then stand-alone trap-pass
// layouts), state [2T] (double buffer: iteration k reads one half and writes the other).
int upload_tables(hot_ctx* c, const hot_slm* slm, const Plan& P, const double* xyz, const int32_t* counts,
                  bool with_state = true) {
  std::vector<double> key;
  key.reserve(10 + P.B + 3 * (size_t)P.T);
  key.push_back(slm->nx);
  key.push_back(slm->ny);
  key.push_back(slm->pitch);
  key.push_back(slm->wavelength);
  key.push_back(slm->focal);
  key.push_back(c->tune_q);
  key.push_back(c->tune_tpl);
  key.push_back(c->tune_seg);
  key.push_back(c->tune_amax);
  key.push_back(c->tune_sepw);
  key.push_back(P.B);
  for (int b = 0; b < P.B; ++b) key.push_back(counts[b]);
  key.insert(key.end(), xyz, xyz + 3 * (size_t)P.T);
  int rc;
  if ((rc = ensure(c, c->st, 2 * sizeof(TrapState) * P.T))) return rc;
  if (with_state && (rc = upload(c, c->st.p, c->h_st.data(), sizeof(TrapState) * P.T))) return rc;
  if (key == c->key && c->coef.p && c->hd.p) return HOT_OK;
  c->key.clear();
  c->amat_valid = false;
  if ((rc = ensure(c, c->coef, sizeof(TrapCoef) * P.T))) return rc;
  if ((rc = ensure(c, c->hd, sizeof(HoloDesc) * 2 * P.B))) return rc;
  if ((rc = upload(c, c->coef.p, c->h_coef.data(), sizeof(TrapCoef) * P.T))) return rc;
  if ((rc = upload(c, c->hd.p, c->h_hd.data(), sizeof(HoloDesc) * 2 * P.B))) return rc;
  c->key.swap(key);
  return HOT_OK;
}

// Read the device degenerate flag (after a stream sync) and clear it.
int take_flag(hot_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->flag_host, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (*c->flag_host) {
    HIP_TRY(launch_fill_u32(c->stream, (unsigned*)c->flag.p, 0u, 1));
    return fail(HOT_EDEGENERATE, "GSW/GS met <|V|> = 0: the phase mask sends no light to any trap");
  }
  return HOT_OK;
}

enum Algo { kRS = 0, kGS = 1, kGSW = 2 };

int ensure_stored(hot_ctx* c, const Plan& P) {
  int rc;
  if ((rc = ensure(c, c->efield, sizeof(float2) * (size_t)P.B * P.n))) return rc;
  if (!c->amat_valid || c->amat.cap < sizeof(float2) * (size_t)P.T * P.n) {
    if ((rc = ensure(c, c->amat, sizeof(float2) * (size_t)P.T * P.n))) return rc;
    HIP_TRY(launch_expdelta(c->stream, P.nx, P.ny, P.B, P.mmax, (const TrapCoef*)c->coef.p,
                            (const HoloDesc*)c->hd.p, (float2*)c->amat.p));
    c->amat_valid = true;
  }
  return HOT_OK;
}

SepArgs sep_args(hot_ctx* c, const Plan& P, int mode, float* phase, int K) {
  SepArgs a;
  a.mode = mode;
  a.W = P.sep_w;
  a.B = P.B;
  a.nx = P.nx;
  a.ny = P.ny;
  a.mmax = P.mmax;
  a.sc = P.sep_sc;
  a.kh = mode == 0 ? P.sep_kh : 1;
  a.one_m = P.one.m;
  a.one_off = P.one.off;
  a.coef = (const TrapCoef*)c->coef.p;
  a.hd = (const HoloDesc*)c->hd.p;
  a.stats = (float*)c->stats.p;
  a.stat_stride = K + 1;
  a.flag = (int*)c->flag.p;
  a.inv_n = (float)(1.0 / (double)P.n);
  a.phase = phase;
  a.partial = (float2*)c->partial.p;
  a.T = P.T;
  a.acc_scale = P.acc_scale;
  a.acc_unscale = P.acc_unscale;
  return a;
}

// Buffer i (0..2) of the iteration kernels' rotating fixed-point sums.
unsigned long long* acc_buf(hot_ctx* c, const Plan& P, int i) {
  return (unsigned long long*)c->acc.p + (size_t)i * kAccRegions * P.T;
}
int ensure_acc(hot_ctx* c, const Plan& P) { return ensure(c, c->acc, 3 * sizeof(uint64_t) * kAccRegions * P.T); }

IterArgs iter_args(hot_ctx* c, const Plan& P, float* phase, int K) {
  IterArgs a;
  a.T = P.T;
  a.acc_scale = P.acc_scale;
  a.acc_unscale = P.acc_unscale;
  a.fg = P.fg;
  a.B = P.B;
  a.nt = P.nt;
  a.q = P.q;
  a.tpl = P.tpl;
  a.rows = P.rows;
  a.mmax = P.mmax;
  if (P.B == 1) a.one = P.one;
  a.fract = P.fract;
  a.coef = (const TrapCoef*)c->coef.p;
  a.hd = (const HoloDesc*)c->hd.p;
  a.stats = (float*)c->stats.p;
  a.stat_stride = K + 1;
  a.flag = (int*)c->flag.p;
  a.phase = phase;
  return a;
}

int solve(hot_ctx* c, const hot_slm* slm, int B, const int32_t* counts, const double* xyz, const double* theta0,
          bool seeded, uint64_t seed, int algo, int iters, const float* w0, float* w_out, float* theta_out,
          float* phase, float* V, hot_stats* stats, int variant) {
  int rc;
  if ((rc = set_dev(c))) return rc;
  Plan P;
  if ((rc = prepare(c, slm, B, counts, xyz, theta0, seeded, seed, P))) return rc;
  const int K = algo == kRS ? 0 : iters;
  const bool stored = variant == HOT_STORED;
  const bool separable = variant == HOT_SEPARABLE;
  const int nblk = stored ? P.nblk_stored : separable ? P.nblk_sep : P.fg.nblk();
  if ((rc = upload_tables(c, slm, P, xyz, counts))) return rc;
  if (stored && (rc = ensure(c, c->partial, sizeof(float2) * (size_t)P.T * nblk))) return rc;
  if ((rc = ensure(c, c->stats, sizeof(float) * 3 * (size_t)B * (K + 1)))) return rc;
  if (stored && (rc = ensure_stored(c, P))) return rc;
  if (!stored && (rc = ensure_acc(c, P))) return rc;
  TrapState* st[2] = {(TrapState*)c->st.p, (TrapState*)c->st.p + P.T};
  if (w0) HIP_TRY(launch_import_w(c->stream, w0, st[0], P.T));

  const HoloDesc* hd = (const HoloDesc*)c->hd.p;
  float2* part = (float2*)c->partial.p;
  float* dstats = (float*)c->stats.p;
  const float inv_n = (float)(1.0 / (double)P.n);
  const int upd = algo == kGSW ? 2 : 1;

  // The K-iteration launch sequence (one kernel per iteration on the fused paths, four on the stored one).
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    hipError_t e = hipSuccess;
    if (separable) {
      // one launch per iteration, with the same rotation of fixed-point sums as the direct path
      SepArgs a = sep_args(c, P, 0, phase, K);
      e = launch_fill_u32(s, (unsigned*)acc_buf(c, P, 1), 0u, 2 * kAccRegions * P.T);
      for (int k = 0; k <= K && e == hipSuccess; ++k) {
        a.upd = k == 0 ? 0 : upd;
        a.st_in = k == 0 ? st[0] : st[(k - 1) & 1];
        a.st_out = st[k & 1];
        a.acc_in = acc_buf(c, P, k % 3);
        a.acc_out = acc_buf(c, P, (k + 1) % 3);
        a.acc_zero = acc_buf(c, P, (k + 2) % 3);
        a.kstat = k - 1;
        a.phase = k == K ? phase : nullptr;  // only the last mask's phase is returned
        e = launch_sep(s, a);
      }
    } else if (!stored) {
      // one launch per iteration: launch k reads buffer k % 3, adds into (k + 1) % 3 (buffer 1 is
      // cleared first, the others by the launches) and clears (k + 2) % 3
      IterArgs a = iter_args(c, P, phase, K);
      e = launch_fill_u32(s, (unsigned*)acc_buf(c, P, 1), 0u, 2 * kAccRegions * P.T);
      for (int k = 0; k <= K && e == hipSuccess; ++k) {
        a.upd = k == 0 ? 0 : upd;
        a.st_in = k == 0 ? st[0] : st[(k - 1) & 1];
        a.st_out = st[k & 1];
        a.acc_in = acc_buf(c, P, k % 3);
        a.acc_out = acc_buf(c, P, (k + 1) % 3);
        a.acc_zero = acc_buf(c, P, (k + 2) % 3);
        a.kstat = k - 1;
        a.phase = k == K ? phase : nullptr;  // only the last mask's phase is returned
        e = launch_iter(s, a);
      }
    } else {
      for (int k = 0; k <= K && e == hipSuccess; ++k) {
        if (k > 0)
          e = launch_update(s, B, V, hd, st[(k - 1) & 1], st[k & 1], dstats, k - 1, K + 1, upd, (int*)c->flag.p);
        if (e == hipSuccess)
          e = launch_backward_stored(s, P.n, B, (const float2*)c->amat.p, st[k & 1], hd, phase, (float2*)c->efield.p);
        if (e == hipSuccess)
          e = launch_forward_stored(s, P.n, B, P.mmax, (const float2*)c->amat.p, (const float2*)c->efield.p, hd,
                                    part);
        if (e == hipSuccess) e = launch_reduce(s, B, P.mmax, nblk, inv_n, part, hd, V);
      }
    }
    // the final mask's V and figures of merit (fused paths: from the last buffer of sums)
    if (e == hipSuccess)
      e = stored ? launch_update(s, B, V, hd, st[K & 1], st[K & 1], dstats, K, K + 1, 0, (int*)c->flag.p)
                 : launch_finish(s, B, P.T, acc_buf(c, P, (K + 1) % 3), P.acc_unscale, hd, st[K & 1], V, dstats, K,
                                 K + 1);
    if (e == hipSuccess && (w_out || theta_out)) e = launch_export_state(s, st[K & 1], P.T, w_out, theta_out);
    return e;
  };

  // Replay a captured graph of the sequence when one with the same shapes and pointers
  // exists (captured on the context's own stream, launched on the caller's).
  bool done = false;
  if (c->use_graphs) {
    std::vector<uint64_t> key = {(uint64_t)B, (uint64_t)P.T, (uint64_t)P.nx, (uint64_t)P.ny, (uint64_t)K,
                                 (uint64_t)algo, (uint64_t)variant, (uint64_t)P.fract, (uint64_t)P.nt, (uint64_t)P.q,
                                 (uint64_t)P.tpl, (uint64_t)P.fg.seg_w, (uint64_t)P.sep_w, (uint64_t)P.sep_sc, (uint64_t)P.sep_kh,
                                 (uint64_t)P.rows, (uint64_t)(uintptr_t)phase,
                                 (uint64_t)(uintptr_t)V, (uint64_t)(uintptr_t)w_out, (uint64_t)(uintptr_t)theta_out,
                                 (uint64_t)(uintptr_t)c->coef.p, (uint64_t)(uintptr_t)c->st.p,
                                 (uint64_t)(uintptr_t)c->hd.p, (uint64_t)(uintptr_t)c->partial.p,
                                 (uint64_t)(uintptr_t)c->stats.p, (uint64_t)(uintptr_t)c->amat.p,
                                 (uint64_t)(uintptr_t)c->efield.p, (uint64_t)(uintptr_t)c->acc.p};
    hot_ctx::GraphEntry* hit = nullptr;
    for (auto& g : c->graphs)
      if (g.key == key) hit = &g;
    if (!hit) {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      bool ok = hipStreamBeginCapture(c->own_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        const hipError_t e = enqueue(c->own_stream);
        const hipError_t e2 = hipStreamEndCapture(c->own_stream, &graph);
        ok = e == hipSuccess && e2 == hipSuccess && graph &&
             hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
      }
      if (!ok) {  // capture not available: run eagerly from now on
        (void)hipGetLastError();
        c->use_graphs = 0;
      } else {
        if (c->graphs.size() >= (size_t)kGraphCache) {
          auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                      [](const auto& x, const auto& y) { return x.last_use < y.last_use; });
          (void)hipGraphExecDestroy(lru->exec);
          c->graphs.erase(lru);
        }
        c->graphs.push_back({std::move(key), exec, 0});
        hit = &c->graphs.back();
      }
    }
    if (hit) {
      hit->last_use = ++c->graph_clock;
      HIP_TRY(hipGraphLaunch(hit->exec, c->stream));
      done = true;
    }
  }
  if (!done) HIP_TRY(enqueue(c->stream));
  if (stats) {
    HIP_TRY(hipMemcpyAsync(stats, dstats, sizeof(float) * 3 * (size_t)B * (K + 1), hipMemcpyDeviceToHost,
                           c->stream));
    return take_flag(c);
  }
  return HOT_OK;
}

int check_batch(const hot_slm* slm, int32_t B, const int32_t* M, const double* xyz, int64_t& T) {
  int rc;
  if ((rc = check_slm(slm))) return rc;
  if (B < 1 || B > HOT_MAX_BATCH) return fail(HOT_EINVAL, "batch size %d outside 1..%d", B, HOT_MAX_BATCH);
  if (!M) return fail(HOT_EINVAL, "M (trap counts) is NULL");
  T = 0;
  for (int b = 0; b < B; ++b) {
    if (M[b] < 1 || M[b] > HOT_MAX_TRAPS)
      return fail(HOT_EINVAL, "hologram %d: trap count %d outside 1..%d", b, M[b], HOT_MAX_TRAPS);
    T += M[b];
  }
  if (T > (1LL << 24)) return fail(HOT_EINVAL, "total trap count %lld too large", (long long)T);
  if (!xyz) return fail(HOT_EINVAL, "xyz is NULL");
  for (int64_t i = 0; i < 3 * T; ++i)
    if (!std::isfinite(xyz[i])) return fail(HOT_EINVAL, "xyz[%lld] is not finite", (long long)i);
  return HOT_OK;
}

// Layout of the allocation-free entry point's workspace for T traps and K iterations (byte
// offsets, each region 256-byte aligned): coefficients [T], state [2][T], descriptors [2],
// fixed-point trap sums [3][kAccRegions][T], statistics [K+1][3], the degenerate flag.  The
// pinned staging buffer uses the same offsets.
struct NoallocLayout {
  size_t coef, st, hd, acc, stats, flag, total;
};
NoallocLayout noalloc_layout(int T, int K) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  NoallocLayout L{};
  size_t o = 0;
  L.coef = o;
  o = up(o + sizeof(TrapCoef) * (size_t)T);
  L.st = o;
  o = up(o + 2 * sizeof(TrapState) * (size_t)T);
  L.hd = o;
  o = up(o + 2 * sizeof(HoloDesc));
  L.acc = o;
  o = up(o + 3 * sizeof(uint64_t) * kAccRegions * (size_t)T);
  L.stats = o;
  o = up(o + 3 * sizeof(float) * ((size_t)K + 1));
  L.flag = o;
  o = up(o + sizeof(int));
  L.total = o;
  return L;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

const char* hot_last_error(void) { return g_err.c_str(); }

int hot_abi_version(void) { return HOT_ABI_VERSION; }

int hot_check_problem(const hot_slm* slm, int32_t M, const double* xyz, int32_t iters) {
  int rc;
  if ((rc = check_slm(slm))) return rc;
  if ((rc = check_traps(M, xyz, "problem"))) return rc;
  if (iters < 0) return fail(HOT_EINVAL, "iters = %d < 0", iters);
  return HOT_OK;
}

int hot_create(hot_ctx** out, int device, void* stream) {
  if (!out) return fail(HOT_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(HOT_EDEVICE, "no HIP device available (%s)", e == hipSuccess ? "count 0" : hipGetErrorString(e));
  }
  if (device < 0 || device >= n) return fail(HOT_EINVAL, "device %d outside 0..%d", device, n - 1);
  hot_ctx* c = new (std::nothrow) hot_ctx();
  if (!c) return fail(HOT_ENOMEM, "context allocation failed");
  c->device = device;
  auto bail = [&](int code) {
    hot_destroy(c);
    return code;
  };
  if (hipSetDevice(device) != hipSuccess) return bail(fail(HOT_EDEVICE, "hipSetDevice(%d) failed", device));
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
      c->num_cu = ncu;
  }
  if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(HOT_EDEVICE, "stream creation failed"));
  c->stream = (hipStream_t)stream;
  for (auto& s : c->ring)
    if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess)
      return bail(fail(HOT_EDEVICE, "event creation failed"));
  if (hipHostMalloc((void**)&c->flag_host, sizeof(int), hipHostMallocDefault) != hipSuccess)
    return bail(fail(HOT_ENOMEM, "pinned flag allocation failed"));
  // the allocation-free entry point's workspace: this device's copy of the fixed array (its
  // address looked up once per device, with the device current), a pinned staging buffer of the
  // same size and an event
  if (scratch_address(device, &c->scratch) != hipSuccess || !c->scratch)
    return bail(fail(HOT_EDEVICE, "the fixed device workspace has no address on device %d", device));
  if (hipHostMalloc((void**)&c->na_host, kScratchBytes, hipHostMallocDefault) != hipSuccess)
    return bail(fail(HOT_ENOMEM, "pinned staging allocation failed"));
  if (hipHostGetDevicePointer((void**)&c->na_dev, c->na_host, 0) != hipSuccess || !c->na_dev)
    return bail(fail(HOT_EDEVICE, "pinned staging buffer has no device mapping"));
  if (hipEventCreateWithFlags(&c->na_ev, hipEventDisableTiming) != hipSuccess)
    return bail(fail(HOT_EDEVICE, "event creation failed"));
  *c->flag_host = 0;
  int rc = ensure(c, c->flag, sizeof(int));
  if (rc) return bail(rc);
  if (launch_fill_u32(c->stream, (unsigned*)c->flag.p, 0u, 1) != hipSuccess)
    return bail(fail(HOT_EDEVICE, "flag initialisation failed"));
  *out = c;
  return HOT_OK;
}

int hot_destroy(hot_ctx* c) {
  if (!c) return HOT_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  for (DevBuf* b : {&c->coef, &c->st, &c->hd, &c->partial, &c->stats, &c->flag, &c->amat, &c->efield, &c->acc,
                    &c->probe, &c->abl})
    if (b->p) (void)hipFree(b->p);
  for (auto& s : c->ring) {
    if (s.pending && s.ev) (void)hipEventSynchronize(s.ev);
    if (s.host) (void)hipHostFree(s.host);
    if (s.ev) (void)hipEventDestroy(s.ev);
  }
  if (c->flag_host) (void)hipHostFree(c->flag_host);
  if (c->na_ev) {
    if (c->na_pending) (void)hipEventSynchronize(c->na_ev);
    (void)hipEventDestroy(c->na_ev);
  }
  if (c->na_host) (void)hipHostFree(c->na_host);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
  return HOT_OK;
}

int hot_set_stream(hot_ctx* c, void* stream) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  c->stream = (hipStream_t)stream;
  return HOT_OK;
}

int hot_set_variant(hot_ctx* c, int variant) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  if (variant != HOT_ONTHEFLY && variant != HOT_STORED && variant != HOT_SEPARABLE)
    return fail(HOT_EINVAL, "unknown variant %d", variant);
  c->variant = variant;
  return HOT_OK;
}

int hot_set_tuning(hot_ctx* c, int key, int value) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  switch (key) {
    case HOT_TUNE_PIXELS_PER_LANE:
      if (value != 0 && value != 1 && value != 2) return fail(HOT_EINVAL, "pixels per lane must be 0, 1 or 2");
      c->tune_q = value;
      return HOT_OK;
    case HOT_TUNE_TRAPS_PER_LANE:
      if (value != 0 && std::find(std::begin(kTplChoices), std::end(kTplChoices), value) == std::end(kTplChoices))
        return fail(HOT_EINVAL, "traps per lane must be 0, 1..6 or 8");
      c->tune_tpl = value;
      return HOT_OK;
    case HOT_TUNE_SEGMENT:
      if (value != 0 && (value < 64 || value > 1024)) return fail(HOT_EINVAL, "segment must be 0 or 64..1024");
      c->tune_seg = value;
      return HOT_OK;
    case HOT_TUNE_GRAPHS:
      if (value != 0 && value != 1) return fail(HOT_EINVAL, "graphs must be 0 or 1");
      c->use_graphs = value;
      return HOT_OK;
    case HOT_TUNE_SEP_WAVES:
      if (value != 0 && value != 1 && value != 2 && value != 4) return fail(HOT_EINVAL, "separable waves must be 0, 1, 2 or 4");
      c->tune_sepw = value;
      return HOT_OK;
    case HOT_TUNE_SEP_SPLIT:
      if (value != 0 && value != 1 && value != 2) return fail(HOT_EINVAL, "separable waves per tile must be 0, 1 or 2");
      c->tune_sepk = value;
      return HOT_OK;
    case HOT_TUNE_SEP_CHUNK:
      if (value < 0 || value > HOT_MAX_TRAPS || value % 16 != 0)
        return fail(HOT_EINVAL, "separable chunk must be 0 or a multiple of 16 up to %d", HOT_MAX_TRAPS);
      c->tune_sepc = value;
      return HOT_OK;
    case HOT_TUNE_ROWS:
      if (value != 0 && value != 1 && value != 2) return fail(HOT_EINVAL, "rows per block must be 0, 1 or 2");
      c->tune_rows = value;
      return HOT_OK;
    case HOT_TUNE_FRACT:
      if (value != 0 && value != 1) return fail(HOT_EINVAL, "explicit reduction must be 0 (as needed) or 1 (always)");
      c->tune_fract = value;
      return HOT_OK;
    case HOT_TUNE_SLICES:
      if (value < 0 || value > 16) return fail(HOT_EINVAL, "slices must be 0..16");
      c->tune_amax = value;
      return HOT_OK;
    default:
      return fail(HOT_EINVAL, "unknown tuning key %d", key);
  }
}

int hot_sync(hot_ctx* c) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = set_dev(c))) return rc;
  return take_flag(c);
}

static int single(hot_ctx* c, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0, uint64_t seed,
                  int algo, int32_t iters, const float* w0, float* w_out, float* theta_out, float* phase, float* V,
                  hot_stats* stats) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = hot_check_problem(slm, M, xyz, iters))) return rc;
  if (!phase || !V) return fail(HOT_EINVAL, "phase and V output pointers are required");
  return solve(c, slm, 1, &M, xyz, theta0, theta0 == nullptr, seed, algo, iters, w0, w_out, theta_out, phase, V,
               stats, c->variant);
}

int hot_rs(hot_ctx* c, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0, uint64_t seed,
           float* phase, float* V, hot_stats* stats) {
  return single(c, slm, M, xyz, theta0, seed, kRS, 0, nullptr, nullptr, nullptr, phase, V, stats);
}

int hot_gs(hot_ctx* c, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0, uint64_t seed,
           int32_t iters, float* phase, float* V, hot_stats* stats) {
  return single(c, slm, M, xyz, theta0, seed, kGS, iters, nullptr, nullptr, nullptr, phase, V, stats);
}

int hot_gsw(hot_ctx* c, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0, uint64_t seed,
            int32_t iters, const float* w0, float* w_out, float* theta_out, float* phase, float* V,
            hot_stats* stats) {
  return single(c, slm, M, xyz, theta0, seed, kGSW, iters, w0, w_out, theta_out, phase, V, stats);
}

int hot_gsw_noalloc(hot_ctx* c, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0, uint64_t seed,
                    int32_t iters, const float* w0, float* w_out, float* theta_out, float* phase, float* V,
                    hot_stats* stats) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = hot_check_problem(slm, M, xyz, iters))) return rc;
  if (!phase || !V) return fail(HOT_EINVAL, "phase and V output pointers are required");
  const NoallocLayout L = noalloc_layout(M, iters);
  if (L.total > kScratchBytes)
    return fail(HOT_EINVAL, "%d traps and %d iterations need %zu bytes of the fixed workspace, more than its %zu", M,
                iters, L.total, kScratchBytes);
  if (!c->scratch || !c->na_host) return fail(HOT_EDEVICE, "the fixed workspace is not set up");
  if ((rc = set_dev(c))) return rc;
  // the staging buffer is rewritten only once the previous call's upload from it has completed
  if (c->na_pending) {
    HIP_TRY(hipEventSynchronize(c->na_ev));
    c->na_pending = false;
  }
  Plan P;
  if ((rc = prepare_into(c, slm, 1, &M, xyz, theta0, theta0 == nullptr, seed, P, (TrapCoef*)(c->na_host + L.coef),
                         (TrapState*)(c->na_host + L.st), (HoloDesc*)(c->na_host + L.hd))))
    return rc;
  char* base = (char*)c->scratch;
  TrapState* st[2] = {(TrapState*)(base + L.st), (TrapState*)(base + L.st) + M};
  unsigned long long* acc = (unsigned long long*)(base + L.acc);
  auto acc_of = [&](int i) { return acc + (size_t)i * kAccRegions * M; };
  int* flag = (int*)(base + L.flag);
  float* dstats = (float*)(base + L.stats);
  const int K = iters;
  // tables in (coefficients, state, descriptors: one copy from the staging buffer's device
  // mapping), then the launch sequence of hot_gsw, eagerly, with every buffer in the workspace
  HIP_TRY(launch_copy16(c->stream, c->na_dev + L.coef, base + L.coef, (L.acc - L.coef) / 16));
  HIP_TRY(hipEventRecord(c->na_ev, c->stream));
  c->na_pending = true;
  HIP_TRY(launch_fill_u32(c->stream, (unsigned*)acc_of(1), 0u, 2 * kAccRegions * M));
  HIP_TRY(launch_fill_u32(c->stream, (unsigned*)flag, 0u, 1));
  if (w0) HIP_TRY(launch_import_w(c->stream, w0, st[0], M));
  IterArgs a;
  a.fg = P.fg;
  a.B = 1;
  a.nt = P.nt;
  a.q = P.q;
  a.tpl = P.tpl;
  a.rows = P.rows;
  a.mmax = P.mmax;
  a.one = P.one;
  a.fract = P.fract;
  a.coef = (const TrapCoef*)(base + L.coef);
  a.hd = (const HoloDesc*)(base + L.hd);
  a.T = M;
  a.acc_scale = P.acc_scale;
  a.acc_unscale = P.acc_unscale;
  a.stats = dstats;
  a.stat_stride = K + 1;
  a.flag = flag;
  for (int k = 0; k <= K; ++k) {
    a.upd = k == 0 ? 0 : kGSW;
    a.st_in = k == 0 ? st[0] : st[(k - 1) & 1];
    a.st_out = st[k & 1];
    a.acc_in = acc_of(k % 3);
    a.acc_out = acc_of((k + 1) % 3);
    a.acc_zero = acc_of((k + 2) % 3);
    a.kstat = k - 1;
    a.phase = k == K ? phase : nullptr;
    HIP_TRY(launch_iter(c->stream, a));
  }
  HIP_TRY(launch_finish(c->stream, 1, M, acc_of((K + 1) % 3), P.acc_unscale, a.hd, st[K & 1], V, dstats, K, K + 1));
  if (w_out || theta_out) HIP_TRY(launch_export_state(c->stream, st[K & 1], M, w_out, theta_out));
  if (stats) {
    // statistics and flag through the pinned staging buffer (its own regions, not the tables')
    HIP_TRY(hipMemcpyAsync(c->na_host + L.stats, dstats, 3 * sizeof(float) * ((size_t)K + 1), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->na_host + L.flag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->na_pending = false;
    memcpy(stats, c->na_host + L.stats, 3 * sizeof(float) * ((size_t)K + 1));
    if (*(const int*)(c->na_host + L.flag))
      return fail(HOT_EDEGENERATE, "GSW met <|V|> = 0: the phase mask sends no light to any trap");
  }
  return HOT_OK;
}

int hot_gsw_batched(hot_ctx* c, const hot_slm* slm, int32_t B, const int32_t* M, const double* xyz,
                    const double* theta0, int32_t iters, float* phase, float* V, hot_stats* stats) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int64_t T;
  int rc;
  if ((rc = check_batch(slm, B, M, xyz, T))) return rc;
  if (iters < 0) return fail(HOT_EINVAL, "iters = %d < 0", iters);
  if (!theta0) return fail(HOT_EINVAL, "theta0 is required for batched calls");
  if (!phase || !V) return fail(HOT_EINVAL, "phase and V output pointers are required");
  return solve(c, slm, B, M, xyz, theta0, false, 0, kGSW, iters, nullptr, nullptr, nullptr, phase, V, stats,
               c->variant == HOT_SEPARABLE ? HOT_SEPARABLE : HOT_ONTHEFLY);
}

int hot_forward_V(hot_ctx* c, const hot_slm* slm, int32_t B, const int32_t* M, const double* xyz,
                  const float* phase, float* V) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int64_t T;
  int rc;
  if ((rc = check_batch(slm, B, M, xyz, T))) return rc;
  if (!phase || !V) return fail(HOT_EINVAL, "phase and V pointers are required");
  if ((rc = set_dev(c))) return rc;
  Plan P;
  std::vector<double> zeros(T, 0.0);
  if ((rc = prepare(c, slm, B, M, xyz, zeros.data(), false, 0, P))) return rc;
  if ((rc = upload_tables(c, slm, P, xyz, M, false))) return rc;
  if (c->variant == HOT_SEPARABLE) {
    if ((rc = ensure(c, c->partial, sizeof(float2) * (size_t)P.T * P.nblk_sep))) return rc;
    SepArgs a = sep_args(c, P, 1, const_cast<float*>(phase), 0);
    HIP_TRY(launch_sep(c->stream, a));
    HIP_TRY(launch_reduce(c->stream, B, P.mmax, P.nblk_sep, a.inv_n, (const float2*)c->partial.p,
                          (const HoloDesc*)c->hd.p, V));
    return HOT_OK;
  }
  const int nblk = P.fgf.nblk();
  if ((rc = ensure(c, c->partial, sizeof(float2) * (size_t)P.T * nblk))) return rc;
  const HoloDesc* hdf = (const HoloDesc*)c->hd.p + B;
  HIP_TRY(launch_forward(c->stream, P.fgf, B, P.mmax, P.tplf, P.fract, (const TrapCoef*)c->coef.p, hdf, phase,
                         (float2*)c->partial.p));
  HIP_TRY(launch_reduce(c->stream, B, P.mmax, nblk, (float)(1.0 / (double)P.n), (const float2*)c->partial.p, hdf, V));
  return HOT_OK;
}

int hot_adjoint(hot_ctx* c, const hot_slm* slm, int32_t B, const int32_t* M, const double* xyz, const float* phase,
                const float* G, float* grad_phase) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int64_t T;
  int rc;
  if ((rc = check_batch(slm, B, M, xyz, T))) return rc;
  if (!phase || !G || !grad_phase) return fail(HOT_EINVAL, "phase, G and grad_phase pointers are required");
  if ((rc = set_dev(c))) return rc;
  Plan P;
  std::vector<double> zeros(T, 0.0);
  if ((rc = prepare(c, slm, B, M, xyz, zeros.data(), false, 0, P))) return rc;
  if ((rc = upload_tables(c, slm, P, xyz, M, false))) return rc;
  if (c->variant == HOT_SEPARABLE) {
    SepArgs a = sep_args(c, P, 3, const_cast<float*>(phase), 0);
    a.vin = G;
    a.grad = grad_phase;
    HIP_TRY(launch_sep(c->stream, a));
    return HOT_OK;
  }
  HIP_TRY(launch_backward(c->stream, P.nx, P.ny, B, P.fract, 1, (const TrapCoef*)c->coef.p, nullptr,
                          (const HoloDesc*)c->hd.p, const_cast<float*>(phase), 1, G, grad_phase));
  return HOT_OK;
}

int hot_encode_u8(hot_ctx* c, int64_t n, const float* phase, uint8_t* frame) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  if (n < 1 || n > (int64_t)HOT_MAX_SIDE * HOT_MAX_SIDE * HOT_MAX_BATCH)
    return fail(HOT_EINVAL, "pixel count %lld out of range", (long long)n);
  if (!phase || !frame) return fail(HOT_EINVAL, "phase and frame pointers are required");
  int rc;
  if ((rc = set_dev(c))) return rc;
  HIP_TRY(launch_encode_u8(c->stream, phase, frame, n));
  return HOT_OK;
}

int hot_time_passes(hot_ctx* c, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
                    int32_t reps, float* phase, float* V, float* ms) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = hot_check_problem(slm, M, xyz, 0))) return rc;
  if (!theta0 || !phase || !V || !ms) return fail(HOT_EINVAL, "theta0, phase, V and ms are required");
  if (reps < 1) return fail(HOT_EINVAL, "reps = %d < 1", reps);
  if ((rc = set_dev(c))) return rc;
  Plan P;
  if ((rc = prepare(c, slm, 1, &M, xyz, theta0, false, 0, P))) return rc;
  const bool stored = c->variant == HOT_STORED;
  const bool separable = c->variant == HOT_SEPARABLE;
  const int nblk = stored ? P.nblk_stored : separable ? P.nblk_sep : std::max(P.fg.nblk(), P.fgf.nblk());
  if ((rc = upload_tables(c, slm, P, xyz, &M))) return rc;
  if ((rc = ensure(c, c->partial, sizeof(float2) * (size_t)P.T * nblk))) return rc;
  if ((rc = ensure(c, c->stats, sizeof(float) * 3 * 2))) return rc;
  if (stored && (rc = ensure_stored(c, P))) return rc;
  if (!stored && (rc = ensure_acc(c, P))) return rc;
  const TrapCoef* coef = (const TrapCoef*)c->coef.p;
  TrapState* st[2] = {(TrapState*)c->st.p, (TrapState*)c->st.p + P.T};
  const HoloDesc* hd = (const HoloDesc*)c->hd.p;
  float2* part = (float2*)c->partial.p;
  const float inv_n = (float)(1.0 / (double)P.n);
  // group 0: one GSW iteration's main kernel (the fused on-the-fly or separable kernel, or the
  // stored pixel + trap pass).  A fused kernel reads buffer 0 (filled beforehand by a pass over
  // the theta0 mask), adds into buffer 1 (its sums then wrap around over the repetitions:
  // integers, and unused) and clears buffer 2.
  IterArgs a = iter_args(c, P, nullptr, 1);  // as every iteration but a solve's last: no mask stored
  a.upd = 2;
  a.st_in = st[0];
  a.st_out = st[1];
  SepArgs sa = sep_args(c, P, 0, phase, 1);
  sa.upd = 2;
  sa.st_in = st[0];
  sa.st_out = st[1];
  if (!stored) {
    a.acc_in = sa.acc_in = acc_buf(c, P, 0);
    a.acc_out = sa.acc_out = acc_buf(c, P, 1);
    a.acc_zero = sa.acc_zero = acc_buf(c, P, 2);
  }
  auto sep_mode = [&](int mode) {
    SepArgs x = sa;
    x.mode = mode;
    if (mode == 0) x.phase = nullptr;  // as in every iteration but the last
    return launch_sep(c->stream, x);
  };
  auto g0 = [&]() -> hipError_t {
    if (separable) return sep_mode(0);
    if (!stored) return launch_iter(c->stream, a);
    hipError_t e = launch_backward_stored(c->stream, P.n, 1, (const float2*)c->amat.p, st[0], hd, phase,
                                          (float2*)c->efield.p);
    if (e != hipSuccess) return e;
    return launch_forward_stored(c->stream, P.n, 1, P.mmax, (const float2*)c->amat.p, (const float2*)c->efield.p, hd,
                                 part);
  };
  // group 1: the reduction to V (per iteration on the stored path; once per solve, from the
  // fixed-point sums, on the fused paths)
  auto g1 = [&]() {
    if (!stored) return launch_collect(c->stream, P.T, acc_buf(c, P, 0), P.acc_unscale, V);
    return launch_reduce(c->stream, 1, P.mmax, P.nblk_stored, inv_n, part, hd, V);
  };
  // a fused path's buffer 0: sums of the theta0 mask (a pass without update)
  auto prime = [&]() -> hipError_t {
    if (stored) return hipSuccess;
    hipError_t e = launch_fill_u32(c->stream, (unsigned*)acc_buf(c, P, 0), 0u, 2 * kAccRegions * P.T);
    if (e != hipSuccess) return e;
    if (separable) {
      SepArgs p0 = sa;
      p0.upd = 0;
      p0.phase = nullptr;
      p0.acc_in = acc_buf(c, P, 2);
      p0.acc_out = acc_buf(c, P, 0);
      p0.acc_zero = acc_buf(c, P, 1);
      return launch_sep(c->stream, p0);
    }
    IterArgs p0 = a;
    p0.upd = 0;
    p0.acc_in = acc_buf(c, P, 2);
    p0.acc_out = acc_buf(c, P, 0);
    p0.acc_zero = acc_buf(c, P, 1);
    return launch_iter(c->stream, p0);
  };
  auto g2 = [&]() {
    if (separable) return sep_mode(2);
    return stored ? launch_backward_stored(c->stream, P.n, 1, (const float2*)c->amat.p, st[0], hd, phase,
                                           (float2*)c->efield.p)
                  : launch_backward(c->stream, P.nx, P.ny, 1, P.fract, 1, coef, st[0], hd, phase, 0, nullptr, nullptr);
  };
  auto g3 = [&]() {
    if (separable) return sep_mode(1);
    return stored ? launch_forward_stored(c->stream, P.n, 1, P.mmax, (const float2*)c->amat.p,
                                          (const float2*)c->efield.p, hd, part)
                  : launch_forward(c->stream, P.fgf, 1, P.mmax, P.tplf, P.fract, coef, hd + 1, phase, part);
  };
  hipEvent_t ev[5];
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  int out = HOT_OK;
  do {
    // V (and the direct path's buffer 0) must hold a real trap field before an update reads it
    if (g2() != hipSuccess || g3() != hipSuccess ||
        launch_reduce(c->stream, 1, P.mmax, stored ? P.nblk_stored : separable ? P.nblk_sep : P.fgf.nblk(), inv_n,
                      part, stored || separable ? hd : hd + 1, V) != hipSuccess ||
        prime() != hipSuccess || g0() != hipSuccess || g1() != hipSuccess) {
      out = fail(HOT_EDEVICE, "launch failed");
      break;
    }
    (void)hipEventRecord(ev[0], c->stream);
    for (int i = 0; i < reps && out == HOT_OK; ++i) if (g0() != hipSuccess) out = fail(HOT_EDEVICE, "launch failed");
    (void)hipEventRecord(ev[1], c->stream);
    for (int i = 0; i < reps && out == HOT_OK; ++i) if (g1() != hipSuccess) out = fail(HOT_EDEVICE, "launch failed");
    (void)hipEventRecord(ev[2], c->stream);
    for (int i = 0; i < reps && out == HOT_OK; ++i) if (g2() != hipSuccess) out = fail(HOT_EDEVICE, "launch failed");
    (void)hipEventRecord(ev[3], c->stream);
    for (int i = 0; i < reps && out == HOT_OK; ++i) if (g3() != hipSuccess) out = fail(HOT_EDEVICE, "launch failed");
    (void)hipEventRecord(ev[4], c->stream);
    if (out != HOT_OK) break;
    if (hipEventSynchronize(ev[4]) != hipSuccess) {
      out = fail(HOT_EDEVICE, "event sync failed");
      break;
    }
    for (int k = 0; k < 4; ++k) {
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, ev[k], ev[k + 1]);
      ms[k] = t / (float)reps;
    }
  } while (0);
  for (auto& e : ev) (void)hipEventDestroy(e);
  return out;
}

int hot_pixel_pass_variant(hot_ctx* c, const hot_slm* slm, int32_t M, const double* xyz, const double* theta0,
                           int placement, int mapping, int block, int32_t reps, float* phase, float* ms) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = hot_check_problem(slm, M, xyz, 0))) return rc;
  if (!theta0 || !phase || !ms) return fail(HOT_EINVAL, "theta0, phase and ms are required");
  if (placement < HOT_REC_LDS || placement > HOT_REC_GLOBAL) return fail(HOT_EINVAL, "unknown placement %d", placement);
  if (mapping != HOT_MAP_LINEAR && mapping != HOT_MAP_SQUARE) return fail(HOT_EINVAL, "unknown mapping %d", mapping);
  if (block != 64 && block != 256) return fail(HOT_EINVAL, "block must be 64 or 256 pixels");
  if (reps < 1) return fail(HOT_EINVAL, "reps = %d < 1", reps);
  if ((rc = set_dev(c))) return rc;
  Plan P;
  if ((rc = prepare(c, slm, 1, &M, xyz, theta0, false, 0, P))) return rc;
  if ((rc = upload_tables(c, slm, P, xyz, &M))) return rc;
  const int nb = abl_blocks(mapping, block, slm->nx, slm->ny);
  if ((rc = ensure(c, c->abl, sizeof(float4) * (size_t)nb * M))) return rc;
  float4* records = (float4*)c->abl.p;
  HIP_TRY(launch_abl_records(c->stream, mapping, block, slm->nx, slm->ny, M, (const TrapCoef*)c->coef.p,
                             (const TrapState*)c->st.p, records));
  HIP_TRY(launch_abl_pixel(c->stream, placement, mapping, block, slm->nx, slm->ny, M, records, phase));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int res = HOT_OK;
  if (hipEventRecord(e0, c->stream) != hipSuccess) res = fail(HOT_EDEVICE, "event record failed");
  for (int i = 0; i < reps && res == HOT_OK; ++i)
    if (launch_abl_pixel(c->stream, placement, mapping, block, slm->nx, slm->ny, M, records, phase) != hipSuccess)
      res = fail(HOT_EDEVICE, "launch failed");
  if (res == HOT_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
    res = fail(HOT_EDEVICE, "event timing failed");
  if (res == HOT_OK) {
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, e0, e1);
    ms[0] = t / (float)reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

int hot_probe_issue(hot_ctx* c, int kind, int waves_per_simd, int64_t reps, double* out) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  if (kind < 0 || kind > 6) return fail(HOT_EINVAL, "probe kind %d outside 0..6", kind);
  if (waves_per_simd != 1 && waves_per_simd != 2 && waves_per_simd != 4 && waves_per_simd != 8)
    return fail(HOT_EINVAL, "waves per SIMD must be 1, 2, 4 or 8");
  if (reps < 1 || reps > (1LL << 24)) return fail(HOT_EINVAL, "reps = %lld outside 1..2^24", (long long)reps);
  if (!out) return fail(HOT_EINVAL, "out is NULL");
  int rc;
  if ((rc = set_dev(c))) return rc;
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  // one block of 4 * waves_per_simd waves per compute unit (two of 1024 threads for 8 waves)
  const int threads = std::min(1024, 256 * waves_per_simd);
  const int blocks = cus * (256 * waves_per_simd / threads);
  const int waves = blocks * threads / 64;
  const size_t sink_bytes = sizeof(float) * (size_t)blocks * threads;
  if ((rc = ensure(c, c->probe, sink_bytes + 32 * (size_t)waves))) return rc;
  float* sink = (float*)c->probe.p;
  unsigned long long* stamps = (unsigned long long*)((char*)c->probe.p + sink_bytes);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int res = HOT_OK;
  std::vector<unsigned long long> h(4 * (size_t)waves);
  do {
    // a short launch first (clocks ramp, code is loaded), then the measured one
    if (launch_probe(c->stream, kind, blocks, threads, std::max<int64_t>(1, reps / 16), 1.0f, sink, stamps) !=
            hipSuccess ||
        hipEventRecord(e0, c->stream) != hipSuccess ||
        launch_probe(c->stream, kind, blocks, threads, reps, 1.0f, sink, stamps) != hipSuccess ||
        hipEventRecord(e1, c->stream) != hipSuccess) {
      res = fail(HOT_EDEVICE, "probe launch failed");
      break;
    }
    if (hipMemcpyAsync(h.data(), stamps, 32 * (size_t)waves, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      res = fail(HOT_EDEVICE, "probe read-back failed");
      break;
    }
    float ev_ms = 0.0f;
    (void)hipEventElapsedTime(&ev_ms, e0, e1);
    unsigned long long rmin = ~0ull, rmax = 0;
    double cyc = 0.0, clk = 0.0;
    for (int w = 0; w < waves; ++w) {
      const unsigned long long c0 = h[4 * w], c1 = h[4 * w + 1], r0 = h[4 * w + 2], r1 = h[4 * w + 3];
      rmin = std::min(rmin, r0);
      rmax = std::max(rmax, r1);
      cyc += (double)(c1 - c0);
      clk += r1 > r0 ? (double)(c1 - c0) / ((double)(r1 - r0) * 1e-8) : 0.0;
    }
    const double span = (double)(rmax - rmin) * 1e-8;  // s_memrealtime ticks at 100 MHz
    const double ops = (double)waves * 64.0 * (double)reps * (double)probe_ops_per_rep(kind);
    out[0] = span > 0.0 ? ops / span : 0.0;
    out[1] = clk / waves;
    out[2] = span;
    out[3] = ev_ms * 1e-3;
    out[4] = cyc / waves;
    out[5] = (double)waves;
  } while (0);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

int hot_probe_copy(hot_ctx* c, const void* src, void* dst, int64_t bytes, int reps, double* out) {
  if (!c) return fail(HOT_EINVAL, "ctx is NULL");
  if (!src || !dst || !out) return fail(HOT_EINVAL, "src, dst and out are required");
  if (bytes < 16 || bytes % 16 != 0) return fail(HOT_EINVAL, "bytes must be a positive multiple of 16");
  if (reps < 1 || reps > 1000) return fail(HOT_EINVAL, "reps = %d outside 1..1000", reps);
  int rc;
  if ((rc = set_dev(c))) return rc;
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  const size_t n16 = (size_t)bytes / 16;
  const int blocks = (int)std::max<size_t>(1, std::min<size_t>((n16 + 1023) / 1024, (size_t)cus * 16));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int res = HOT_OK;
  do {
    if (launch_probe_copy(c->stream, src, dst, n16, blocks) != hipSuccess || hipEventRecord(e0, c->stream) != hipSuccess) {
      res = fail(HOT_EDEVICE, "copy launch failed");
      break;
    }
    for (int i = 0; i < reps && res == HOT_OK; ++i)
      if (launch_probe_copy(c->stream, src, dst, n16, blocks) != hipSuccess) res = fail(HOT_EDEVICE, "copy launch failed");
    if (res != HOT_OK || hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      if (res == HOT_OK) res = fail(HOT_EDEVICE, "copy timing failed");
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    out[0] = ms > 0.0f ? 2.0 * (double)bytes * reps / (ms * 1e-3) : 0.0;  // bytes read + written per second
    out[1] = ms / reps;
  } while (0);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

}  // extern "C"
