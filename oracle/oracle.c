/*
 * oracle.c -- plain FP64 CPU oracle of the phase-only hologram solver of
 * S. Bianchi and R. Di Leonardo, "Real-time optical micro-manipulation using
 * optimized holograms generated on the GPU" (arXiv:0907.4027).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load or call this library.  It shares no source,
 * header, table or constant with the HIP implementation, and it is deliberately
 * slow and literal: every quantity is evaluated in double precision with libm,
 * straight from the paper's equations, with no blocking, caching or fusion
 * beyond what the equations state.
 *
 * Conventions (readings of points the paper leaves open):
 *   - pixel j = r*nx + c (row-major), x_j = (c - (nx-1)/2) * pitch,
 *     y_j = (r - (ny-1)/2) * pitch: origin on the optical axis, every pixel counts;
 *   - phases are radians; the phase mask is returned in [0, 2*pi); arg(0) = 0;
 *   - sigma = population std(I) / mean(I);
 *   - GSW order: w = 1, theta = theta0, phi = backward; then K times
 *     {V = forward(phi); stats; update w; theta = arg V; phi = backward};
 *     then a final V = forward(phi) and its stats.  K iterations therefore use
 *     K+1 backward and K+1 forward passes.  GS is the same loop without the
 *     weight update; RS (Eq. 3) is the first backward plus one forward.
 *   - the forward sum runs over fixed 4096-pixel chunks, each summed in pixel
 *     order, chunks combined in order, so the result does not depend on the
 *     number of OpenMP threads.
 *
 * Parity pins (tests/test_oracle_pins.py): single-trap closed form, binary
 * grating Fourier coefficient, FFT special case, backward/forward duality,
 * GS/GSW ascent, mirror and conjugation symmetry, translation covariance,
 * brute force on tiny grids, finite-difference gradient.
 * Parity unpinned: the update's degenerate branches (<|V|> = 0: update skipped,
 * ORC_EDEGENERATE; |V_m| below 1e-12 <|V|>: that floor, theta_m kept), which no
 * FP64 workload reaches.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CHUNK 4096

static const double ORC_PI = 3.14159265358979323846264338327950288;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EDEGENERATE = -4 };

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Coordinates of pixel j (Section 3, below Eq. 2: "coordinates of the j-th pixel"). */
static void pixel_xy(int64_t j, int nx, int ny, double pitch, double* x, double* y) {
  int64_t r = j / nx, c = j % nx;
  *x = ((double)c - 0.5 * (double)(nx - 1)) * pitch;
  *y = ((double)r - 0.5 * (double)(ny - 1)) * pitch;
}

/* Eq. 2: phase acquired on propagation from pixel (x, y) to trap t = (x_m, y_m, z_m):
 * lens term z_m*pi/(lambda f^2) * (x^2 + y^2) plus grating term 2*pi/(lambda f) * (x x_m + y y_m). */
static double delta(double x, double y, const double* t, double lam, double f) {
  return t[2] * ORC_PI / (lam * f * f) * (x * x + y * y) + 2.0 * ORC_PI / (lam * f) * (x * t[0] + y * t[1]);
}

static double wrap_2pi(double a) {
  double p = fmod(a, 2.0 * ORC_PI);
  if (p < 0) p += 2.0 * ORC_PI;
  if (p >= 2.0 * ORC_PI) p = 0.0;
  return p;
}

/* Backward propagation (Eq. 3 with weights w_m as in Section 4):
 * S_j = sum_m w_m exp(i (Delta_j^m + theta_m)),  phi_j = arg S_j in [0, 2 pi).
 * idx == NULL: every pixel, outputs indexed by j; else the npix listed pixels,
 * outputs indexed by list position.  S (2 per output, re/im) may be NULL. */
void orc_backward(int nx, int ny, double pitch, double lam, double f, int M, const double* xyz,
                  const double* w, const double* theta, int64_t npix, const int64_t* idx,
                  double* phi, double* S) {
  int64_t cnt = idx ? npix : (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < cnt; ++k) {
    int64_t j = idx ? idx[k] : k;
    double x, y, re = 0.0, im = 0.0;
    pixel_xy(j, nx, ny, pitch, &x, &y);
    for (int m = 0; m < M; ++m) {
      double a = delta(x, y, xyz + 3 * m, lam, f) + theta[m];
      double wm = w ? w[m] : 1.0;
      re += wm * cos(a);
      im += wm * sin(a);
    }
    if (S) { S[2 * k] = re; S[2 * k + 1] = im; }
    phi[k] = (re == 0.0 && im == 0.0) ? 0.0 : wrap_2pi(atan2(im, re));
  }
}

/* Forward propagation, Eq. 1: V_m = (1/N) sum_j exp(i (phi_j - Delta_j^m)).  V: 2M (re, im). */
int orc_forward(int nx, int ny, double pitch, double lam, double f, int M, const double* xyz,
                const double* phi, double* V) {
  int64_t N = (int64_t)nx * ny;
  int64_t nch = (N + ORC_CHUNK - 1) / ORC_CHUNK;
  double* part = (double*)calloc((size_t)(nch * 2 * (M > 0 ? M : 1)), sizeof(double));
  if (!part) return ORC_ENOMEM;
#pragma omp parallel for schedule(static)
  for (int64_t ch = 0; ch < nch; ++ch) {
    double* acc = part + ch * 2 * M;
    int64_t j1 = (ch + 1) * ORC_CHUNK < N ? (ch + 1) * ORC_CHUNK : N;
    for (int64_t j = ch * ORC_CHUNK; j < j1; ++j) {
      double x, y;
      pixel_xy(j, nx, ny, pitch, &x, &y);
      for (int m = 0; m < M; ++m) {
        double a = phi[j] - delta(x, y, xyz + 3 * m, lam, f);
        acc[2 * m] += cos(a);
        acc[2 * m + 1] += sin(a);
      }
    }
  }
  for (int m = 0; m < M; ++m) {
    double re = 0.0, im = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch) { re += part[ch * 2 * M + 2 * m]; im += part[ch * 2 * M + 2 * m + 1]; }
    V[2 * m] = re / (double)N;
    V[2 * m + 1] = im / (double)N;
  }
  free(part);
  return ORC_OK;
}

/* Efficiency and uniformity (Section 3): I_m = |V_m|^2, e = sum I,
 * u = 1 - (max I - min I)/(max I + min I); sigma = std(I)/mean(I) (population). */
void orc_stats(int M, const double* V, double* out3) {
  double e = 0.0, mx = -1.0, mn = 1e300;
  for (int m = 0; m < M; ++m) {
    double I = V[2 * m] * V[2 * m] + V[2 * m + 1] * V[2 * m + 1];
    e += I;
    if (I > mx) mx = I;
    if (I < mn) mn = I;
  }
  double mean = M > 0 ? e / M : 0.0, var = 0.0;
  for (int m = 0; m < M; ++m) {
    double I = V[2 * m] * V[2 * m] + V[2 * m + 1] * V[2 * m + 1];
    var += (I - mean) * (I - mean);
  }
  var = M > 0 ? var / M : 0.0;
  out3[0] = e;
  out3[1] = (mx + mn) > 0.0 ? 1.0 - (mx - mn) / (mx + mn) : 0.0;
  out3[2] = mean > 0.0 ? sqrt(var) / mean : 0.0;
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): theta_m = 2 pi (z >> 40) 2^-24. */
void orc_theta_seed(int M, uint64_t seed, double* theta) {
  uint64_t s = seed;
  for (int m = 0; m < M; ++m) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    theta[m] = 2.0 * ORC_PI * (double)(z >> 40) * (1.0 / 16777216.0);
  }
}

/* RS (algo 0), GS (algo 1) or GSW (algo 2) following the order in the header.
 * theta0: M radians; w0: M initial weights or NULL (all 1).  Outputs (any may be NULL
 * except phi and V): phi N, V 2M, stats 3*(K+1) (RS: 3), w_out M, theta_out M,
 * w_trace (K+1)*M and V_trace (K+1)*2M hold w^k and V^k = forward(phi^k). */
int orc_solve(int algo, int nx, int ny, double pitch, double lam, double f, int M, const double* xyz,
              const double* theta0, const double* w0, int iters, double* phi, double* V, double* stats,
              double* w_out, double* theta_out, double* w_trace, double* V_trace) {
  if (nx <= 0 || ny <= 0 || M <= 0 || iters < 0 || algo < 0 || algo > 2) return ORC_EINVAL;
  int K = algo == 0 ? 0 : iters;
  double* w = (double*)malloc(sizeof(double) * M);
  double* th = (double*)malloc(sizeof(double) * M);
  if (!w || !th) { free(w); free(th); return ORC_ENOMEM; }
  for (int m = 0; m < M; ++m) { w[m] = w0 ? w0[m] : 1.0; th[m] = theta0[m]; }
  int rc = ORC_OK;
  orc_backward(nx, ny, pitch, lam, f, M, xyz, w, th, 0, NULL, phi, NULL);
  for (int k = 0; k <= K; ++k) {
    rc = orc_forward(nx, ny, pitch, lam, f, M, xyz, phi, V);
    if (rc) break;
    if (stats) orc_stats(M, V, stats + 3 * k);
    if (w_trace) memcpy(w_trace + (size_t)k * M, w, sizeof(double) * M);
    if (V_trace) memcpy(V_trace + (size_t)k * 2 * M, V, sizeof(double) * 2 * M);
    if (k == K) break;
    /* update weights (GSW: w_m <- w_m <|V|>/|V_m|, <> = mean over m) and phases theta_m <- arg V_m */
    double mean = 0.0;
    for (int m = 0; m < M; ++m) mean += hypot(V[2 * m], V[2 * m + 1]);
    mean /= M;
    if (!(mean > 0.0)) { rc = ORC_EDEGENERATE; break; }
    for (int m = 0; m < M; ++m) {
      double a = hypot(V[2 * m], V[2 * m + 1]);
      int tiny = a < 1e-12 * mean;
      if (algo == 2) w[m] *= mean / (tiny ? 1e-12 * mean : a);
      if (!tiny) th[m] = atan2(V[2 * m + 1], V[2 * m]);
    }
    orc_backward(nx, ny, pitch, lam, f, M, xyz, w, th, 0, NULL, phi, NULL);
  }
  if (w_out) memcpy(w_out, w, sizeof(double) * M);
  if (theta_out) memcpy(theta_out, th, sizeof(double) * M);
  free(w);
  free(th);
  return rc;
}

/* Adjoint of Eq. 1: for a real loss L(V) with G_m = dL/dRe V_m + i dL/dIm V_m,
 * dL/dphi_j = sum_m Re(conj(G_m) dV_m/dphi_j) = (1/N) Im(exp(-i phi_j) sum_m G_m exp(i Delta_j^m)).
 * G: 2M (re, im); grad: N. */
void orc_adjoint(int nx, int ny, double pitch, double lam, double f, int M, const double* xyz,
                 const double* phi, const double* G, double* grad) {
  int64_t N = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) {
    double x, y, re = 0.0, im = 0.0;
    pixel_xy(j, nx, ny, pitch, &x, &y);
    for (int m = 0; m < M; ++m) {
      double a = delta(x, y, xyz + 3 * m, lam, f);
      double c = cos(a), s = sin(a);
      re += G[2 * m] * c - G[2 * m + 1] * s;
      im += G[2 * m] * s + G[2 * m + 1] * c;
    }
    /* Im(exp(-i phi) (re + i im)) = im cos(phi) - re sin(phi) */
    grad[j] = (im * cos(phi[j]) - re * sin(phi[j])) / (double)N;
  }
}

/* Trap-intensity loss L = -sum_m log I_m + 10 var(I)/mean(I)^2 (population var), I_m = |V_m|^2.
 * Writes dL/dI_m into g (M). */
static double loss_and_dI(int M, const double* V, double* g) {
  double mu = 0.0, var = 0.0, L = 0.0;
  for (int m = 0; m < M; ++m) mu += V[2 * m] * V[2 * m] + V[2 * m + 1] * V[2 * m + 1];
  mu /= M;
  for (int m = 0; m < M; ++m) {
    double I = V[2 * m] * V[2 * m] + V[2 * m + 1] * V[2 * m + 1];
    var += (I - mu) * (I - mu);
    L -= log(I);
  }
  var /= M;
  L += 10.0 * var / (mu * mu);
  if (g)
    for (int m = 0; m < M; ++m) {
      double I = V[2 * m] * V[2 * m] + V[2 * m + 1] * V[2 * m + 1];
      g[m] = -1.0 / I + 10.0 * (2.0 * (I - mu) / (M * mu * mu) - 2.0 * var / (M * mu * mu * mu));
    }
  return L;
}

/* Loss of the phase mask phi and (if grad != NULL) its analytic gradient dL/dphi (N),
 * through G_m = 2 (dL/dI_m) V_m and the adjoint above.  V_out (2M) may be NULL. */
double orc_loss_grad(int nx, int ny, double pitch, double lam, double f, int M, const double* xyz,
                     const double* phi, double* V_out, double* grad) {
  double* V = (double*)malloc(sizeof(double) * 2 * M);
  double* g = (double*)malloc(sizeof(double) * M);
  double* G = (double*)malloc(sizeof(double) * 2 * M);
  double L = NAN;
  if (V && g && G && orc_forward(nx, ny, pitch, lam, f, M, xyz, phi, V) == ORC_OK) {
    L = loss_and_dI(M, V, g);
    if (grad) {
      for (int m = 0; m < M; ++m) { G[2 * m] = 2.0 * g[m] * V[2 * m]; G[2 * m + 1] = 2.0 * g[m] * V[2 * m + 1]; }
      orc_adjoint(nx, ny, pitch, lam, f, M, xyz, phi, G, grad);
    }
    if (V_out) memcpy(V_out, V, sizeof(double) * 2 * M);
  }
  free(V);
  free(g);
  free(G);
  return L;
}
