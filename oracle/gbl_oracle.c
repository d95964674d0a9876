/*
 * gbl_oracle.c -- plain, slow, FP64 CPU oracle for the Galactic-Binary (GB)
 * template + likelihood hot path of the LISA global fit (arXiv:2405.04690).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * library (HIP) shares no code, header, table or constant generator with it.
 *
 * What it computes, and where each piece comes from:
 *   - Whittle log-likelihood and noise-weighted inner product: Sec. 2,
 *     eq. (like) and eq. (inner).
 *   - Likelihood change for adding / swapping one source: Sec. 2,
 *     eq. (addsource) and eq. (swapsource).
 *   - XYZ -> AET combination: Sec. 2 (first-generation-1.5 TDI, equal arms).
 *   - Instrument PSD: Sec. 3, eq. (psd) with the acceleration and OMS terms.
 *   - The GB waveform: the paper only says "based on FastGB" (Sec. 2.A and
 *     appendix "GB Waveform Generation").  The waveform below is this
 *     project's own reading, stated in full: Estabrook-Wahlquist single-link
 *     response, rigid equal-arm circular orbit, first-generation Michelson TDI,
 *     and a heterodyned slow/fast split with the slow envelope sampled at N
 *     midpoints and Fourier transformed.  Every absolute waveform value is
 *     therefore pinned only by the brute-force time-domain synthesis, the
 *     closed-form limits and the invariants in the tests.
 *
 * Everything is double precision and written for clarity, not speed: the
 * only "algorithm" beyond the definitions is a textbook recursive radix-2
 * FFT (pinned against the direct DFT sum in the tests).
 *
 * Conventions (readings where the paper is silent):
 *   params[8] = (A, f0 [Hz], fdot [Hz/s], phi0, iota, psi, lambda, beta),
 *     physical units, ecliptic longitude lambda and latitude beta.
 *   Frequency bins f_k = k/T, Delta f = 1/T.  Fourier convention
 *     x~(f_k) = dt * sum_n x(n dt) exp(-2 pi i k n / M).
 *   Analysis band k in [ceil(f_lo T), floor(f_hi T)]; bins outside count 0.
 *   Residual layout [n_res][2 channels A,E][n_bins] complex (re, im).
 *   PSD layout      [n_psd][2][n_bins] real.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C 299792458.0           /* speed of light [m/s] */
#define ORC_AU 1.495978707e11       /* astronomical unit [m] */
#define ORC_YEAR 31557600.0         /* Julian year [s]; orbit period */
#define ORC_PI 3.14159265358979323846

typedef double complex cplx;

/* Run configuration: observation time, cadence, arm length, analysis band. */
typedef struct {
  double T;
  double dt;
  double L;
  double f_lo;
  double f_hi;
} gblo_config;

/* ------------------------------------------------------------------------ */
/* Threads                                                                  */
/* ------------------------------------------------------------------------ */

int gblo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Band bookkeeping (Sec. 2: sums over positive frequencies, read as the   */
/* analysis band [f_lo, f_hi])                                              */
/* ------------------------------------------------------------------------ */

int gblo_band(const gblo_config* cfg, int64_t* k_min, int64_t* n_bins) {
  int64_t lo = (int64_t)ceil(cfg->f_lo * cfg->T);
  int64_t hi = (int64_t)floor(cfg->f_hi * cfg->T);
  *k_min = lo;
  *n_bins = hi - lo + 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Orbit: rigid equal-arm triangle on a 1 AU circular heliocentric orbit,   */
/* first order in the eccentricity e = L / (2 sqrt(3) AU).  Spacecraft      */
/* index i = 0, 1, 2 (labels 1, 2, 3), orientation offset 2 pi i / 3.       */
/* ------------------------------------------------------------------------ */

void gblo_orbit_position(const gblo_config* cfg, int i, double t, double x[3]) {
  double e = cfg->L / (2.0 * sqrt(3.0) * ORC_AU);
  double a = 2.0 * ORC_PI * t / ORC_YEAR;
  double b = 2.0 * ORC_PI * (double)i / 3.0;
  x[0] = ORC_AU * cos(a) + 0.5 * e * ORC_AU * (cos(2.0 * a - b) - 3.0 * cos(b));
  x[1] = ORC_AU * sin(a) + 0.5 * e * ORC_AU * (sin(2.0 * a - b) - 3.0 * sin(b));
  x[2] = -sqrt(3.0) * e * ORC_AU * cos(a - b);
}

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ------------------------------------------------------------------------ */
/* Source frame: propagation direction k = -Omega and the complex           */
/* polarisation tensor  H = A [ (1 + cos^2 iota) eps_+ + 2 i cos iota eps_x ]*/
/* so that h_ij(xi) = Re[ H_ij exp(i Phi(xi)) ] with                        */
/* Phi(xi) = phi0 + 2 pi f0 xi + pi fdot xi^2.                              */
/* H is returned as [3][3][2] (re, im).                                     */
/* ------------------------------------------------------------------------ */

static void source_frame(const double* p, double khat[3], cplx H[3][3]) {
  double A = p[0], iota = p[4], psi = p[5], lam = p[6], beta = p[7];
  double Om[3] = {cos(beta) * cos(lam), cos(beta) * sin(lam), sin(beta)};
  double P[3] = {sin(lam), -cos(lam), 0.0};
  double Q[3] = {-sin(beta) * cos(lam), -sin(beta) * sin(lam), cos(beta)};
  double ci = cos(iota);
  for (int i = 0; i < 3; i++) khat[i] = -Om[i];
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) {
      double ep = P[i] * P[j] - Q[i] * Q[j];
      double ex = P[i] * Q[j] + Q[i] * P[j];
      double eps_p = cos(2.0 * psi) * ep + sin(2.0 * psi) * ex;
      double eps_x = -sin(2.0 * psi) * ep + cos(2.0 * psi) * ex;
      H[i][j] = A * ((1.0 + ci * ci) * eps_p + 2.0 * I * ci * eps_x);
    }
  }
}

void gblo_source_frame(const double* p, double khat[3], double* H_out /*[3][3][2]*/) {
  cplx H[3][3];
  source_frame(p, khat, H);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      H_out[2 * (3 * i + j)] = creal(H[i][j]);
      H_out[2 * (3 * i + j) + 1] = cimag(H[i][j]);
    }
}

/* n^T H n for a unit vector n */
static cplx contract(cplx H[3][3], const double n[3]) {
  cplx g = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) g += n[i] * H[i][j] * n[j];
  return g;
}

/* ------------------------------------------------------------------------ */
/* Exact single-link response (Estabrook-Wahlquist), fractional frequency,  */
/* for the photon sent from spacecraft s and received at r at time t:       */
/*   y_{s->r}(t) = [G(xi_s) - G(xi_r)] / (2 (1 - k.n)),                      */
/*   G(xi) = n^T h(xi) n,  n = (x_r - x_s)/L frozen at reception time t,     */
/*   xi_r = t - k.x_r/c,  xi_s = t - L/c - k.x_s/c.                          */
/* The carrier phase is formed in long double: it is used by the pins, where */
/* 2 pi f0 t reaches 1e6 rad.                                               */
/* ------------------------------------------------------------------------ */

static double g_of_xi(cplx g, const double* p, long double xi) {
  long double ph = (long double)p[3] + 2.0L * 3.14159265358979323846264338327950288L * (long double)p[1] * xi +
                   3.14159265358979323846264338327950288L * (long double)p[2] * xi * xi;
  return (double)((long double)creal(g) * cosl(ph) - (long double)cimag(g) * sinl(ph));
}

double gblo_link_response(const gblo_config* cfg, const double* p, int s, int r, double t) {
  double khat[3];
  cplx H[3][3];
  source_frame(p, khat, H);
  double xs[3], xr[3], n[3];
  gblo_orbit_position(cfg, s, t, xs);
  gblo_orbit_position(cfg, r, t, xr);
  for (int i = 0; i < 3; i++) n[i] = (xr[i] - xs[i]) / cfg->L;
  cplx g = contract(H, n);
  long double xi_r = (long double)t - (long double)dot3(khat, xr) / ORC_C;
  long double xi_s = (long double)t - (long double)(cfg->L / ORC_C) - (long double)dot3(khat, xs) / ORC_C;
  return (g_of_xi(g, p, xi_s) - g_of_xi(g, p, xi_r)) / (2.0 * (1.0 - dot3(khat, n)));
}

/* ------------------------------------------------------------------------ */
/* Heterodyned slow envelope of one link (the fast/slow split):             */
/*   y_{s->r}(t) = Re[ exp(2 pi i q t / T) s_{s->r}(t) ]   exactly, with     */
/*   s = -i G [(theta/2)/(1-k.n)] sinc(theta/2) exp(-i theta/2) exp(i phi_r) */
/*   delta = (L/c)(1 - k.n),  f_r = f0 + fdot xi_r,                           */
/*   theta = 2 pi f_r delta - pi fdot delta^2,                               */
/*   phi_r = Phi(xi_r) - 2 pi q t / T, written without ever forming          */
/*           2 pi f0 t.                                                     */
/* ------------------------------------------------------------------------ */

static cplx link_envelope(const gblo_config* cfg, const double* p, const double khat[3], cplx H[3][3], int64_t q, int s,
                          int r, double t) {
  double f0 = p[1], fdot = p[2], phi0 = p[3];
  double Lc = cfg->L / ORC_C;
  double xs[3], xr[3], n[3];
  gblo_orbit_position(cfg, s, t, xs);
  gblo_orbit_position(cfg, r, t, xr);
  for (int i = 0; i < 3; i++) n[i] = (xr[i] - xs[i]) / cfg->L;
  double kn = dot3(khat, n);
  double kxr = dot3(khat, xr) / ORC_C;
  double delta = Lc * (1.0 - kn);
  double fr = f0 + fdot * (t - kxr);
  double theta = 2.0 * ORC_PI * fr * delta - ORC_PI * fdot * delta * delta;
  double amp = ORC_PI * fr * Lc - 0.5 * ORC_PI * fdot * Lc * Lc * (1.0 - kn);
  double dfq = f0 - (double)q / cfg->T;
  double phir = phi0 + 2.0 * ORC_PI * dfq * t + ORC_PI * fdot * t * t - 2.0 * ORC_PI * (f0 + fdot * t) * kxr +
                ORC_PI * fdot * kxr * kxr;
  double u = 0.5 * theta;
  double sinc = (fabs(u) < 1e-6) ? 1.0 - u * u / 6.0 : sin(u) / u;
  cplx g = contract(H, n);
  return -I * g * amp * sinc * cexp(-I * u) * cexp(I * phir);
}

void gblo_link_envelope(const gblo_config* cfg, const double* p, int64_t q, int s, int r, double t, double out[2]) {
  double khat[3];
  cplx H[3][3];
  source_frame(p, khat, H);
  cplx v = link_envelope(cfg, p, khat, H, q, s, r, t);
  out[0] = creal(v);
  out[1] = cimag(v);
}

/* ------------------------------------------------------------------------ */
/* FFT: textbook recursive radix-2 decimation in time, forward sign,        */
/* X[k] = sum_n x[n] exp(-2 pi i k n / n_len).  n_len a power of two.       */
/* ------------------------------------------------------------------------ */

static void fft_rec(cplx* x, int n_len, cplx* scratch) {
  if (n_len == 1) return;
  int h = n_len / 2;
  cplx* ev = scratch;
  cplx* od = scratch + h;
  for (int i = 0; i < h; i++) {
    ev[i] = x[2 * i];
    od[i] = x[2 * i + 1];
  }
  fft_rec(ev, h, x);
  fft_rec(od, h, x);
  for (int k = 0; k < h; k++) {
    cplx w = cexp(-2.0 * I * ORC_PI * (double)k / (double)n_len) * od[k];
    x[k] = ev[k] + w;
    x[k + h] = ev[k] - w;
  }
}

int gblo_fft(int n_len, double* data /*[n_len][2], in place*/) {
  if (n_len < 1 || (n_len & (n_len - 1))) return -2;
  cplx* x = (cplx*)malloc(sizeof(cplx) * n_len);
  cplx* s = (cplx*)malloc(sizeof(cplx) * n_len);
  for (int i = 0; i < n_len; i++) x[i] = data[2 * i] + I * data[2 * i + 1];
  fft_rec(x, n_len, s);
  for (int i = 0; i < n_len; i++) {
    data[2 * i] = creal(x[i]);
    data[2 * i + 1] = cimag(x[i]);
  }
  free(x);
  free(s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Fast heterodyned waveform, one template, in the order of the method:     */
/*  1. carrier bin q = floor(f0 T), window start k0 = q - N/2;              */
/*  2. slow samples at the midpoints t_n = (n + 1/2) T / N;                 */
/*  3. the six link envelopes s_{s->r}(t_n);                                */
/*  4. TDI pieces: X = (1 - D^2)(R_12 - R_13), R_ab = y_{b->a} + D y_{a->b}, */
/*     so X = (1 - D^2)(U_X + D V_X) with U_X = s_{2->1} - s_{3->1},         */
/*     V_X = s_{1->2} - s_{1->3}; Y, Z by cyclic relabelling; then A, E, T;  */
/*  5. U~[k] = (1/2)(T/N) exp(-i pi k/N) DFT_N[U](k), k = -N/2..N/2-1;       */
/*  6. per bin, with x = 2 pi (q+k) L/(c T) and D -> exp(-i x):             */
/*     C[j] = (1 - exp(-2 i x)) (U~[k] + exp(-i x) V~[k]),  j = k + N/2;      */
/*  7. output bin j is global bin k0 + j.                                   */
/* out_A/out_E/out_T are [N][2]; out_T may be NULL.                         */
/* ------------------------------------------------------------------------ */

/* Boundary reading: any non-finite parameter, or |f0 T| >= 2^52, makes the
 * template undefined; its slices are NaN and its start bin 0. */
static int params_finite(const gblo_config* cfg, const double* p) {
  for (int i = 0; i < 8; i++)
    if (!isfinite(p[i])) return 0;
  return fabs(p[1] * cfg->T) < 4503599627370496.0; /* 2^52: the carrier bin is an exact integer */
}

static void waveform_one(const gblo_config* cfg, const double* p, int N, cplx* oA, cplx* oE, cplx* oT,
                         int64_t* start) {
  if (!params_finite(cfg, p)) {
    for (int j = 0; j < N; j++) {
      oA[j] = oE[j] = NAN + I * NAN;
      if (oT) oT[j] = NAN + I * NAN;
    }
    *start = 0;
    return;
  }
  double khat[3];
  cplx H[3][3];
  source_frame(p, khat, H);
  int64_t q = (int64_t)floor(p[1] * cfg->T);
  *start = q - N / 2;

  /* series: 0 U_A, 1 V_A, 2 U_E, 3 V_E, 4 U_T, 5 V_T */
  cplx* ser = (cplx*)malloc(sizeof(cplx) * 6 * N);
  cplx* scr = (cplx*)malloc(sizeof(cplx) * N);
  const double r2 = sqrt(2.0), r6 = sqrt(6.0), r3 = sqrt(3.0);
  for (int n = 0; n < N; n++) {
    double t = ((double)n + 0.5) * cfg->T / (double)N;
    /* s[s][r]: link from spacecraft s to r (0-based) */
    cplx l[3][3];
    for (int s = 0; s < 3; s++)
      for (int r = 0; r < 3; r++) l[s][r] = (s == r) ? 0.0 : link_envelope(cfg, p, khat, H, q, s, r, t);
    cplx UX = l[1][0] - l[2][0], VX = l[0][1] - l[0][2];
    cplx UY = l[2][1] - l[0][1], VY = l[1][2] - l[1][0];
    cplx UZ = l[0][2] - l[1][2], VZ = l[2][0] - l[2][1];
    ser[0 * N + n] = (UZ - UX) / r2;
    ser[1 * N + n] = (VZ - VX) / r2;
    ser[2 * N + n] = (UX - 2.0 * UY + UZ) / r6;
    ser[3 * N + n] = (VX - 2.0 * VY + VZ) / r6;
    ser[4 * N + n] = (UX + UY + UZ) / r3;
    ser[5 * N + n] = (VX + VY + VZ) / r3;
  }
  int n_ser = oT ? 6 : 4;
  for (int s = 0; s < n_ser; s++) fft_rec(ser + s * N, N, scr);

  cplx* outs[3] = {oA, oE, oT};
  for (int j = 0; j < N; j++) {
    int k = j - N / 2;
    int idx = (k % N + N) % N;
    cplx F = 0.5 * (cfg->T / (double)N) * cexp(-I * ORC_PI * (double)k / (double)N);
    double x = 2.0 * ORC_PI * (double)(q + k) * cfg->L / (ORC_C * cfg->T);
    cplx D = cexp(-I * x);
    for (int c = 0; c < n_ser / 2; c++) {
      cplx Ut = F * ser[(2 * c) * N + idx];
      cplx Vt = F * ser[(2 * c + 1) * N + idx];
      outs[c][j] = (1.0 - D * D) * (Ut + D * Vt);
    }
  }
  free(ser);
  free(scr);
}

int gblo_waveform(const gblo_config* cfg, const double* params, int64_t B, int N, double* A, double* E, double* Tch,
                  int64_t* start_bin) {
  if (N < 2 || (N & (N - 1))) return -2;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < B; b++) {
    waveform_one(cfg, params + 8 * b, N, (cplx*)(A + 2 * N * b), (cplx*)(E + 2 * N * b),
                 Tch ? (cplx*)(Tch + 2 * N * b) : NULL, start_bin + b);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Instrument PSD in A and E, eq. (psd):                                    */
/*   S_n = 8 sin^2 x [ 2 S_pm (3 + 2 cos x + cos 2x) + S_op (2 + cos x) ],  */
/*   x = 2 pi f L / c,                                                      */
/*   S_pm = S_acc (2 pi c f)^-2 [1 + (0.4 mHz/f)^2][1 + (f/8 mHz)^4],         */
/*   S_op = S_oms (2 pi f / c)^2 [1 + (2 mHz/f)^4].                          */
/* noise[4] = (sqrt S_oms^A, sqrt S_acc^A, sqrt S_oms^E, sqrt S_acc^E).      */
/* ------------------------------------------------------------------------ */

double gblo_psd_value(const gblo_config* cfg, double f, double sqrt_oms, double sqrt_acc) {
  double x = 2.0 * ORC_PI * f * cfg->L / ORC_C;
  double S_acc = sqrt_acc * sqrt_acc;
  double S_oms = sqrt_oms * sqrt_oms;
  double S_pm = S_acc * pow(2.0 * ORC_PI * ORC_C * f, -2.0) * (1.0 + pow(0.4e-3 / f, 2.0)) * (1.0 + pow(f / 8e-3, 4.0));
  double S_op = S_oms * pow(2.0 * ORC_PI * f / ORC_C, 2.0) * (1.0 + pow(2e-3 / f, 4.0));
  return 8.0 * sin(x) * sin(x) * (2.0 * S_pm * (3.0 + 2.0 * cos(x) + cos(2.0 * x)) + S_op * (2.0 + cos(x)));
}

int gblo_psd_eval(const gblo_config* cfg, const double* noise, int64_t P, double* S /*[P][2][n_bins]*/) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
#pragma omp parallel for
  for (int64_t pi = 0; pi < P; pi++)
    for (int c = 0; c < 2; c++)
      for (int64_t i = 0; i < nb; i++) {
        double f = (double)(k_min + i) / cfg->T;
        S[(pi * 2 + c) * nb + i] = gblo_psd_value(cfg, f, noise[4 * pi + 2 * c], noise[4 * pi + 2 * c + 1]);
      }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Galactic foreground (Sec. 3, "Galactic foreground noise                  */
/* parameterization"): the confusion-noise strain sensitivity               */
/*   h_fg(f) = 1/2 A_fg f^(-7/3) exp(-s1 f^alpha) [1 + tanh(-s2 (f - f_k))]  */
/* enters the A and E PSD as S_fg = 6 x^2 sin^2 x h_fg(f), x = 2 pi f L / c, */
/* added to S_n of both channels (one foreground shared by A and E).        */
/* fg[5] = (A_fg, alpha, f_k [Hz], s1, s2).                                 */
/* Noise sets with the foreground are noise[9] = the four instrument        */
/* parameters followed by fg[5].                                            */
/* ------------------------------------------------------------------------ */

double gblo_foreground_value(const gblo_config* cfg, double f, const double* fg) {
  double x = 2.0 * ORC_PI * f * cfg->L / ORC_C;
  double h = 0.5 * fg[0] * pow(f, -7.0 / 3.0) * exp(-fg[3] * pow(f, fg[1])) * (1.0 + tanh(-fg[4] * (f - fg[2])));
  return 6.0 * x * x * sin(x) * sin(x) * h;
}

/* S[P][2][n_bins] for noise sets of n_par = 4 (instrument only) or 9
 * (instrument + foreground) parameters */
int gblo_psd_eval_n(const gblo_config* cfg, const double* noise, int32_t n_par, int64_t P, double* S) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  if (n_par != 4 && n_par != 9) return -1;
#pragma omp parallel for
  for (int64_t pi = 0; pi < P; pi++)
    for (int c = 0; c < 2; c++)
      for (int64_t i = 0; i < nb; i++) {
        double f = (double)(k_min + i) / cfg->T;
        const double* th = noise + n_par * pi;
        double v = gblo_psd_value(cfg, f, th[2 * c], th[2 * c + 1]);
        if (n_par == 9) v += gblo_foreground_value(cfg, f, th + 4);
        S[(pi * 2 + c) * nb + i] = v;
      }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Log-likelihoods.                                                         */
/* Base (eq. like):  lnL = -1/2 <R|R> - sum_ch sum_k ln S_ch,k,              */
/* <b|c> = 4 Delta f Re sum_ch sum_k conj(b) c / S  (eq. inner, A and E).     */
/* ------------------------------------------------------------------------ */

double gblo_loglike(const gblo_config* cfg, const double* R /*[2][n_bins][2]*/, const double* S /*[2][n_bins]*/) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  double df = 1.0 / cfg->T;
  double rr = 0.0, lg = 0.0;
  for (int c = 0; c < 2; c++)
    for (int64_t i = 0; i < nb; i++) {
      double re = R[2 * (c * nb + i)], im = R[2 * (c * nb + i) + 1];
      rr += (re * re + im * im) / S[c * nb + i];
      lg += log(S[c * nb + i]);
    }
  return -0.5 * 4.0 * df * rr - lg;
}

/* PSD-parameter log-likelihood: the base likelihood with S built from the
 * n_par (4, or 9 with the foreground) noise parameters of each set;
 * noise [P][n_par], res_idx [P]. */
int gblo_psd_loglike_n(const gblo_config* cfg, const double* residual, int32_t n_res, const double* noise,
                       int32_t n_par, const int32_t* res_idx, int64_t P, double* logl) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  if (n_par != 4 && n_par != 9) return -1;
  for (int64_t pi = 0; pi < P; pi++)
    if (res_idx[pi] < 0 || res_idx[pi] >= n_res) return -1;
#pragma omp parallel for
  for (int64_t pi = 0; pi < P; pi++) {
    double* S = (double*)malloc(sizeof(double) * 2 * nb);
    gblo_psd_eval_n(cfg, noise + n_par * pi, n_par, 1, S);
    logl[pi] = gblo_loglike(cfg, residual + (int64_t)res_idx[pi] * 2 * nb * 2, S);
    free(S);
  }
  return 0;
}

int gblo_psd_loglike(const gblo_config* cfg, const double* residual, int32_t n_res, const double* noise,
                     const int32_t* res_idx, int64_t P, double* logl) {
  return gblo_psd_loglike_n(cfg, residual, n_res, noise, 4, res_idx, P, logl);
}

/* ------------------------------------------------------------------------ */
/* Likelihood change for swapping source r (old) for a (new), eq. (swapsource),
 * on channels A and E, restricted to the template windows clipped to the    */
/* analysis band.  With R = d - H (H contains r):                            */
/*   dlnL = -1/2 [ <a|a> + <r|r> - 2<a|r> - 2<R|a> + 2<R|r> ]   (literal)    */
/*        = <R|a - r> - 1/2 <a - r|a - r>             (cancellation free)    */
/* Birth: r has zero amplitude (eq. addsource); death: a has zero amplitude. */
/* terms (optional) [B][6] = (<a|a>, <r|r>, <a|r>, <R|a>, <R|r>, literal).   */
/* psd_is_inverse != 0: psd holds 1/S instead of S.                          */
/* ------------------------------------------------------------------------ */

int gblo_delta_loglike(const gblo_config* cfg, const double* residual, int32_t n_res, const double* psd, int32_t n_psd,
                       int32_t psd_is_inverse, const double* params_old, const double* params_new, int32_t N,
                       const int32_t* res_idx, const int32_t* psd_idx, int64_t B, double* dlogl, double* terms) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  if (N < 2 || (N & (N - 1))) return -2;
  for (int64_t b = 0; b < B; b++) {
    if (res_idx[b] < 0 || res_idx[b] >= n_res) return -1;
    if (psd_idx[b] < 0 || psd_idx[b] >= n_psd) return -1;
  }
  double df = 1.0 / cfg->T;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < B; b++) {
    if (!params_finite(cfg, params_new + 8 * b) || !params_finite(cfg, params_old + 8 * b)) {
      dlogl[b] = NAN;
      if (terms)
        for (int i = 0; i < 6; i++) terms[6 * b + i] = NAN;
      continue;
    }
    cplx* a = (cplx*)malloc(sizeof(cplx) * 2 * N);
    cplx* r = (cplx*)malloc(sizeof(cplx) * 2 * N);
    int64_t ka, kr;
    waveform_one(cfg, params_new + 8 * b, N, a, a + N, NULL, &ka);
    waveform_one(cfg, params_old + 8 * b, N, r, r + N, NULL, &kr);
    const cplx* R = (const cplx*)(residual + (int64_t)res_idx[b] * 2 * nb * 2);
    const double* S = psd + (int64_t)psd_idx[b] * 2 * nb;
    double aa = 0, rr = 0, ar = 0, Ra = 0, Rr = 0, Rd = 0, dd = 0;
    /* union of the two windows: every bin of a's window, then the bins of
       r's window that are not in a's window */
    for (int pass = 0; pass < 2; pass++) {
      int64_t k0 = pass == 0 ? ka : kr;
      for (int j = 0; j < N; j++) {
        int64_t k = k0 + j;
        if (pass == 1 && k >= ka && k < ka + N) continue;
        if (k < k_min || k >= k_min + nb) continue;
        for (int c = 0; c < 2; c++) {
          cplx av = (k >= ka && k < ka + N) ? a[c * N + (k - ka)] : 0.0;
          cplx rv = (k >= kr && k < kr + N) ? r[c * N + (k - kr)] : 0.0;
          cplx Rv = R[c * nb + (k - k_min)];
          double w = psd_is_inverse ? S[c * nb + (k - k_min)] : 1.0 / S[c * nb + (k - k_min)];
          cplx d = av - rv;
          aa += creal(conj(av) * av) * w;
          rr += creal(conj(rv) * rv) * w;
          ar += creal(conj(av) * rv) * w;
          Ra += creal(conj(Rv) * av) * w;
          Rr += creal(conj(Rv) * rv) * w;
          Rd += creal(conj(Rv) * d) * w;
          dd += creal(conj(d) * d) * w;
        }
      }
    }
    double f4 = 4.0 * df;
    dlogl[b] = f4 * Rd - 0.5 * f4 * dd;
    if (terms) {
      double* t = terms + 6 * b;
      t[0] = f4 * aa;
      t[1] = f4 * rr;
      t[2] = f4 * ar;
      t[3] = f4 * Ra;
      t[4] = f4 * Rr;
      t[5] = -0.5 * (t[0] + t[1] - 2.0 * t[2] - 2.0 * t[3] + 2.0 * t[4]);
    }
    free(a);
    free(r);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Inner products of stored band slices (eq. inner, channels A and E): for   */
/* template b with slices A[b], E[b] of width N starting at global bin       */
/* start_bin[b],                                                            */
/*   out[b][0] = <h|h>,  out[b][1] = <R|h>,  R = residual[res_idx[b]],       */
/* over the slice's bins inside the analysis band.                          */
/* ------------------------------------------------------------------------ */

int gblo_inner(const gblo_config* cfg, const double* A, const double* E, const int64_t* start_bin, int32_t N,
               const double* residual, int32_t n_res, const double* psd, int32_t n_psd, int32_t psd_is_inverse,
               const int32_t* res_idx, const int32_t* psd_idx, int64_t B, double* out) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  for (int64_t b = 0; b < B; b++) {
    if (res_idx[b] < 0 || res_idx[b] >= n_res) return -1;
    if (psd_idx[b] < 0 || psd_idx[b] >= n_psd) return -1;
  }
  double f4 = 4.0 / cfg->T;
  for (int64_t b = 0; b < B; b++) {
    const cplx* h[2] = {(const cplx*)(A + 2 * b * N), (const cplx*)(E + 2 * b * N)};
    const cplx* R = (const cplx*)(residual + (int64_t)res_idx[b] * 2 * nb * 2);
    const double* S = psd + (int64_t)psd_idx[b] * 2 * nb;
    double hh = 0.0, Rh = 0.0;
    for (int c = 0; c < 2; c++)
      for (int j = 0; j < N; j++) {
        int64_t k = start_bin[b] + j;
        if (k < k_min || k >= k_min + nb) continue;
        double w = psd_is_inverse ? S[c * nb + (k - k_min)] : 1.0 / S[c * nb + (k - k_min)];
        hh += creal(conj(h[c][j]) * h[c][j]) * w;
        Rh += creal(conj(R[c * nb + (k - k_min)]) * h[c][j]) * w;
      }
    out[2 * b] = f4 * hh;
    out[2 * b + 1] = f4 * Rh;
  }
  return 0;
}

/* Optimal SNR sqrt(<h|h>) and observed SNR <d|h> / sqrt(<h|h>) (Sec. 2,
 * after eq. like) of the width-N templates of params; data may be NULL (then
 * snr_obs is not written). */
int gblo_snr(const gblo_config* cfg, const double* params, int64_t B, int32_t N, const double* psd, int32_t n_psd,
             int32_t psd_is_inverse, const int32_t* psd_idx, const double* data, int32_t n_data,
             const int32_t* data_idx, double* snr_opt, double* snr_obs) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  if (N < 2 || (N & (N - 1))) return -2;
  double* A = (double*)malloc(sizeof(double) * 2 * N);
  double* E = (double*)malloc(sizeof(double) * 2 * N);
  int rc = 0;
  for (int64_t b = 0; b < B && rc == 0; b++) {
    int64_t sb;
    double o[2];
    if (!params_finite(cfg, params + 8 * b)) {
      snr_opt[b] = NAN;
      if (data) snr_obs[b] = NAN;
      continue;
    }
    waveform_one(cfg, params + 8 * b, N, (cplx*)A, (cplx*)E, NULL, &sb);
    int32_t ri = data ? data_idx[b] : 0;
    if (data) {
      rc = gblo_inner(cfg, A, E, &sb, N, data, n_data, psd, n_psd, psd_is_inverse, &ri, psd_idx + b, 1, o);
    } else {
      /* no data: <h|h> only, against a residual of zeros */
      double* z = (double*)calloc((size_t)4 * nb, sizeof(double));
      rc = gblo_inner(cfg, A, E, &sb, N, z, 1, psd, n_psd, psd_is_inverse, &ri, psd_idx + b, 1, o);
      free(z);
    }
    snr_opt[b] = sqrt(o[0]);
    if (data) snr_obs[b] = o[1] / sqrt(o[0]);
  }
  free(A);
  free(E);
  return rc;
}

/* Overlap of two templates (Sec. 4 "Cataloging Operation": sources are
 * grouped by their overlap; the overlap of templates a and b is the
 * normalised inner product of eq. inner over A and E):
 *   out[b] = (<a|a>, <b|b>, <a|b>, <a|b> / sqrt(<a|a> <b|b>))
 * for width-N templates of params_a[b] and params_b[b], weighted by
 * psd[psd_idx[b]]; bins outside the band contribute zero.  Undefined
 * parameters give NaN; a zero template gives a NaN overlap (0/0). */
int gblo_overlap(const gblo_config* cfg, const double* params_a, const double* params_b, int64_t B, int32_t N,
                 const double* psd, int32_t n_psd, int32_t psd_is_inverse, const int32_t* psd_idx, double* out) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  if (N < 2 || (N & (N - 1))) return -2;
  for (int64_t b = 0; b < B; b++)
    if (psd_idx[b] < 0 || psd_idx[b] >= n_psd) return -1;
  const double f4 = 4.0 / cfg->T;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < B; b++) {
    const double* pa = params_a + 8 * b;
    const double* pb = params_b + 8 * b;
    double* o = out + 4 * b;
    if (!params_finite(cfg, pa) || !params_finite(cfg, pb)) {
      o[0] = o[1] = o[2] = o[3] = NAN;
      continue;
    }
    cplx* ha = (cplx*)malloc(sizeof(cplx) * 2 * N);
    cplx* hb = (cplx*)malloc(sizeof(cplx) * 2 * N);
    int64_t ka, kb;
    waveform_one(cfg, pa, N, ha, ha + N, NULL, &ka);
    waveform_one(cfg, pb, N, hb, hb + N, NULL, &kb);
    const double* S = psd + (int64_t)psd_idx[b] * 2 * nb;
    double aa = 0, bb = 0, ab = 0;
    for (int c = 0; c < 2; c++) {
      for (int j = 0; j < N; j++) {
        int64_t k = ka + j;
        if (k < k_min || k >= k_min + nb) continue;
        double w = psd_is_inverse ? S[c * nb + (k - k_min)] : 1.0 / S[c * nb + (k - k_min)];
        aa += creal(conj(ha[c * N + j]) * ha[c * N + j]) * w;
        int64_t jb = k - kb;
        if (jb >= 0 && jb < N) ab += creal(conj(ha[c * N + j]) * hb[c * N + jb]) * w;
      }
      for (int j = 0; j < N; j++) {
        int64_t k = kb + j;
        if (k < k_min || k >= k_min + nb) continue;
        double w = psd_is_inverse ? S[c * nb + (k - k_min)] : 1.0 / S[c * nb + (k - k_min)];
        bb += creal(conj(hb[c * N + j]) * hb[c * N + j]) * w;
      }
    }
    o[0] = f4 * aa;
    o[1] = f4 * bb;
    o[2] = f4 * ab;
    o[3] = o[2] / sqrt(o[0] * o[1]);
    free(ha);
    free(hb);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Residual update: residual[res_idx[b]] += sign * (A, E) of template b,     */
/* clipped to the band.  Used to build data d = sum h + n and residuals.     */
/* ------------------------------------------------------------------------ */

int gblo_scatter_add(const gblo_config* cfg, const double* params, int64_t B, int32_t N, double sign,
                     double* residual, int32_t n_res, const int32_t* res_idx) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  if (N < 2 || (N & (N - 1))) return -2;
  cplx* a = (cplx*)malloc(sizeof(cplx) * 2 * N);
  for (int64_t b = 0; b < B; b++) {
    if (res_idx[b] < 0 || res_idx[b] >= n_res) {
      free(a);
      return -1;
    }
    if (!params_finite(cfg, params + 8 * b)) continue; /* undefined templates add nothing */
    int64_t k0;
    waveform_one(cfg, params + 8 * b, N, a, a + N, NULL, &k0);
    cplx* R = (cplx*)(residual + (int64_t)res_idx[b] * 2 * nb * 2);
    for (int c = 0; c < 2; c++)
      for (int j = 0; j < N; j++) {
        int64_t k = k0 + j;
        if (k < k_min || k >= k_min + nb) continue;
        R[c * nb + (k - k_min)] += sign * a[c * N + j];
      }
  }
  free(a);
  return 0;
}

/* ======================================================================== */
/* Sampler arithmetic (Sec. 4 and the appendix algorithms gb1 / gb2).        */
/* ======================================================================== */

/* Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
 * SC'11), written from its published definition: ten rounds of
 * (hi0, lo0) = X0 * M0, (hi1, lo1) = X2 * M1 (128-bit products),
 * X <- (hi1 ^ X1 ^ K0, lo1, hi0 ^ X3 ^ K1, lo0), keys bumped by the Weyl
 * constants between rounds. */
static void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; r++) {
    unsigned __int128 p0 = (unsigned __int128)M0 * x[0];
    unsigned __int128 p1 = (unsigned __int128)M1 * x[2];
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
  for (int i = 0; i < 4; i++) out[i] = x[i];
}

void gblo_philox(const uint64_t* ctr, const uint64_t* key, uint64_t* out) { philox4x64_10(ctr, key, out); }

/* Uniform in (0, 1) for draw `idx` of stream (sweep, move, unit):
 * counter = (sweep, move << 40 | unit, idx / 4, 0), word idx % 4,
 * u = (top 53 bits + 1/2) 2^-53. */
static double rng_uniform(uint64_t seed, int64_t sweep, int move, uint64_t unit, uint64_t idx) {
  uint64_t ctr[4] = {(uint64_t)sweep, ((uint64_t)move << 40) | unit, idx >> 2, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t o[4];
  philox4x64_10(ctr, key, o);
  return ((double)(o[idx & 3] >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

double gblo_rng_uniform(uint64_t seed, int64_t sweep, int move, uint64_t unit, uint64_t idx) {
  return rng_uniform(seed, sweep, move, unit, idx);
}

/* Sampler configuration (readings where the paper is silent):
 *  - sub-band b covers bins [k_band0 + b W, k_band0 + (b+1) W); W is the
 *    sub-band width (band_width, even; 0 means W = N, the template width);
 *    the analysis window of band b holds every bin a template of the band can
 *    reach: [k_band0 + b W - W/2 - N/2, k_band0 + (b+1) W + W/2 + N/2),
 *    2W + N bins (bands b-1..b+1 when W = N);
 *  - sampling coordinates u = (log10 A, f0, fdot, phi0, cos iota, psi,
 *    lambda, sin beta) with a uniform prior on a box; f0 of band b ranges over
 *    the band widened by W/2 on each side (samples may move halfway into the
 *    neighbours); phi0, psi, lambda are periodic (periods 2 pi, pi, 2 pi);
 *  - group stretch: z ~ g(z) ~ 1/sqrt(z) on [1/a, a], u' = X + z (u - X) with
 *    the friend X drawn uniformly from the n_friends entries of the band's
 *    stationary group (cold-chain sources of all walkers, sorted by f0) that
 *    surround the current f0; proposal factor z^(d-1), d = 8; periodic
 *    differences are taken on the circle and the result wrapped, and a
 *    proposal whose stretched periodic difference reaches half a period is
 *    rejected (beyond it the reverse move would not return);
 *  - reversible jump: every slot is flipped once per RJ step, in random order
 *    (birth from the prior: q = p, so the prior/proposal ratio is 1);
 *  - only the likelihood is tempered: accept iff ln u < beta dlnL + ln(prior
 *    ratio) + ln(proposal ratio). */
typedef struct {
  int32_t n_temps, n_walkers, n_bands, n_slots, N, n_prop, n_friends, group_every;
  int64_t k_band0;
  double stretch_a;
  uint64_t seed;
  double prior_lo[8], prior_hi[8]; /* f0 bounds unused (per band) */
  /* after the tempering step of every sweep: */
  int32_t adapt_ladder;    /* 1: adapt each band's ladder (gblo_sweep_adapt_ladder) */
  int32_t shift_ownership; /* 1: move cold-chain sources to the band their f0 now lies in */
  double adapt_lag;        /* t0 of the adaptation's decay t0 / (t + t0) */
  double adapt_time;       /* nu: the adaptation's time scale */
  int32_t band_width;      /* W, even; 0: W = N */
} gblo_sweep_config;

/* sub-band width W */
static int64_t band_w(const gblo_sweep_config* sc) { return sc->band_width > 0 ? sc->band_width : sc->N; }

#define MOVE_INMODEL 0
#define MOVE_RJ 1
#define MOVE_PT 2
#define MOVE_PTPERM 3

static const double PERIOD[8] = {0, 0, 0, 2.0 * ORC_PI, 0, ORC_PI, 2.0 * ORC_PI, 0};

static void band_f0_range(const gblo_config* cfg, const gblo_sweep_config* sc, int b, double* lo, double* hi) {
  double W = (double)band_w(sc);
  *lo = ((double)sc->k_band0 + ((double)b - 0.5) * W) / cfg->T;
  *hi = ((double)sc->k_band0 + ((double)b + 1.5) * W) / cfg->T;
}

/* sampling coordinates -> physical parameters */
static void u_to_params(const double* u, double* p) {
  p[0] = pow(10.0, u[0]);
  p[1] = u[1];
  p[2] = u[2];
  p[3] = u[3];
  p[4] = acos(u[4]);
  p[5] = u[5];
  p[6] = u[6];
  p[7] = asin(u[7]);
}

static int in_prior(const gblo_config* cfg, const gblo_sweep_config* sc, int b, const double* u) {
  double flo, fhi;
  band_f0_range(cfg, sc, b, &flo, &fhi);
  if (!(u[1] >= flo && u[1] < fhi)) return 0;
  for (int i = 0; i < 8; i++) {
    if (i == 1 || PERIOD[i] > 0) continue;
    if (!(u[i] >= sc->prior_lo[i] && u[i] <= sc->prior_hi[i])) return 0;
  }
  return 1;
}

/* Residual window of one walker: bins [k_band0 + b W - W/2 - N/2,
 * k_band0 + (b+1) W + W/2 + N/2) clipped to the analysis band, channels A and
 * E; its templates have width N. */
typedef struct {
  int64_t k0;   /* first global bin of the window */
  int len;      /* 2 W + N */
  int N;        /* template width */
  cplx* r[2];   /* per channel */
} window_t;

static int64_t win_start(const gblo_sweep_config* sc, int b) {
  return sc->k_band0 + (int64_t)b * band_w(sc) - band_w(sc) / 2 - sc->N / 2;
}

static int win_len(const gblo_sweep_config* sc) { return (int)(2 * band_w(sc) + sc->N); }

/* add s * template(u) to the window (bins outside the window or the band are dropped) */
static void window_add_template(const gblo_config* cfg, int64_t k_min, int64_t nb, window_t* w, const double* u,
                                double s) {
  int N = w->N;
  double p[8];
  u_to_params(u, p);
  cplx* a = (cplx*)malloc(sizeof(cplx) * 2 * N);
  int64_t ks;
  waveform_one(cfg, p, N, a, a + N, NULL, &ks);
  for (int c = 0; c < 2; c++)
    for (int j = 0; j < N; j++) {
      int64_t k = ks + j;
      if (k < w->k0 || k >= w->k0 + w->len || k < k_min || k >= k_min + nb) continue;
      w->r[c][k - w->k0] += s * a[c * N + j];
    }
  free(a);
}

/* swap likelihood change against the window residual R (eq. swapsource, in
 * the cancellation-free form <R|a - r> - 1/2 <a - r|a - r>); a null u means a
 * zero template (birth / death). */
static double window_dlogl(const gblo_config* cfg, int64_t k_min, int64_t nb, const window_t* w,
                           const double* inv_psd /*[2][nb]*/, const double* u_old, const double* u_new) {
  window_t d;
  d.k0 = w->k0;
  d.len = w->len;
  d.N = w->N;
  d.r[0] = (cplx*)calloc(w->len, sizeof(cplx));
  d.r[1] = (cplx*)calloc(w->len, sizeof(cplx));
  if (u_new) window_add_template(cfg, k_min, nb, &d, u_new, 1.0);
  if (u_old) window_add_template(cfg, k_min, nb, &d, u_old, -1.0);
  double Rd = 0, dd = 0;
  for (int c = 0; c < 2; c++)
    for (int i = 0; i < w->len; i++) {
      int64_t k = w->k0 + i;
      if (k < k_min || k >= k_min + nb) continue;
      double wgt = inv_psd[c * nb + (k - k_min)];
      Rd += creal(conj(w->r[c][i]) * d.r[c][i]) * wgt;
      dd += creal(conj(d.r[c][i]) * d.r[c][i]) * wgt;
    }
  free(d.r[0]);
  free(d.r[1]);
  return 4.0 / cfg->T * (Rd - 0.5 * dd);
}

static void window_load(int64_t k_min, int64_t nb, window_t* w, const cplx* buf /*[2][nb]*/) {
  for (int c = 0; c < 2; c++)
    for (int i = 0; i < w->len; i++) {
      int64_t k = w->k0 + i;
      w->r[c][i] = (k >= k_min && k < k_min + nb) ? buf[c * nb + (k - k_min)] : 0.0;
    }
}

static void window_store_add(int64_t k_min, int64_t nb, const window_t* w, cplx* buf) {
  for (int c = 0; c < 2; c++)
    for (int i = 0; i < w->len; i++) {
      int64_t k = w->k0 + i;
      if (k >= k_min && k < k_min + nb) buf[c * nb + (k - k_min)] += w->r[c][i];
    }
}

static double wrap(double x, double P) {
  double y = fmod(x, P);
  return y < 0 ? y + P : y;
}

/* group stretch draw (see the configuration comment) */
static int stretch_propose(const gblo_sweep_config* sc, const double* u, const double* group /*[G][8]*/, int G,
                           double uf, double uz, double* u_new, double* log_ratio) {
  if (G <= 0) return 0;
  /* lower bound of u's f0 in the sorted group, then the n_friends window around it */
  int lo = 0, hi = G;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (group[8 * mid + 1] < u[1])
      lo = mid + 1;
    else
      hi = mid;
  }
  int nf = sc->n_friends < G ? sc->n_friends : G;
  int start = lo - nf / 2;
  if (start < 0) start = 0;
  if (start > G - nf) start = G - nf;
  int j = start + (int)floor(uf * nf);
  const double* X = group + 8 * j;
  double a = sc->stretch_a;
  double z = ((a - 1.0) * uz + 1.0) * ((a - 1.0) * uz + 1.0) / a;
  int reversible = 1;
  for (int i = 0; i < 8; i++) {
    double diff = u[i] - X[i];
    if (PERIOD[i] > 0) {
      /* shortest signed difference on the circle, in (-P/2, P/2]; the move
       * is reversible (same friend, 1/z) only while z * diff stays inside
       * (-P/2, P/2), so a proposal beyond that is rejected */
      diff = wrap(diff + 0.5 * PERIOD[i], PERIOD[i]) - 0.5 * PERIOD[i];
      if (!(fabs(z * diff) < 0.5 * PERIOD[i])) reversible = 0;
      u_new[i] = wrap(X[i] + z * diff, PERIOD[i]);
    } else {
      u_new[i] = X[i] + z * diff;
    }
  }
  *log_ratio = 7.0 * log(z);
  return reversible;
}

/* the stretch proposal and the prior box on their own (for the tests) */
int gblo_stretch_propose(const gblo_sweep_config* sc, const double* u, const double* group, int G, double uf,
                         double uz, double* u_new, double* log_ratio) {
  return stretch_propose(sc, u, group, G, uf, uz, u_new, log_ratio);
}

int gblo_in_prior(const gblo_config* cfg, const gblo_sweep_config* sc, int b, const double* u) {
  return in_prior(cfg, sc, b, u);
}

/* state layout: u [n_t][n_w][n_b][n_slot][8], exists [n_t][n_w][n_b][n_slot],
 * betas [n_b][n_t], resid [2 parity][n_w][2][nb] (parity p buffer holds the
 * data minus the cold-chain sources of the bands with b % 2 == p),
 * inv_psd [n_w][2][nb], group [n_b][n_w * n_slot][8] + group_count [n_b],
 * stats [8] = in-model (proposed, accepted), births (proposed, accepted),
 * deaths (proposed, accepted), swaps (proposed, accepted). */
#define UIDX(sc, t, w, b, s) ((((int64_t)(t) * (sc)->n_walkers + (w)) * (sc)->n_bands + (b)) * (sc)->n_slots + (s))

/* Alg. gb1 for one (t, w, b): in-model (move 0) or RJ (move 1) band loop. */
/* ln of the prior box volume of band b in sampling coordinates (the uniform
 * prior density is its inverse) */
static double log_box_volume(const gblo_config* cfg, const gblo_sweep_config* sc, int b) {
  double flo, fhi, v = 0.0;
  band_f0_range(cfg, sc, b, &flo, &fhi);
  for (int k = 0; k < 8; k++) {
    double w = sc->prior_hi[k] - sc->prior_lo[k];
    if (k == 1) w = fhi - flo;
    else if (PERIOD[k] > 0) w = PERIOD[k];
    v += log(w);
  }
  return v;
}

/* One band loop of Alg. gb1 for chain (t, w, b).  It reads only the
 * opposite-parity cold-chain buffer; at t = 0 the change of the band's
 * sources is returned in *dsum_out (window of bands b-1..b+1, owned by the
 * caller) for the caller to add to the own-parity buffer. */
static void band_loop(const gblo_config* cfg, const gblo_sweep_config* sc, int move, int64_t sweep, int t, int w,
                      int b, double* u, int32_t* exists, const double* betas, const double* resid,
                      const double* inv_psd, const double* group, const int32_t* group_count, int64_t* stats,
                      const double* prop_u, const double* rj_logq, window_t* dsum_out) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  int par = b & 1;
  int S = sc->n_slots;
  window_t win;
  win.k0 = win_start(sc, b);
  win.len = win_len(sc);
  win.N = sc->N;
  win.r[0] = (cplx*)malloc(sizeof(cplx) * win.len);
  win.r[1] = (cplx*)malloc(sizeof(cplx) * win.len);
  window_t dsum = {win.k0, win.len, win.N,
                   {(cplx*)calloc(win.len, sizeof(cplx)), (cplx*)calloc(win.len, sizeof(cplx))}};
  const cplx* opp = (const cplx*)(resid + ((int64_t)(1 - par) * sc->n_walkers + w) * 2 * nb * 2);
  window_load(k_min, nb, &win, opp);
  /* residual of the band: subtract the band's current sources */
  for (int s = 0; s < S; s++)
    if (exists[UIDX(sc, t, w, b, s)]) window_add_template(cfg, k_min, nb, &win, u + 8 * UIDX(sc, t, w, b, s), -1.0);
  const double beta = betas[(int64_t)b * sc->n_temps + t];
  const double* ipsd = inv_psd + (int64_t)w * 2 * nb;
  const uint64_t unit = ((uint64_t)t * sc->n_walkers + w) * sc->n_bands + b;
  double un[8];
  if (move == MOVE_INMODEL) {
    const double* grp = group + (int64_t)b * sc->n_walkers * S * 8;
    int G = group_count[b];
    for (int p = 0; p < sc->n_prop; p++) {
      double r_pick = rng_uniform(sc->seed, sweep, move, unit, 8 * (uint64_t)p + 0);
      double r_friend = rng_uniform(sc->seed, sweep, move, unit, 8 * (uint64_t)p + 1);
      double r_z = rng_uniform(sc->seed, sweep, move, unit, 8 * (uint64_t)p + 2);
      double r_acc = rng_uniform(sc->seed, sweep, move, unit, 8 * (uint64_t)p + 3);
      int g = 0;
      for (int s = 0; s < S; s++) g += exists[UIDX(sc, t, w, b, s)] != 0;
      if (g == 0) continue;
      int pick = (int)floor(r_pick * g), s_k = -1;
      for (int s = 0, c = 0; s < S; s++)
        if (exists[UIDX(sc, t, w, b, s)]) {
          if (c == pick) {
            s_k = s;
            break;
          }
          c++;
        }
      double* uk = u + 8 * UIDX(sc, t, w, b, s_k);
      double lr;
      stats[0]++;
      if (!stretch_propose(sc, uk, grp, G, r_friend, r_z, un, &lr)) continue;
      if (!in_prior(cfg, sc, b, un)) continue;
      double dl = window_dlogl(cfg, k_min, nb, &win, ipsd, uk, un);
      if (log(r_acc) < beta * dl + lr) {
        window_add_template(cfg, k_min, nb, &win, uk, 1.0);
        window_add_template(cfg, k_min, nb, &win, un, -1.0);
        if (t == 0) {
          window_add_template(cfg, k_min, nb, &dsum, uk, 1.0);
          window_add_template(cfg, k_min, nb, &dsum, un, -1.0);
        }
        for (int i = 0; i < 8; i++) uk[i] = un[i];
        stats[1]++;
      }
    }
  } else {
    /* flip every slot once, in a random order (Fisher-Yates) */
    int order[64];
    for (int s = 0; s < S; s++) order[s] = s;
    for (int j = S - 1; j >= 1; j--) {
      int r = (int)floor(rng_uniform(sc->seed, sweep, move, unit, (uint64_t)j) * (j + 1));
      int tmp = order[j];
      order[j] = order[r];
      order[r] = tmp;
    }
    double flo, fhi;
    band_f0_range(cfg, sc, b, &flo, &fhi);
    for (int i = 0; i < S; i++) {
      int s = order[i];
      uint64_t base = 64 + 16 * (uint64_t)i;
      double r_acc = rng_uniform(sc->seed, sweep, move, unit, base);
      int64_t ui = UIDX(sc, t, w, b, s);
      double* us = u + 8 * ui;
      if (exists[ui]) {
        /* death: new template zero; with the prior proposal (q = p) the densities
         * cancel, otherwise ln alpha gains ln q(theta) - ln p(theta) */
        stats[4]++;
        double dl = window_dlogl(cfg, k_min, nb, &win, ipsd, us, NULL);
        double lpq = rj_logq ? rj_logq[ui] + log_box_volume(cfg, sc, b) : 0.0;
        if (log(r_acc) < beta * dl + lpq) {
          window_add_template(cfg, k_min, nb, &win, us, 1.0);
          if (t == 0) window_add_template(cfg, k_min, nb, &dsum, us, 1.0);
          exists[ui] = 0;
          stats[5]++;
        }
      } else {
        stats[2]++;
        if (prop_u) {
          /* birth from the given proposal: ln alpha gains ln p(theta) - ln q(theta) */
          for (int k = 0; k < 8; k++) un[k] = prop_u[8 * ui + k];
          if (!in_prior(cfg, sc, b, un)) continue;
          double dl = window_dlogl(cfg, k_min, nb, &win, ipsd, NULL, un);
          if (log(r_acc) < beta * dl - log_box_volume(cfg, sc, b) - rj_logq[ui]) {
            window_add_template(cfg, k_min, nb, &win, un, -1.0);
            if (t == 0) window_add_template(cfg, k_min, nb, &dsum, un, -1.0);
            for (int k = 0; k < 8; k++) us[k] = un[k];
            exists[ui] = 1;
            stats[3]++;
          }
          continue;
        }
        /* birth from the prior */
        for (int k = 0; k < 8; k++) {
          double r = rng_uniform(sc->seed, sweep, move, unit, base + 1 + k);
          double lo = sc->prior_lo[k], hi = sc->prior_hi[k];
          if (k == 1) {
            lo = flo;
            hi = fhi;
          } else if (PERIOD[k] > 0) {
            lo = 0.0;
            hi = PERIOD[k];
          }
          un[k] = lo + (hi - lo) * r;
        }
        double dl = window_dlogl(cfg, k_min, nb, &win, ipsd, NULL, un);
        if (log(r_acc) < beta * dl) {
          window_add_template(cfg, k_min, nb, &win, un, -1.0);
          if (t == 0) window_add_template(cfg, k_min, nb, &dsum, un, -1.0);
          for (int k = 0; k < 8; k++) us[k] = un[k];
          exists[ui] = 1;
          stats[3]++;
        }
      }
    }
  }
  /* cold chain: the change of the band's sources, for its own buffer */
  if (t == 0) {
    *dsum_out = dsum;
  } else {
    free(dsum.r[0]);
    free(dsum.r[1]);
  }
  free(win.r[0]);
  free(win.r[1]);
}

/* band log-likelihood of the source set (t, w_src, b) against walker w_res's
 * residual (the opposite-parity cold-chain buffer over bands b-1..b+1):
 * -1/2 <r'|r'> over the window, r' = buffer - sum h (Alg. gb2). */
static double band_loglike(const gblo_config* cfg, const gblo_sweep_config* sc, int t, int w_src, int b, int w_res,
                           const double* u, const int32_t* exists, const double* resid, const double* inv_psd) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  window_t win;
  win.k0 = win_start(sc, b);
  win.len = win_len(sc);
  win.N = sc->N;
  win.r[0] = (cplx*)malloc(sizeof(cplx) * win.len);
  win.r[1] = (cplx*)malloc(sizeof(cplx) * win.len);
  int par = b & 1;
  window_load(k_min, nb, &win, (const cplx*)(resid + ((int64_t)(1 - par) * sc->n_walkers + w_res) * 2 * nb * 2));
  for (int s = 0; s < sc->n_slots; s++)
    if (exists[UIDX(sc, t, w_src, b, s)])
      window_add_template(cfg, k_min, nb, &win, u + 8 * UIDX(sc, t, w_src, b, s), -1.0);
  const double* ipsd = inv_psd + (int64_t)w_res * 2 * nb;
  double rr = 0;
  for (int c = 0; c < 2; c++)
    for (int i = 0; i < win.len; i++) {
      int64_t k = win.k0 + i;
      if (k < k_min || k >= k_min + nb) continue;
      rr += creal(conj(win.r[c][i]) * win.r[c][i]) * ipsd[c * nb + (k - k_min)];
    }
  free(win.r[0]);
  free(win.r[1]);
  return -0.5 * 4.0 / cfg->T * rr;
}

double gblo_band_loglike(const gblo_config* cfg, const gblo_sweep_config* sc, int t, int w_src, int b, int w_res,
                         const double* u, const int32_t* exists, const double* resid, const double* inv_psd) {
  return band_loglike(cfg, sc, t, w_src, b, w_res, u, exists, resid, inv_psd);
}

/* walker permutation of temperature t in band b (Fisher-Yates) */
static void pt_permutation(const gblo_sweep_config* sc, int64_t sweep, int b, int t, int* perm) {
  for (int i = 0; i < sc->n_walkers; i++) perm[i] = i;
  uint64_t unit = (uint64_t)b * sc->n_temps + t;
  for (int j = sc->n_walkers - 1; j >= 1; j--) {
    int r = (int)floor(rng_uniform(sc->seed, sweep, MOVE_PTPERM, unit, (uint64_t)j) * (j + 1));
    int tmp = perm[j];
    perm[j] = perm[r];
    perm[r] = tmp;
  }
}

static void swap_sets(const gblo_sweep_config* sc, int t1, int w1, int t2, int w2, int b, double* u, int32_t* ex) {
  for (int s = 0; s < sc->n_slots; s++) {
    int64_t i1 = UIDX(sc, t1, w1, b, s), i2 = UIDX(sc, t2, w2, b, s);
    for (int k = 0; k < 8; k++) {
      double tmp = u[8 * i1 + k];
      u[8 * i1 + k] = u[8 * i2 + k];
      u[8 * i2 + k] = tmp;
    }
    int32_t e = ex[i1];
    ex[i1] = ex[i2];
    ex[i2] = e;
  }
}

/* eq. temp-final: walker i at inverse temperature bI holds parameters n,
 * walker j at bII holds m; L_xy = likelihood of walker x's data at parameters
 * y.  Returns ln alpha = bI (ln L_im - ln L_in) + bII (ln L_jn - ln L_jm). */
static double pt_log_alpha(double bI, double bII, double lnL_im, double lnL_in, double lnL_jn, double lnL_jm) {
  return bI * (lnL_im - lnL_in) + bII * (lnL_jn - lnL_jm);
}

double gblo_pt_log_alpha(double bI, double bII, double lnL_im, double lnL_in, double lnL_jn, double lnL_jm) {
  return pt_log_alpha(bI, bII, lnL_im, lnL_in, lnL_jn, lnL_jm);
}

/* Alg. gb2 for band b and ensemble index i: swaps from the hottest pair down,
 * accepted with the residual-aware ratio (eq. temp-final). */
/* It reads only the opposite-parity cold-chain buffer; an accepted swap at
 * t = 1 returns the change of walker w_0's cold-chain sources in *dw_out
 * (dw_out->r[0] stays NULL otherwise) for the caller to add to the
 * own-parity buffer of walker *w0_out. */
static void pt_chain(const gblo_config* cfg, const gblo_sweep_config* sc, int64_t sweep, int b, int i, double* u,
                     int32_t* exists, const double* betas, const double* resid, const double* inv_psd,
                     int64_t* stats, double* cold_logl, window_t* dw_out, int* w0_out, int32_t* acc_t) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  int nt = sc->n_temps;
  int* wt = (int*)malloc(sizeof(int) * nt);
  int* perm = (int*)malloc(sizeof(int) * sc->n_walkers);
  for (int t = 0; t < nt; t++) {
    pt_permutation(sc, sweep, b, t, perm);
    wt[t] = perm[i];
  }
  double* Lc = (double*)malloc(sizeof(double) * nt);
  for (int t = 0; t < nt; t++) Lc[t] = band_loglike(cfg, sc, t, wt[t], b, wt[t], u, exists, resid, inv_psd);
  const double* bt = betas + (int64_t)b * nt;
  for (int t = nt - 1; t >= 1; t--) {
    /* L1: sources of (t-1) against walker w_t's residual; L2: sources of t against w_(t-1)'s */
    double L1 = band_loglike(cfg, sc, t - 1, wt[t - 1], b, wt[t], u, exists, resid, inv_psd);
    double L2 = band_loglike(cfg, sc, t, wt[t], b, wt[t - 1], u, exists, resid, inv_psd);
    double la = pt_log_alpha(bt[t], bt[t - 1], L1, Lc[t], L2, Lc[t - 1]);
    double r = rng_uniform(sc->seed, sweep, MOVE_PT, (uint64_t)b * sc->n_walkers + i, (uint64_t)t);
    stats[6]++;
    if (log(r) < la) {
      stats[7]++;
      acc_t[t]++;
      if (t == 1) {
        /* new cold-chain sources for walker w_0: update its own-parity buffer */
        window_t dw;
        dw.k0 = win_start(sc, b);
        dw.len = win_len(sc);
        dw.N = sc->N;
        dw.r[0] = (cplx*)calloc(dw.len, sizeof(cplx));
        dw.r[1] = (cplx*)calloc(dw.len, sizeof(cplx));
        for (int s = 0; s < sc->n_slots; s++) {
          if (exists[UIDX(sc, 0, wt[0], b, s)])
            window_add_template(cfg, k_min, nb, &dw, u + 8 * UIDX(sc, 0, wt[0], b, s), 1.0);
          if (exists[UIDX(sc, 1, wt[1], b, s)])
            window_add_template(cfg, k_min, nb, &dw, u + 8 * UIDX(sc, 1, wt[1], b, s), -1.0);
        }
        *dw_out = dw;
        *w0_out = wt[0];
      }
      swap_sets(sc, t, wt[t], t - 1, wt[t - 1], b, u, exists);
      Lc[t] = L1;
      Lc[t - 1] = L2;
    }
  }
  /* band log-likelihood of the cold chain of walker w_0 after the swaps */
  if (cold_logl) cold_logl[(int64_t)wt[0] * sc->n_bands + b] = Lc[0];
  free(wt);
  free(perm);
  free(Lc);
}

/* One step of the sweep over all bands of one parity:
 * move 0 in-model, 1 reversible jump (Alg. gb1), 2 tempering (Alg. gb2). */
/* prop_u / rj_logq (both NULL: prior RJ proposal): per slot, the birth
 * candidate (read for empty slots) and ln q of the proposal density at the
 * candidate (empty slot) or at the current source (occupied slot).
 * cold_logl [n_w][n_b] (may be NULL): tempering writes the cold chain's band
 * log-likelihood after the swaps. */
/* swap_acc [n_b][n_t] (may be NULL): tempering adds, per band, the number of
 * accepted swaps between rungs t-1 and t at entry t. */
int gblo_sweep_step(const gblo_config* cfg, const gblo_sweep_config* sc, int move, int parity, int64_t sweep,
                    double* u, int32_t* exists, const double* betas, double* resid, const double* inv_psd,
                    const double* group, const int32_t* group_count, int64_t* stats, const double* prop_u,
                    const double* rj_logq, double* cold_logl, int32_t* swap_acc) {
  if (sc->n_slots > 64 || sc->n_slots < 1) return -1;
  if ((prop_u == NULL) != (rj_logq == NULL)) return -1;
  if (sc->band_width < 0 || (sc->band_width & 1)) return -1;
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  /* The units of one step -- band loops (t, w, b), or tempering chains
   * (b, i) -- touch disjoint slots and read only the opposite-parity
   * buffers, so they may run in any order; their cold-chain changes are then
   * added to the own-parity buffers one by one in the sequential order (b,
   * then t, w or i), which gives exactly the sums of a sequential loop. */
  const int per_band = move == MOVE_PT ? sc->n_walkers : sc->n_temps * sc->n_walkers;
  const int n_par_bands = (sc->n_bands - parity + 1) / 2;
  const int64_t n_units = (int64_t)n_par_bands * per_band;
  window_t* dw = (window_t*)calloc((size_t)(n_units > 0 ? n_units : 1), sizeof(window_t));
  int* w0 = (int*)calloc((size_t)(n_units > 0 ? n_units : 1), sizeof(int));
  int64_t* st = (int64_t*)calloc((size_t)(n_units > 0 ? n_units : 1) * 8, sizeof(int64_t));
  int32_t* acc = (int32_t*)calloc((size_t)(n_units > 0 ? n_units : 1) * sc->n_temps, sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < n_units; q++) {
    const int b = parity + 2 * (int)(q / per_band);
    const int r = (int)(q % per_band);
    if (move == MOVE_PT) {
      pt_chain(cfg, sc, sweep, b, r, u, exists, betas, resid, inv_psd, st + 8 * q, cold_logl, dw + q, w0 + q,
               acc + (int64_t)sc->n_temps * q);
    } else {
      const int t = r / sc->n_walkers, w = r % sc->n_walkers;
      band_loop(cfg, sc, move, sweep, t, w, b, u, exists, betas, resid, inv_psd, group, group_count, st + 8 * q,
                prop_u, rj_logq, dw + q);
      w0[q] = w;
    }
  }
  for (int64_t q = 0; q < n_units; q++) {
    for (int k = 0; k < 8; k++) stats[k] += st[8 * q + k];
    if (swap_acc && move == MOVE_PT) {
      const int b = parity + 2 * (int)(q / per_band);
      for (int t = 0; t < sc->n_temps; t++) swap_acc[(int64_t)b * sc->n_temps + t] += acc[(int64_t)sc->n_temps * q + t];
    }
    if (dw[q].r[0]) {
      const int b = parity + 2 * (int)(q / per_band);
      cplx* own = (cplx*)(resid + ((int64_t)(b & 1) * sc->n_walkers + w0[q]) * 2 * nb * 2);
      window_store_add(k_min, nb, dw + q, own);
      free(dw[q].r[0]);
      free(dw[q].r[1]);
    }
  }
  free(dw);
  free(w0);
  free(st);
  free(acc);
  return 0;
}

/* ------------------------------------------------------------------------
 * Temperature-ladder adaptation (appendix "Parallel tempering in a
 * residual-based analysis": each sub-band's ladder adapts on its own, after
 * Vousden, Farr & Mandel 2016).  With T = 1/beta, the gaps between adjacent
 * rungs evolve as S_j = ln(T_(j+1) - T_j), dS_j = kappa (A_j - A_(j+1)),
 * kappa = t0 / (nu (t + t0)), A_j the fraction of accepted swaps between
 * rungs j and j+1 at this sweep (swap_acc[b][j+1] / n_walkers), t the sweep
 * index; the coldest (beta = 1) and hottest rungs stay fixed, the rungs in
 * between are the coldest temperature plus the running sum of the new gaps.
 * swap_acc is cleared afterwards.
 * ------------------------------------------------------------------------ */
int gblo_sweep_adapt_ladder(const gblo_sweep_config* sc, int64_t sweep, double* betas, int32_t* swap_acc) {
  const int nt = sc->n_temps;
  const double kappa = sc->adapt_lag / (sc->adapt_time * ((double)sweep + sc->adapt_lag));
  double* gap = (double*)malloc(sizeof(double) * (nt > 1 ? nt : 1));
  for (int b = 0; b < sc->n_bands; b++) {
    double* bt = betas + (int64_t)b * nt;
    int32_t* ac = swap_acc + (int64_t)b * nt;
    if (nt > 2) {
      /* new gaps of the rungs 0..nt-2 (the last rung does not move) */
      for (int j = 0; j + 2 < nt; j++) {
        const double A_lo = (double)ac[j + 1] / (double)sc->n_walkers; /* rungs j, j+1 */
        const double A_hi = (double)ac[j + 2] / (double)sc->n_walkers; /* rungs j+1, j+2 */
        gap[j] = (1.0 / bt[j + 1] - 1.0 / bt[j]) * exp(kappa * (A_lo - A_hi));
      }
      double T = 1.0 / bt[0];
      for (int j = 0; j + 2 < nt; j++) {
        T += gap[j];
        bt[j + 1] = 1.0 / T;
      }
    }
    for (int t = 0; t < nt; t++) ac[t] = 0;
  }
  free(gap);
  return 0;
}

/* ------------------------------------------------------------------------
 * Sub-band ownership (Sec. 4 "Galactic binary search and parameter
 * estimation"): samples may roam half a band into the neighbours; a
 * cold-chain source whose f0 has left its band's nominal range [k_band0 +
 * b W, k_band0 + (b+1) W) / T moves to the neighbouring band it now lies in,
 * into that band's lowest free cold-chain slot (it stays if there is none).
 * The source then belongs to the opposite parity: it is added back to the
 * old parity's buffer and removed from the new one's.  Per walker, bands in
 * increasing order, slots in increasing order.  stats (may be NULL): [0]
 * sources moved, [1] sources that found no free slot.
 * ------------------------------------------------------------------------ */
int gblo_sweep_shift_ownership(const gblo_config* cfg, const gblo_sweep_config* sc, double* u, int32_t* exists,
                               double* resid, int64_t* stats) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  const int S = sc->n_slots;
  for (int w = 0; w < sc->n_walkers; w++)
    for (int b = 0; b < sc->n_bands; b++)
      for (int s = 0; s < S; s++) {
        const int64_t ui = UIDX(sc, 0, w, b, s);
        if (!exists[ui]) continue;
        const double f0 = u[8 * ui + 1];
        const double lo = (double)(sc->k_band0 + (int64_t)b * band_w(sc)) / cfg->T;
        const double hi = (double)(sc->k_band0 + (int64_t)(b + 1) * band_w(sc)) / cfg->T;
        int bb = f0 < lo ? b - 1 : (f0 >= hi ? b + 1 : b);
        if (bb == b || bb < 0 || bb >= sc->n_bands) continue;
        int s2 = -1;
        for (int j = 0; j < S && s2 < 0; j++)
          if (!exists[UIDX(sc, 0, w, bb, j)]) s2 = j;
        if (s2 < 0) {
          if (stats) stats[1]++;
          continue;
        }
        const int64_t u2 = UIDX(sc, 0, w, bb, s2);
        for (int k = 0; k < 8; k++) u[8 * u2 + k] = u[8 * ui + k];
        exists[u2] = 1;
        exists[ui] = 0;
        double p[8];
        u_to_params(u + 8 * u2, p);
        const int32_t ri_old = (b & 1) * sc->n_walkers + w, ri_new = (bb & 1) * sc->n_walkers + w;
        gblo_scatter_add(cfg, p, 1, sc->N, 1.0, resid, 2 * sc->n_walkers, &ri_old);
        gblo_scatter_add(cfg, p, 1, sc->N, -1.0, resid, 2 * sc->n_walkers, &ri_new);
        if (stats) stats[0]++;
      }
  return 0;
}

/* Stationary group per band: the cold-chain (t = 0) sources of every walker,
 * sorted by f0 (ties by walker, then slot). */
int gblo_sweep_group(const gblo_sweep_config* sc, const double* u, const int32_t* exists, double* group,
                     int32_t* group_count) {
  int S = sc->n_slots;
  for (int b = 0; b < sc->n_bands; b++) {
    double* g = group + (int64_t)b * sc->n_walkers * S * 8;
    int n = 0;
    for (int w = 0; w < sc->n_walkers; w++)
      for (int s = 0; s < S; s++)
        if (exists[UIDX(sc, 0, w, b, s)]) {
          for (int k = 0; k < 8; k++) g[8 * n + k] = u[8 * UIDX(sc, 0, w, b, s) + k];
          n++;
        }
    /* insertion sort by f0 (stable) */
    for (int i = 1; i < n; i++) {
      double tmp[8];
      for (int k = 0; k < 8; k++) tmp[k] = g[8 * i + k];
      int j = i - 1;
      while (j >= 0 && g[8 * j + 1] > tmp[1]) {
        for (int k = 0; k < 8; k++) g[8 * (j + 1) + k] = g[8 * j + k];
        j--;
      }
      for (int k = 0; k < 8; k++) g[8 * (j + 1) + k] = tmp[k];
    }
    group_count[b] = n;
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Noise-PSD step of the sweep (Sec. 3 eq. psd with the likelihood of Sec. 2
 * eq. like; Sec. 4: the PSD parameters are sampled with ensemble stretch
 * moves, eq. stretch, and vertical tempering: chain (t, w) always uses walker
 * w's residual, so a temperature swap is the plain eq. temp-orig).
 * theta [n_tn][n_w][n_par] = (sqrt S_oms^A, sqrt S_acc^A, sqrt S_oms^E,
 * sqrt S_acc^E) and, with n_par = 9, the foreground (A_fg, alpha, f_k, s1,
 * s2); uniform prior box; full residual of walker w = the sum of its
 * two cold-chain buffers minus the data.  Random numbers: stretch unit
 * t n_w + w, move 4, draws 4 h + (0 partner, 1 z, 2 accept) for half h;
 * swaps unit w, move 5, draw t.  stats: stretch (proposed, accepted), swaps
 * (proposed, accepted).
 * ------------------------------------------------------------------------ */
#define MOVE_PSD 4
#define MOVE_PSDPT 5

typedef struct {
  int32_t n_tn, n_walkers;
  int32_t n_par; /* 4: instrument noise only; 9: with the Galactic foreground (Sec. 3) */
  double stretch_a;
  uint64_t seed;
  double prior_lo[9], prior_hi[9];
} gblo_psd_sweep_config;

int gblo_psd_sweep_step(const gblo_config* cfg, const gblo_psd_sweep_config* pc, int64_t sweep, double* theta,
                        double* logl, const double* betas, const double* data, const double* resid,
                        double* inv_psd, int64_t* stats) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  const int nt = pc->n_tn, nw = pc->n_walkers, np_ = pc->n_par;
  if (nw < 2 || nw % 2) return -1;
  if (np_ != 4 && np_ != 9) return -1;
  /* full residual per walker: buffer 0 + buffer 1 - data */
  double* R = (double*)malloc(sizeof(double) * (size_t)nw * 2 * nb * 2);
  for (int w = 0; w < nw; w++)
    for (int64_t i = 0; i < 2 * nb * 2; i++)
      R[(int64_t)w * 2 * nb * 2 + i] = resid[((int64_t)0 * nw + w) * 2 * nb * 2 + i] +
                                       resid[((int64_t)1 * nw + w) * 2 * nb * 2 + i] - data[i];
  int32_t* ridx = (int32_t*)malloc(sizeof(int32_t) * (size_t)nt * nw);
  for (int t = 0; t < nt; t++)
    for (int w = 0; w < nw; w++) ridx[t * nw + w] = w;
  /* current log-likelihoods against the current residuals */
  gblo_psd_loglike_n(cfg, R, nw, theta, np_, ridx, (int64_t)nt * nw, logl);
  double* prop = (double*)malloc(sizeof(double) * (size_t)nt * nw * np_);
  double* lprop = (double*)malloc(sizeof(double) * (size_t)nt * nw);
  int* ok = (int*)malloc(sizeof(int) * (size_t)nt * nw);
  double* lz = (double*)malloc(sizeof(double) * (size_t)nt * nw);
  const int half = nw / 2;
  for (int h = 0; h < 2; h++) {
    /* proposals for the walkers of half h, partners from the other half (eq. stretch) */
    for (int t = 0; t < nt; t++)
      for (int w = h; w < nw; w += 2) {
        uint64_t unit = (uint64_t)t * nw + w;
        double r_pick = rng_uniform(pc->seed, sweep, MOVE_PSD, unit, 4 * (uint64_t)h + 0);
        double r_z = rng_uniform(pc->seed, sweep, MOVE_PSD, unit, 4 * (uint64_t)h + 1);
        int j = 2 * (int)floor(r_pick * half) + (1 - h);
        double a = pc->stretch_a;
        double z = ((a - 1.0) * r_z + 1.0) * ((a - 1.0) * r_z + 1.0) / a;
        const double* X = theta + ((int64_t)t * nw + j) * np_;
        const double* Y = theta + ((int64_t)t * nw + w) * np_;
        double* P = prop + ((int64_t)t * nw + w) * np_;
        int inside = 1;
        for (int k = 0; k < np_; k++) {
          P[k] = X[k] + z * (Y[k] - X[k]);
          if (!(P[k] >= pc->prior_lo[k] && P[k] <= pc->prior_hi[k])) inside = 0;
        }
        ok[t * nw + w] = inside;
        lz[t * nw + w] = (double)(np_ - 1) * log(z); /* z^(d-1), d = n_par */
      }
    for (int t = 0; t < nt; t++)
      for (int w = h; w < nw; w += 2)
        if (ok[t * nw + w])
          gblo_psd_loglike_n(cfg, R, nw, prop + ((int64_t)t * nw + w) * np_, np_, &w, 1, lprop + t * nw + w);
    for (int t = 0; t < nt; t++)
      for (int w = h; w < nw; w += 2) {
        stats[0]++;
        if (!ok[t * nw + w]) continue;
        uint64_t unit = (uint64_t)t * nw + w;
        double r_acc = rng_uniform(pc->seed, sweep, MOVE_PSD, unit, 4 * (uint64_t)h + 2);
        double la = betas[t] * (lprop[t * nw + w] - logl[t * nw + w]) + lz[t * nw + w];
        if (log(r_acc) < la) {
          for (int k = 0; k < np_; k++) theta[((int64_t)t * nw + w) * np_ + k] = prop[((int64_t)t * nw + w) * np_ + k];
          logl[t * nw + w] = lprop[t * nw + w];
          stats[1]++;
        }
      }
  }
  /* temperature swaps per walker, hottest pair first (eq. temp-orig) */
  for (int w = 0; w < nw; w++)
    for (int t = nt - 1; t >= 1; t--) {
      stats[2]++;
      double r = rng_uniform(pc->seed, sweep, MOVE_PSDPT, (uint64_t)w, (uint64_t)t);
      double la = (betas[t - 1] - betas[t]) * (logl[t * nw + w] - logl[(t - 1) * nw + w]);
      if (log(r) < la) {
        for (int k = 0; k < np_; k++) {
          double tmp = theta[((int64_t)t * nw + w) * np_ + k];
          theta[((int64_t)t * nw + w) * np_ + k] = theta[((int64_t)(t - 1) * nw + w) * np_ + k];
          theta[((int64_t)(t - 1) * nw + w) * np_ + k] = tmp;
        }
        double tl = logl[t * nw + w];
        logl[t * nw + w] = logl[(t - 1) * nw + w];
        logl[(t - 1) * nw + w] = tl;
        stats[3]++;
      }
    }
  /* the cold chain's PSD for the GB likelihood */
  double* S = (double*)malloc(sizeof(double) * 2 * nb);
  for (int w = 0; w < nw; w++) {
    gblo_psd_eval_n(cfg, theta + (int64_t)w * np_, np_, 1, S);
    for (int64_t i = 0; i < 2 * nb; i++) inv_psd[(int64_t)w * 2 * nb + i] = 1.0 / S[i];
  }
  free(S);
  free(R);
  free(ridx);
  free(prop);
  free(lprop);
  free(ok);
  free(lz);
  return 0;
}

/* ------------------------------------------------------------------------
 * Search for the loudest remaining source per sub-band (appendix
 * "Algorithm for fitting proposal distributions"; Sec. 4 "Online updating of
 * RJ sampling distributions", the search RJ proposal): independent,
 * fixed-dimensional (one source, d = 8), parallel-tempered ensemble samplers,
 * one per sub-band, with the stretch proposal of eq. stretch; the prior
 * confines f0 to the sub-band (no roaming across its edges); the target is
 * the likelihood gain of adding the source to the residual,
 *   l(u) = <R|h(u)> - 1/2 <h(u)|h(u)>   (eq. addsource),
 * tempered as beta_t l.  A sub-band has converged when its best cold-chain
 * l has not improved for n_stall consecutive iterations; converged bands
 * stop moving.
 *   u [n_b][n_t][n_w][8] sampling coordinates (log10 A, f0, fdot, phi0,
 *   cos iota, psi, lambda, sin beta), logl [n_b][n_t][n_w], betas [n_t],
 *   best_u [n_b][8], best_logl [n_b], stall [n_b].
 * One iteration: for half h = 0, 1 every chain (b, t, w) with w % 2 == h
 * proposes Y = X_j + z (X_w - X_j), j = 2 floor(U0 n_w/2) + 1 - h of the same
 * (b, t), z = ((a-1) U1 + 1)^2 / a (periodic coordinates on the circle, with
 * the group stretch's reversibility rule), accepted iff ln U2 < beta_t (l' - l)
 * + 7 ln z inside the prior box; then per (b, w) swaps from the hottest pair
 * down with eq. temp-orig; then the best-point bookkeeping (first maximum
 * over the cold walkers).  Random numbers: stretch unit (b n_t + t) n_w + w,
 * move 6, draws 4 (iteration-local) h + k; swaps unit b n_w + w, move 7,
 * draw t.  stats: [0] proposed, [1] accepted, [2] swaps proposed, [3]
 * accepted.
 * ------------------------------------------------------------------------ */
#define MOVE_SEARCH 6
#define MOVE_SEARCH_PT 7

typedef struct {
  int32_t n_bands, n_temps, n_walkers; /* n_walkers even */
  int32_t N;                           /* template width */
  int32_t width;                       /* sub-band width in bins */
  int32_t n_stall;                     /* convergence: iterations without improvement */
  int64_t k_band0;                     /* first bin of sub-band 0 */
  double stretch_a;
  uint64_t seed;
  double prior_lo[8], prior_hi[8];     /* f0 and the periodic coordinates are set per band / by period */
} gblo_search_config;

static const double SEARCH_PERIOD[8] = {0, 0, 0, 2.0 * ORC_PI, 0, ORC_PI, 2.0 * ORC_PI, 0};

static void search_box(const gblo_config* cfg, const gblo_search_config* sc, int b, double* lo, double* hi) {
  for (int k = 0; k < 8; k++) {
    lo[k] = sc->prior_lo[k];
    hi[k] = sc->prior_hi[k];
    if (SEARCH_PERIOD[k] > 0) {
      lo[k] = 0.0;
      hi[k] = SEARCH_PERIOD[k];
    }
  }
  lo[1] = (double)(sc->k_band0 + (int64_t)b * sc->width) / cfg->T;
  hi[1] = (double)(sc->k_band0 + (int64_t)(b + 1) * sc->width) / cfg->T;
}

static int search_in_prior(const gblo_config* cfg, const gblo_search_config* sc, int b, const double* u) {
  double lo[8], hi[8];
  search_box(cfg, sc, b, lo, hi);
  if (!(u[1] >= lo[1] && u[1] < hi[1])) return 0;
  for (int k = 0; k < 8; k++) {
    if (k == 1 || SEARCH_PERIOD[k] > 0) continue;
    if (!(u[k] >= lo[k] && u[k] <= hi[k])) return 0;
  }
  return 1;
}

/* l(u) for a list of sampling points: the birth likelihood change */
static void search_logl(const gblo_config* cfg, const gblo_search_config* sc, const double* residual,
                        const double* psd, int64_t n, const double* u, double* out) {
  double* pn = (double*)malloc(sizeof(double) * 8 * (size_t)(n > 0 ? n : 1));
  double* po = (double*)calloc(8 * (size_t)(n > 0 ? n : 1), sizeof(double));
  int32_t* idx = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  for (int64_t i = 0; i < n; i++) {
    u_to_params(u + 8 * i, pn + 8 * i);
    for (int k = 1; k < 8; k++) po[8 * i + k] = pn[8 * i + k]; /* zero amplitude: a birth */
  }
  gblo_delta_loglike(cfg, residual, 1, psd, 1, 0, po, pn, sc->N, idx, idx, n, out, NULL);
  free(pn);
  free(po);
  free(idx);
}

/* logl of every chain at its current point */
int gblo_search_eval(const gblo_config* cfg, const gblo_search_config* sc, const double* residual,
                     const double* psd, const double* u, double* logl) {
  search_logl(cfg, sc, residual, psd, (int64_t)sc->n_bands * sc->n_temps * sc->n_walkers, u, logl);
  return 0;
}

int gblo_search_step(const gblo_config* cfg, const gblo_search_config* sc, int64_t iter, const double* residual,
                     const double* psd, double* u, double* logl, const double* betas, double* best_u,
                     double* best_logl, int32_t* stall, int64_t* stats) {
  const int nb = sc->n_bands, nt = sc->n_temps, nw = sc->n_walkers, half = nw / 2;
  if (nw < 2 || nw % 2) return -1;
  const int64_t n_half = (int64_t)nb * nt * half;
  double* prop = (double*)malloc(sizeof(double) * 8 * (size_t)n_half);
  double* lprop = (double*)malloc(sizeof(double) * (size_t)n_half);
  double* lz = (double*)malloc(sizeof(double) * (size_t)n_half);
  int* ok = (int*)malloc(sizeof(int) * (size_t)n_half);
  const double a = sc->stretch_a;
  for (int h = 0; h < 2; h++) {
    for (int b = 0; b < nb; b++)
      for (int t = 0; t < nt; t++)
        for (int i = 0; i < half; i++) {
          const int w = 2 * i + h;
          const int64_t s = ((int64_t)b * nt + t) * half + i;
          ok[s] = 0;
          if (stall[b] >= sc->n_stall) continue; /* converged band */
          const uint64_t unit = ((uint64_t)b * nt + t) * nw + w;
          const double r_pick = rng_uniform(sc->seed, iter, MOVE_SEARCH, unit, 4 * (uint64_t)h + 0);
          const double r_z = rng_uniform(sc->seed, iter, MOVE_SEARCH, unit, 4 * (uint64_t)h + 1);
          const int j = 2 * (int)floor(r_pick * half) + (1 - h);
          const double z = ((a - 1.0) * r_z + 1.0) * ((a - 1.0) * r_z + 1.0) / a;
          const double* X = u + 8 * (((int64_t)b * nt + t) * nw + j);
          const double* Y = u + 8 * (((int64_t)b * nt + t) * nw + w);
          double* P = prop + 8 * s;
          int rev = 1;
          for (int k = 0; k < 8; k++) {
            double diff = Y[k] - X[k];
            if (SEARCH_PERIOD[k] > 0) {
              diff = wrap(diff + 0.5 * SEARCH_PERIOD[k], SEARCH_PERIOD[k]) - 0.5 * SEARCH_PERIOD[k];
              if (!(fabs(z * diff) < 0.5 * SEARCH_PERIOD[k])) rev = 0;
              P[k] = wrap(X[k] + z * diff, SEARCH_PERIOD[k]);
            } else {
              P[k] = X[k] + z * diff;
            }
          }
          ok[s] = rev && search_in_prior(cfg, sc, b, P);
          lz[s] = 7.0 * log(z);
        }
    /* likelihood of the proposals inside the prior */
    int64_t n_ok = 0;
    for (int64_t s = 0; s < n_half; s++) n_ok += ok[s];
    double* pu = (double*)malloc(sizeof(double) * 8 * (size_t)(n_ok > 0 ? n_ok : 1));
    double* pl = (double*)malloc(sizeof(double) * (size_t)(n_ok > 0 ? n_ok : 1));
    for (int64_t s = 0, c = 0; s < n_half; s++)
      if (ok[s]) {
        for (int k = 0; k < 8; k++) pu[8 * c + k] = prop[8 * s + k];
        c++;
      }
    search_logl(cfg, sc, residual, psd, n_ok, pu, pl);
    for (int64_t s = 0, c = 0; s < n_half; s++)
      if (ok[s]) lprop[s] = pl[c++];
    free(pu);
    free(pl);
    for (int b = 0; b < nb; b++)
      for (int t = 0; t < nt; t++)
        for (int i = 0; i < half; i++) {
          const int w = 2 * i + h;
          const int64_t s = ((int64_t)b * nt + t) * half + i;
          if (stall[b] >= sc->n_stall) continue;
          stats[0]++;
          if (!ok[s]) continue;
          const int64_t c = ((int64_t)b * nt + t) * nw + w;
          const uint64_t unit = ((uint64_t)b * nt + t) * nw + w;
          const double r_acc = rng_uniform(sc->seed, iter, MOVE_SEARCH, unit, 4 * (uint64_t)h + 2);
          if (log(r_acc) < betas[t] * (lprop[s] - logl[c]) + lz[s]) {
            for (int k = 0; k < 8; k++) u[8 * c + k] = prop[8 * s + k];
            logl[c] = lprop[s];
            stats[1]++;
          }
        }
  }
  /* temperature swaps per (band, walker), hottest pair first (eq. temp-orig) */
  for (int b = 0; b < nb; b++) {
    if (stall[b] >= sc->n_stall) continue;
    for (int w = 0; w < nw; w++)
      for (int t = nt - 1; t >= 1; t--) {
        stats[2]++;
        const double r = rng_uniform(sc->seed, iter, MOVE_SEARCH_PT, (uint64_t)b * nw + w, (uint64_t)t);
        const int64_t c1 = ((int64_t)b * nt + t) * nw + w, c0 = ((int64_t)b * nt + t - 1) * nw + w;
        if (log(r) < (betas[t - 1] - betas[t]) * (logl[c1] - logl[c0])) {
          for (int k = 0; k < 8; k++) {
            const double tmp = u[8 * c1 + k];
            u[8 * c1 + k] = u[8 * c0 + k];
            u[8 * c0 + k] = tmp;
          }
          const double tl = logl[c1];
          logl[c1] = logl[c0];
          logl[c0] = tl;
          stats[3]++;
        }
      }
  }
  /* best cold-chain point per band */
  for (int b = 0; b < nb; b++) {
    if (stall[b] >= sc->n_stall) continue;
    int wb = 0;
    for (int w = 1; w < nw; w++)
      if (logl[(int64_t)b * nt * nw + w] > logl[(int64_t)b * nt * nw + wb]) wb = w;
    const double m = logl[(int64_t)b * nt * nw + wb];
    if (m > best_logl[b]) {
      best_logl[b] = m;
      for (int k = 0; k < 8; k++) best_u[8 * b + k] = u[8 * ((int64_t)b * nt * nw + wb) + k];
      stall[b] = 0;
    } else {
      stall[b]++;
    }
  }
  free(prop);
  free(lprop);
  free(lz);
  free(ok);
  return 0;
}

/* Restart around the best points: every chain of band b moves to
 * best_u[b] + sigma * n (n standard normals by Box-Muller from the uniforms
 * of unit (b n_t + t) n_w + w, move 8, draws 0..7; coordinate k gets
 * sigma[k]; periodic coordinates wrapped, the others clamped into the box),
 * its logl is re-evaluated and the band's stall counter cleared (the best
 * point stays). */
#define MOVE_SEARCH_BALL 8
int gblo_search_ball(const gblo_config* cfg, const gblo_search_config* sc, int64_t iter, const double* sigma,
                     const double* residual, const double* psd, double* u, double* logl, const double* best_u,
                     int32_t* stall) {
  const int nb = sc->n_bands, nt = sc->n_temps, nw = sc->n_walkers;
  for (int b = 0; b < nb; b++) {
    double lo[8], hi[8];
    search_box(cfg, sc, b, lo, hi);
    for (int t = 0; t < nt; t++)
      for (int w = 0; w < nw; w++) {
        const uint64_t unit = ((uint64_t)b * nt + t) * nw + w;
        double* x = u + 8 * (((int64_t)b * nt + t) * nw + w);
        for (int p = 0; p < 4; p++) {
          const double u1 = rng_uniform(sc->seed, iter, MOVE_SEARCH_BALL, unit, 2 * (uint64_t)p);
          const double u2 = rng_uniform(sc->seed, iter, MOVE_SEARCH_BALL, unit, 2 * (uint64_t)p + 1);
          const double r = sqrt(-2.0 * log(u1));
          const double n0 = r * cos(2.0 * ORC_PI * u2), n1 = r * sin(2.0 * ORC_PI * u2);
          for (int q = 0; q < 2; q++) {
            const int k = 2 * p + q;
            double v = best_u[8 * b + k] + sigma[k] * (q ? n1 : n0);
            if (SEARCH_PERIOD[k] > 0) {
              v = wrap(v, SEARCH_PERIOD[k]);
            } else {
              /* f0 stays strictly inside [lo, hi) */
              const double top = k == 1 ? nextafter(hi[k], lo[k]) : hi[k];
              v = v < lo[k] ? lo[k] : (v > top ? top : v);
            }
            x[k] = v;
          }
        }
      }
    stall[b] = 0;
  }
  return gblo_search_eval(cfg, sc, residual, psd, u, logl);
}

/* ------------------------------------------------------------------------
 * Correlated A/E noise (Sec. 2: with unequal noise in the links the A and E
 * channels are no longer uncorrelated, and the likelihood needs the noise
 * matrix across channels).  Noise model: every link y_{s->r} carries its own
 * optical-metrology noise o_{sr} and the Doppler noises of the two test
 * masses it bounces off, delta_{rs} + D delta_{sr} (delta_{ab}: the test
 * mass on craft a facing craft b, D the one-arm delay exp(-i x),
 * x = 2 pi f L / c); the twelve noises are independent with the spectral
 * shapes of eq. psd: S_op = s_o^2 (2 pi f / c)^2 [1 + (2 mHz/f)^4] per link,
 * S_pm = s_a^2 (2 pi c f)^-2 [1 + (0.4 mHz/f)^2][1 + (f/8 mHz)^4] per test
 * mass.  The channels are the first-generation Michelson combinations
 * X = (1 - D^2)[(y_{1->0} + D y_{0->1}) - (y_{2->0} + D y_{0->2})] (and
 * cyclic), A = (Z - X)/sqrt 2, E = (X - 2Y + Z)/sqrt 6, so their noise
 * covariance is C = T diag(S_j) T^H with T the coefficients of the twelve
 * noises in (A, E).
 * levels[12]: s_o of the links 0->1, 0->2, 1->0, 1->2, 2->0, 2->1, then s_a
 * of the test masses (0,1), (0,2), (1,0), (1,2), (2,0), (2,1).
 * Output per bin: K = C^-1 as (K_AA, K_EE, Re K_AE, Im K_AE) and ln det C.
 * ------------------------------------------------------------------------ */
static int link_index(int s, int r) { /* (s -> r) in the order above */
  static const int tab[3][3] = {{-1, 0, 1}, {2, -1, 3}, {4, 5, -1}};
  return tab[s][r];
}

/* coefficients of the 12 noises in y_{s->r} */
static void link_noise(int s, int r, cplx D, cplx* coef /*[12]*/) {
  for (int j = 0; j < 12; j++) coef[j] = 0;
  coef[link_index(s, r)] += 1.0;           /* o_{sr} */
  coef[6 + link_index(r, s)] += 1.0;       /* delta_{rs} */
  coef[6 + link_index(s, r)] += D;         /* D delta_{sr} */
}

/* coefficients of the 12 noises in the Michelson combination at vertex v
 * with arms to b1 and b2 */
static void michelson_noise(int v, int b1, int b2, cplx D, cplx* coef) {
  cplx t1[12], t2[12], t3[12], t4[12];
  link_noise(b1, v, D, t1); /* y_{b1->v} */
  link_noise(v, b1, D, t2); /* y_{v->b1} */
  link_noise(b2, v, D, t3);
  link_noise(v, b2, D, t4);
  const cplx f = 1.0 - D * D;
  for (int j = 0; j < 12; j++) coef[j] = f * ((t1[j] + D * t2[j]) - (t3[j] + D * t4[j]));
}

void gblo_noise_matrix_value(const gblo_config* cfg, double f, const double* levels, double out[5]) {
  const double x = 2.0 * ORC_PI * f * cfg->L / ORC_C;
  const cplx D = cexp(-I * x);
  cplx X[12], Y[12], Z[12];
  michelson_noise(0, 1, 2, D, X);
  michelson_noise(1, 2, 0, D, Y);
  michelson_noise(2, 0, 1, D, Z);
  double S[12];
  for (int j = 0; j < 6; j++)
    S[j] = levels[j] * levels[j] * pow(2.0 * ORC_PI * f / ORC_C, 2.0) * (1.0 + pow(2e-3 / f, 4.0));
  for (int j = 6; j < 12; j++)
    S[j] = levels[j] * levels[j] * pow(2.0 * ORC_PI * ORC_C * f, -2.0) * (1.0 + pow(0.4e-3 / f, 2.0)) *
           (1.0 + pow(f / 8e-3, 4.0));
  double caa = 0, cee = 0;
  cplx cae = 0;
  for (int j = 0; j < 12; j++) {
    const cplx a = (Z[j] - X[j]) / sqrt(2.0);
    const cplx e = (X[j] - 2.0 * Y[j] + Z[j]) / sqrt(6.0);
    caa += creal(a * conj(a)) * S[j];
    cee += creal(e * conj(e)) * S[j];
    cae += a * conj(e) * S[j];
  }
  /* C = [[caa, cae], [conj(cae), cee]];  K = C^-1 = [[cee, -cae], [-conj(cae), caa]] / det */
  const double det = caa * cee - creal(cae * conj(cae));
  out[0] = cee / det;
  out[1] = caa / det;
  out[2] = -creal(cae) / det;
  out[3] = -cimag(cae) / det;
  out[4] = log(det);
}

int gblo_noise_matrix(const gblo_config* cfg, const double* levels, int64_t P, double* out /*[P][5][n_bins]*/) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
#pragma omp parallel for
  for (int64_t pi = 0; pi < P; pi++)
    for (int64_t i = 0; i < nb; i++) {
      double v[5];
      gblo_noise_matrix_value(cfg, (double)(k_min + i) / cfg->T, levels + 12 * pi, v);
      for (int c = 0; c < 5; c++) out[(pi * 5 + c) * nb + i] = v[c];
    }
  return 0;
}

/* 4 df Re sum_k a_k^H K_k b_k over the band for full-band series a, b [2][nb] */
static double matrix_inner(const gblo_config* cfg, int64_t nb, const cplx* a, const cplx* b, const double* K) {
  double s = 0;
  for (int64_t k = 0; k < nb; k++) {
    const cplx kae = K[2 * nb + k] + I * K[3 * nb + k];
    const cplx Kb0 = K[k] * b[k] + kae * b[nb + k];
    const cplx Kb1 = conj(kae) * b[k] + K[nb + k] * b[nb + k];
    s += creal(conj(a[k]) * Kb0 + conj(a[nb + k]) * Kb1);
  }
  return 4.0 / cfg->T * s;
}

/* eq. like with the channel matrix: -1/2 <R|R>_K - sum_k ln det C_k */
double gblo_loglike_matrix(const gblo_config* cfg, const double* R /*[2][nb][2]*/, const double* K /*[5][nb]*/) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  double ld = 0;
  for (int64_t k = 0; k < nb; k++) ld += K[4 * nb + k];
  return -0.5 * matrix_inner(cfg, nb, (const cplx*)R, (const cplx*)R, K) - ld;
}

/* eq. swapsource with the channel matrix:
 *   dlogl[b] = <R|a - r>_K - 1/2 <a - r|a - r>_K
 * with R = residual[res_idx[b]], K = Kmat[k_idx[b]] ([n_K][5][n_bins] as
 * gblo_noise_matrix writes it); templates clipped to the band. */
int gblo_delta_loglike_matrix(const gblo_config* cfg, const double* residual, int32_t n_res, const double* Kmat,
                              int32_t n_K, const double* params_old, const double* params_new, int32_t N,
                              const int32_t* res_idx, const int32_t* k_idx, int64_t B, double* dlogl) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  if (N < 2 || (N & (N - 1))) return -2;
  for (int64_t b = 0; b < B; b++)
    if (res_idx[b] < 0 || res_idx[b] >= n_res || k_idx[b] < 0 || k_idx[b] >= n_K) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < B; b++) {
    const double* po = params_old + 8 * b;
    const double* pn = params_new + 8 * b;
    if (!params_finite(cfg, po) || !params_finite(cfg, pn)) {
      dlogl[b] = NAN;
      continue;
    }
    /* d = a - r on the full band (plain, slow) */
    cplx* d = (cplx*)calloc((size_t)(2 * nb), sizeof(cplx));
    cplx* h = (cplx*)malloc(sizeof(cplx) * 2 * N);
    int64_t k0;
    waveform_one(cfg, pn, N, h, h + N, NULL, &k0);
    for (int c = 0; c < 2; c++)
      for (int j = 0; j < N; j++) {
        int64_t k = k0 + j;
        if (k >= k_min && k < k_min + nb) d[c * nb + (k - k_min)] += h[c * N + j];
      }
    waveform_one(cfg, po, N, h, h + N, NULL, &k0);
    for (int c = 0; c < 2; c++)
      for (int j = 0; j < N; j++) {
        int64_t k = k0 + j;
        if (k >= k_min && k < k_min + nb) d[c * nb + (k - k_min)] -= h[c * N + j];
      }
    const cplx* R = (const cplx*)(residual + (int64_t)res_idx[b] * 2 * nb * 2);
    const double* K = Kmat + (int64_t)k_idx[b] * 5 * nb;
    dlogl[b] = matrix_inner(cfg, nb, R, d, K) - 0.5 * matrix_inner(cfg, nb, d, d, K);
    free(d);
    free(h);
  }
  return 0;
}
