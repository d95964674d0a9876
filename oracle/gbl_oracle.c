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
 * four noise parameters of each set; noise [P][4], res_idx [P]. */
int gblo_psd_loglike(const gblo_config* cfg, const double* residual, int32_t n_res, const double* noise,
                     const int32_t* res_idx, int64_t P, double* logl) {
  int64_t k_min, nb;
  gblo_band(cfg, &k_min, &nb);
  for (int64_t pi = 0; pi < P; pi++)
    if (res_idx[pi] < 0 || res_idx[pi] >= n_res) return -1;
#pragma omp parallel for
  for (int64_t pi = 0; pi < P; pi++) {
    double* S = (double*)malloc(sizeof(double) * 2 * nb);
    gblo_psd_eval(cfg, noise + 4 * pi, 1, S);
    logl[pi] = gblo_loglike(cfg, residual + (int64_t)res_idx[pi] * 2 * nb * 2, S);
    free(S);
  }
  return 0;
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
