// gbl_device.hpp -- device building blocks of the GB template + likelihood path
// for CDNA4 (gfx950, wave64).
//
// One wavefront builds one template:
//   decode      parameters -> propagation direction, polarisation coefficients,
//               carrier bin q = floor(f0 T)                     (Sec. 2, D ~ 8)
//   slow part   the six heterodyned link envelopes at N midpoint samples and
//               their first-generation Michelson / AET combinations
//   FFT         length-N transform of 4 (A,E) or 6 (A,E,T) series in LDS
//   per bin     midpoint phase, the exact per-bin delay factors of TDI
// The physics is the rigid, equal-arm reading of the FastGB-style split the
// paper builds on (Sec. 2 "Input Template Models"; appendix "GB Waveform
// Generation"): y_{s->r}(t) = Re[exp(2 pi i q t/T) s_{s->r}(t)] with
//   s = -i G w exp(-i u) exp(i phi_r),  u = theta/2 = (1 - k.n) * amp,
//   amp = pi f_r L/c - pi fdot (L/c)^2 (1 - k.n)/2,  w = amp * sin(u)/u,
//   G = n^T H n,  phi_r = Phi(xi_r) - 2 pi q t/T,  xi_r = t - k.x_r/c.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbl {

constexpr double kC = 299792458.0;        // speed of light [m/s]
constexpr double kAU = 1.495978707e11;    // astronomical unit [m]
constexpr double kYear = 31557600.0;      // Julian year [s]: orbital period
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kSqrt3 = 1.73205080756887729353;
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt3 = 0.57735026918962576451;
constexpr double kInvSqrt6 = 0.40824829046386301637;

struct cd {
  double re, im;
};

__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cd mul_negi(cd a) { return {a.im, -a.re}; }  // -i a
__device__ __forceinline__ cd mul_posi(cd a) { return {-a.im, a.re}; }  // +i a

// Configuration-wide constants handed to every kernel by value.
struct Geo {
  double T;       // observation time [s]
  double L;       // arm length [m]
  double Lc;      // L / c [s]
  double inv_L;   // 1 / L
  double eh;      // e AU / 2 with e = L / (2 sqrt 3 AU)
  double ez;      // sqrt(3) e AU
  double df4;     // 4 / T  (4 Delta f of the inner product)
  int64_t k_min;  // first analysis bin
  int64_t n_bins; // number of analysis bins
};

// Tables for one template width N, built once per context.
struct WaveTables {
  const double* basis;  // [N][4] cos a, sin a, cos 2a, sin 2a at t_n = (n+1/2) T/N, a = 2 pi t/yr
  const cd* fft_tw;     // [N]    exp(-2 pi i m / N)
  const cd* bin_F;      // [N]    (1/2)(T/N) exp(-i pi k / N),   k = j - N/2
  const cd* bin_E;      // [N]    exp(-2 pi i k L / (c T)),      k = j - N/2
};

// ---------------------------------------------------------------------------
// exp(2 pi i c) for a phase c given in cycles.  The reduction is exact in
// binary floating point: r = c - rint(c) in [-1/2, 1/2], then the octant
// f = r - n/4 in [-1/8, 1/8]; x = 2 pi f in [-pi/4, pi/4] feeds Taylor
// polynomials (sin through x^15, cos through x^16; next terms < 5e-17) and
// the result is rotated by n quarter turns.
// ---------------------------------------------------------------------------
__device__ __forceinline__ cd expi_cycles(double c) {
  double r = c - rint(c);
  double n4 = rint(4.0 * r);
  double f = r - 0.25 * n4;
  double x = kTwoPi * f;
  double v = x * x;
  double sn = -1.0 / 1307674368000.0;  // -1/15!
  sn = sn * v + 1.0 / 6227020800.0;    // +1/13!
  sn = sn * v - 1.0 / 39916800.0;      // -1/11!
  sn = sn * v + 1.0 / 362880.0;        // +1/9!
  sn = sn * v - 1.0 / 5040.0;          // -1/7!
  sn = sn * v + 1.0 / 120.0;           // +1/5!
  sn = sn * v - 1.0 / 6.0;             // -1/3!
  sn = (sn * v) * x + x;
  double cs = 1.0 / 20922789888000.0;  // +1/16!
  cs = cs * v - 1.0 / 87178291200.0;   // -1/14!
  cs = cs * v + 1.0 / 479001600.0;     // +1/12!
  cs = cs * v - 1.0 / 3628800.0;       // -1/10!
  cs = cs * v + 1.0 / 40320.0;         // +1/8!
  cs = cs * v - 1.0 / 720.0;           // -1/6!
  cs = cs * v + 1.0 / 24.0;            // +1/4!
  cs = cs * v - 0.5;                   // -1/2!
  cs = cs * v + 1.0;
  int q = ((int)n4) & 3;
  double re = (q == 0) ? cs : (q == 1) ? -sn : (q == 2) ? -cs : sn;
  double im = (q == 0) ? sn : (q == 1) ? cs : (q == 2) ? -sn : -cs;
  return {re, im};
}

// ---------------------------------------------------------------------------
// Source decode (uniform across the wave)
// ---------------------------------------------------------------------------
struct Src {
  double f0, fdot, phi0_cyc, dfq;  // phi0 / (2 pi); dfq = f0 - q/T
  int64_t q;                   // carrier bin floor(f0 T)
  double kc[3];                // khat / c
  double kh[3];                // khat = -(sky direction)
  double pv[3], qv[3];         // polarisation basis vectors
  cd cp, cx;                   // n^T H n = cp (p.n^2 - q.n^2) + cx 2 (p.n)(q.n)
  cd eq;                       // exp(-2 pi i q L / (c T))
  int state;                   // 0 regular, 1 exactly zero amplitude, 2 non-finite parameters
};

__device__ __forceinline__ Src decode_source(const double* __restrict__ prm, const Geo& g) {
  Src s;
  double A = prm[0], f0 = prm[1], fdot = prm[2], phi0 = prm[3];
  double iota = prm[4], psi = prm[5], lam = prm[6], beta = prm[7];
  bool finite = isfinite(A) && isfinite(f0) && isfinite(fdot) && isfinite(phi0) && isfinite(iota) &&
                isfinite(psi) && isfinite(lam) && isfinite(beta) && fabs(f0 * g.T) < 4503599627370496.0;
  s.state = finite ? (A == 0.0 ? 1 : 0) : 2;
  if (!finite) {
    f0 = 0.0;  // keep the arithmetic below well defined
  }
  s.f0 = f0;
  s.fdot = fdot;
  s.phi0_cyc = phi0 / kTwoPi;
  double qd = floor(f0 * g.T);
  s.q = (int64_t)qd;
  s.dfq = f0 - qd / g.T;
  double sl, cl, sb, cb;
  sincos(lam, &sl, &cl);
  sincos(beta, &sb, &cb);
  s.kh[0] = -cb * cl;
  s.kh[1] = -cb * sl;
  s.kh[2] = -sb;
  for (int i = 0; i < 3; i++) s.kc[i] = s.kh[i] / kC;
  s.pv[0] = sl;
  s.pv[1] = -cl;
  s.pv[2] = 0.0;
  s.qv[0] = -sb * cl;
  s.qv[1] = -sb * sl;
  s.qv[2] = cb;
  double ci = cos(iota);
  double s2p, c2p;
  sincos(2.0 * psi, &s2p, &c2p);
  double ap = A * (1.0 + ci * ci);
  double ax = 2.0 * A * ci;
  s.cp = {ap * c2p, -ax * s2p};
  s.cx = {ap * s2p, ax * c2p};
  s.eq = expi_cycles(-qd * g.Lc / g.T);
  return s;
}

// ---------------------------------------------------------------------------
// sin(u)/u and cos(u) for the link phase u = theta/2 in [0, ~1.6] (f < 30 mHz):
// Taylor series in v = u^2 evaluated by Horner's rule, truncated where the
// next term is below 2e-17 for |u| <= 2.7 (f up to ~51 mHz).  Larger |u|
// (far outside the analysis band) falls back to the library sincos.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sinc_cos(double u, double& sinc, double& cosu) {
  double v = u * u;
  if (v <= 7.29) {
    double s = 1.0 / 15511210043330985984000000.0;   // +1/25!
    s = s * v - 1.0 / 25852016738884976640000.0;     // -1/23!
    s = s * v + 1.0 / 51090942171709440000.0;        // +1/21!
    s = s * v - 1.0 / 121645100408832000.0;          // -1/19!
    s = s * v + 1.0 / 355687428096000.0;             // +1/17!
    s = s * v - 1.0 / 1307674368000.0;               // -1/15!
    s = s * v + 1.0 / 6227020800.0;                  // +1/13!
    s = s * v - 1.0 / 39916800.0;                    // -1/11!
    s = s * v + 1.0 / 362880.0;                      // +1/9!
    s = s * v - 1.0 / 5040.0;                        // -1/7!
    s = s * v + 1.0 / 120.0;                         // +1/5!
    s = s * v - 1.0 / 6.0;                           // -1/3!
    s = s * v + 1.0;
    double c = -1.0 / 403291461126605635584000000.0;  // -1/26!
    c = c * v + 1.0 / 620448401733239439360000.0;     // +1/24!
    c = c * v - 1.0 / 1124000727777607680000.0;       // -1/22!
    c = c * v + 1.0 / 2432902008176640000.0;          // +1/20!
    c = c * v - 1.0 / 6402373705728000.0;             // -1/18!
    c = c * v + 1.0 / 20922789888000.0;               // +1/16!
    c = c * v - 1.0 / 87178291200.0;                  // -1/14!
    c = c * v + 1.0 / 479001600.0;                    // +1/12!
    c = c * v - 1.0 / 3628800.0;                      // -1/10!
    c = c * v + 1.0 / 40320.0;                        // +1/8!
    c = c * v - 1.0 / 720.0;                          // -1/6!
    c = c * v + 1.0 / 24.0;                           // +1/4!
    c = c * v - 0.5;                                  // -1/2!
    c = c * v + 1.0;
    sinc = s;
    cosu = c;
  } else {
    double su, cu;
    sincos(u, &su, &cu);
    sinc = su / u;
    cosu = cu;
  }
}

// ---------------------------------------------------------------------------
// Slow part: the A, E (and T) TDI pieces U, V at one midpoint sample.
// Spacecraft i = 0, 1, 2 sit at orientation angle 2 pi i/3 of the rigid
// equal-arm orbit; arm m joins craft m -> (m+1) mod 3.
// out[0..5] = U_A, V_A, U_E, V_E, U_T, V_T  (T only when NS == 6).
// ---------------------------------------------------------------------------
template <int NS>
__device__ __forceinline__ void slow_sample(const Src& s, const Geo& g, const double* __restrict__ basis, int n,
                                            double t, cd* out) {
  // orientation cosines/sines of the three craft
  constexpr double cbs[3] = {1.0, -0.5, -0.5};
  constexpr double sbs[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
  const double ca = basis[4 * n + 0], sa = basis[4 * n + 1];
  const double c2a = basis[4 * n + 2], s2a = basis[4 * n + 3];

  // receiver phases exp(i phi_r), instantaneous frequencies f_r
  // phases in cycles: phi_r / (2 pi) = phi0/(2 pi) + dfq t + fdot t^2/2
  //                                    - (f0 + fdot t) k.x_r/c + fdot (k.x_r/c)^2 / 2
  cd P[3];
  double fr[3];
  double base = s.phi0_cyc + s.dfq * t + 0.5 * s.fdot * t * t;
  double fwd = s.f0 + s.fdot * t;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    double x = kAU * ca + g.eh * (c2a * cbs[i] + s2a * sbs[i] - 3.0 * cbs[i]);
    double y = kAU * sa + g.eh * (s2a * cbs[i] - c2a * sbs[i] - 3.0 * sbs[i]);
    double z = -g.ez * (ca * cbs[i] + sa * sbs[i]);
    double kx = s.kc[0] * x + s.kc[1] * y + s.kc[2] * z;  // k.x_i / c
    P[i] = expi_cycles(base - fwd * kx + 0.5 * s.fdot * kx * kx);
    fr[i] = s.f0 + s.fdot * (t - kx);
  }

  // arm projections: k.n, G = n^T H n for arm m (craft m -> m+1)
  double kn[3];
  cd G[3];
#pragma unroll
  for (int m = 0; m < 3; m++) {
    const int j = (m + 1) % 3;
    double dcb = cbs[j] - cbs[m], dsb = sbs[j] - sbs[m];
    double nx = g.inv_L * g.eh * (c2a * dcb + s2a * dsb - 3.0 * dcb);
    double ny = g.inv_L * g.eh * (s2a * dcb - c2a * dsb - 3.0 * dsb);
    double nz = -g.inv_L * g.ez * (ca * dcb + sa * dsb);
    kn[m] = s.kh[0] * nx + s.kh[1] * ny + s.kh[2] * nz;
    double pn = s.pv[0] * nx + s.pv[1] * ny;  // p has no z component
    double qn = s.qv[0] * nx + s.qv[1] * ny + s.qv[2] * nz;
    double ep = pn * pn - qn * qn;
    double ex = 2.0 * pn * qn;
    G[m] = {s.cp.re * ep + s.cx.re * ex, s.cp.im * ep + s.cx.im * ex};
  }

  // link envelope s_{snd->rcv}: arm m traversed forward (sign +1) or backward
  auto link = [&](int m, double sgn, int rcv) -> cd {
    double om = 1.0 - sgn * kn[m];
    double amp = kPi * fr[rcv] * g.Lc - 0.5 * kPi * s.fdot * g.Lc * g.Lc * om;
    double u = om * amp;
    double sc, cu;
    sinc_cos(u, sc, cu);
    double w = amp * sc;
    cd z = {cu, -u * sc};  // exp(-i u)
    cd t1 = z * P[rcv];
    cd t2 = G[m] * t1;
    return mul_negi(w * t2);
  };
  cd l12 = link(0, 1.0, 1), l21 = link(0, -1.0, 0);
  cd l23 = link(1, 1.0, 2), l32 = link(1, -1.0, 1);
  cd l31 = link(2, 1.0, 0), l13 = link(2, -1.0, 2);

  cd UX = l21 - l31, VX = l12 - l13;
  cd UY = l32 - l12, VY = l23 - l21;
  cd UZ = l13 - l23, VZ = l31 - l32;
  out[0] = kInvSqrt2 * (UZ - UX);
  out[1] = kInvSqrt2 * (VZ - VX);
  out[2] = kInvSqrt6 * (UX - 2.0 * UY + UZ);
  out[3] = kInvSqrt6 * (VX - 2.0 * VY + VZ);
  if constexpr (NS == 6) {
    out[4] = kInvSqrt3 * (UX + UY + UZ);
    out[5] = kInvSqrt3 * (VX + VY + VZ);
  }
}

// ---------------------------------------------------------------------------
// Small in-register DFTs (forward sign), natural-order output.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dft2(cd* x) {
  cd a = x[0], b = x[1];
  x[0] = a + b;
  x[1] = a - b;
}

template <int S = 1>
__device__ __forceinline__ void dft4s(cd* x) {
  // elements x[0], x[S], x[2S], x[3S]
  cd a0 = x[0], a1 = x[S], a2 = x[2 * S], a3 = x[3 * S];
  cd t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
  x[0] = t0 + t2;
  x[2 * S] = t0 - t2;
  x[S] = t1 + mul_negi(t3);
  x[3 * S] = t1 + mul_posi(t3);
}

__device__ __forceinline__ void dft4(cd* x) { dft4s<1>(x); }

// exp(-2 pi i m / 16), m = 0..15
__device__ __forceinline__ cd w16(int m) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
  constexpr double re[16] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1};
  constexpr double im[16] = {0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1, 1, c1, h, s1};
  return {re[m & 15], im[m & 15]};
}

__device__ __forceinline__ void dft8(cd* x) {
  // 8 = 4 x 2: n = n2 + 2 n1; X[k1 + 4 k2]
  cd y0[4] = {x[0], x[2], x[4], x[6]};
  cd y1[4] = {x[1], x[3], x[5], x[7]};
  dft4(y0);
  dft4(y1);
#pragma unroll
  for (int k1 = 1; k1 < 4; k1++) y1[k1] = y1[k1] * w16(2 * k1);
#pragma unroll
  for (int k1 = 0; k1 < 4; k1++) {
    x[k1] = y0[k1] + y1[k1];
    x[k1 + 4] = y0[k1] - y1[k1];
  }
}

__device__ __forceinline__ void dft16(cd* x) {
  // 16 = 4 x 4: n = n2 + 4 n1; X[k1 + 4 k2]
  cd y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; n2++) {
#pragma unroll
    for (int n1 = 0; n1 < 4; n1++) y[n2][n1] = x[n2 + 4 * n1];
    dft4(y[n2]);
#pragma unroll
    for (int k1 = 1; k1 < 4; k1++)
      if (n2 > 0) y[n2][k1] = y[n2][k1] * w16(n2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; k1++) {
    cd z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4(z);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++) x[k1 + 4 * k2] = z[k2];
  }
}

template <int R>
__device__ __forceinline__ void dft_small(cd* x) {
  if constexpr (R == 2) dft2(x);
  if constexpr (R == 4) dft4(x);
  if constexpr (R == 8) dft8(x);
  if constexpr (R == 16) dft16(x);
}

// ---------------------------------------------------------------------------
// Wave-level in-place decimation-in-frequency FFT over NSER series of length N
// stored in LDS with one padding element per 16 (bank-conflict avoidance).
// Radix plan: 128 = 16x8, 256 = 16x16, 512 = 16x16x2, 1024 = 16x16x4.
// Output X[k] sits at the digit-reversed position fft_pos<N>(k).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

template <int N>
struct FftPlan;
template <>
struct FftPlan<128> {
  static constexpr int R1 = 16, R2 = 8, R3 = 1;
};
template <>
struct FftPlan<256> {
  static constexpr int R1 = 16, R2 = 16, R3 = 1;
};
template <>
struct FftPlan<512> {
  static constexpr int R1 = 16, R2 = 16, R3 = 2;
};
template <>
struct FftPlan<1024> {
  static constexpr int R1 = 16, R2 = 16, R3 = 4;
};

template <int N>
constexpr int series_pitch() {
  return N + N / 16;
}

template <int N>
__device__ __forceinline__ int fft_pos(int k) {
  using P = FftPlan<N>;
  int k1 = k % P::R1;
  int r = k / P::R1;
  int k2 = r % P::R2;
  int k3 = r / P::R2;
  return k1 * (N / P::R1) + k2 * (N / (P::R1 * P::R2)) + k3;
}

template <int N, int R, int ST, int NSER>
__device__ __forceinline__ void fft_pass(cd* buf, const cd* __restrict__ tw, int lane) {
  constexpr int NB = N / R;  // butterflies per series
  constexpr int SP = series_pitch<N>();
  constexpr int TWS = N / (R * ST);
  for (int item = lane; item < NSER * NB; item += 64) {
    int sidx = item / NB, beta = item % NB;
    int grp = beta / ST, i = beta % ST;
    int base = grp * R * ST + i;
    cd* b = buf + sidx * SP;
    cd x[R];
#pragma unroll
    for (int r = 0; r < R; r++) x[r] = b[lds_pad(base + ST * r)];
    dft_small<R>(x);
    if constexpr (ST > 1) {
#pragma unroll
      for (int r = 1; r < R; r++) x[r] = x[r] * tw[TWS * i * r];
    }
#pragma unroll
    for (int r = 0; r < R; r++) b[lds_pad(base + ST * r)] = x[r];
  }
}

template <int N, int NSER>
__device__ __forceinline__ void wave_fft(cd* buf, const cd* __restrict__ tw, int lane) {
  using P = FftPlan<N>;
  fft_pass<N, P::R1, N / P::R1, NSER>(buf, tw, lane);
  __syncthreads();
  fft_pass<N, P::R2, N / (P::R1 * P::R2), NSER>(buf, tw, lane);
  __syncthreads();
  if constexpr (P::R3 > 1) {
    fft_pass<N, P::R3, 1, NSER>(buf, tw, lane);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One template: slow part -> FFT -> per-bin TDI factors.  On return, for the
// bins j = lane + 64 m (m < N/64) the lane may read channel c's spectrum with
// bin_value(); the LDS workspace is left holding the transformed series.
// ---------------------------------------------------------------------------
template <int N, int NSER>
__device__ __forceinline__ void template_transform(const Src& s, const Geo& g, const WaveTables& tb, cd* buf,
                                                   int lane) {
  constexpr int SP = series_pitch<N>();
#pragma unroll 1
  for (int n = lane; n < N; n += 64) {
    double t = ((double)n + 0.5) * g.T / (double)N;
    cd v[6];
    slow_sample<NSER>(s, g, tb.basis, n, t, v);
#pragma unroll
    for (int c = 0; c < NSER; c++) buf[c * SP + lds_pad(n)] = v[c];
  }
  __syncthreads();
  wave_fft<N, NSER>(buf, tb.fft_tw, lane);
}

// Spectrum of channel c (0 = A, 1 = E, 2 = T) at window bin j, from the
// transformed U/V series in LDS: C = (1 - D^2) F (U + D V), D = exp(-i x),
// x = 2 pi (q + k) L/(c T), F = (1/2)(T/N) exp(-i pi k/N), k = j - N/2.
template <int N>
__device__ __forceinline__ cd bin_value(const Src& s, const WaveTables& tb, const cd* buf, int c, int j) {
  constexpr int SP = series_pitch<N>();
  int kk = (j + N / 2) & (N - 1);
  int pos = lds_pad(fft_pos<N>(kk));
  cd U = buf[(2 * c) * SP + pos];
  cd V = buf[(2 * c + 1) * SP + pos];
  cd D = s.eq * tb.bin_E[j];
  cd D2 = D * D;
  cd one_m = {1.0 - D2.re, -D2.im};
  return one_m * (tb.bin_F[j] * (U + D * V));
}

}  // namespace gbl
