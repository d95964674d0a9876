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

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbl {

constexpr int kWave = 64;                // wavefront width of CDNA
constexpr double kC = 299792458.0;        // speed of light [m/s]
constexpr double kAU = 1.495978707e11;    // astronomical unit [m]
constexpr double kYear = 31557600.0;      // Julian year [s]: orbital period
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kSqrt3 = 1.73205080756887729353;
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt3 = 0.57735026918962576451;
constexpr double kInvSqrt6 = 0.40824829046386301637;

// Complex numbers in the response precision F (double, or float in the mixed
// mode).  Phases, their reduction and every likelihood sum stay in double.
// Aligned to their size, so that a value moves in one 16-byte (8-byte) LDS
// access: the LDS layouts are laid out against bank conflicts of whole-value
// accesses, and a value split into two 8-byte halves would conflict.
template <typename F>
struct alignas(2 * sizeof(F)) cx {
  F re, im;
};
using cd = cx<double>;
using cf = cx<float>;

template <typename F>
__device__ __forceinline__ cx<F> operator+(cx<F> a, cx<F> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename F>
__device__ __forceinline__ cx<F> operator-(cx<F> a, cx<F> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename F>
__device__ __forceinline__ cx<F> operator*(cx<F> a, cx<F> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename F>
__device__ __forceinline__ cx<F> operator*(F s, cx<F> a) {
  return {s * a.re, s * a.im};
}
template <typename F>
__device__ __forceinline__ cx<F> mul_negi(cx<F> a) {
  return {a.im, -a.re};
}  // -i a
template <typename F>
__device__ __forceinline__ cx<F> mul_posi(cx<F> a) {
  return {-a.im, a.re};
}  // +i a
template <typename F, typename G>
__device__ __forceinline__ cx<F> cvt(cx<G> a) {
  return {(F)a.re, (F)a.im};
}
// a complex value of a decoded source read field by field (the source may sit
// in the constant address space, which the copy constructor cannot bind)
template <typename F, typename C>
__device__ __forceinline__ cx<F> load_cx(const C& c) {
  return {(F)c.re, (F)c.im};
}

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

// Tables for one template width N, built once per context (the complex
// tables exist in both precisions; the orbit basis is always double).
template <typename F>
struct WaveTables {
  const double* basis;  // [N][4] cos a, sin a, cos 2a, sin 2a at t_n = (n+1/2) T/N, a = 2 pi t/yr
  const cx<F>* fft_tw;  // [N]    exp(-2 pi i m / N)
  const cx<F>* bin_F;   // [N]    (1/2)(T/N) exp(-i pi k / N),   k = j - N/2
  const cx<F>* bin_W;   // [N]    exp(-2 pi i k L/(c T)):  the bin's TDI delay factor over the carrier's
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
struct alignas(16) Src {
  double f0, fdot, phi0_cyc, dfq;  // phi0 / (2 pi); dfq = f0 - q/T
  int64_t q;                   // carrier bin floor(f0 T)
  // The orbit enters through the four basis values b = (cos a, sin a, cos 2a,
  // sin 2a) of the orientation angle a, and every projection the response
  // needs is an affine function of b whose coefficients depend on the source
  // alone: v = c[0] cos a + c[1] sin a + c[2] cos 2a + c[3] sin 2a + c[4].
  double xr[3][5];             // k.x_r / c of receivers (craft) r = 0, 1, 2 [s]
  double kn[2][5], qn[2][5];   // k.n_m and q.n_m of arms m = 0, 1
  double pn[2][3];             // p.n_m (cos 2a, sin 2a, 1: p has no z component)
  cd cp, cx2;                  // n^T H n = cp (p.n^2 - q.n^2) + cx2 (p.n)(q.n)
  cd dq;                       // exp(-2 pi i q L/(c T)): the carrier's TDI delay factor
  int state;                   // 0 regular, 1 exactly zero amplitude, 2 non-finite parameters
};

// Validity and carrier bin only (cheap; used before the full decode).
// state: 0 regular, 1 exactly zero amplitude, 2 undefined (non-finite or |f0 T| >= 2^52)
struct SrcHead {
  int state;
  int64_t q;
};

__device__ __forceinline__ SrcHead source_head(const double* __restrict__ prm, const Geo& g) {
  bool finite = true;
#pragma unroll
  for (int i = 0; i < 8; i++) finite = finite && isfinite(prm[i]);
  double f0T = prm[1] * g.T;
  finite = finite && fabs(f0T) < 4503599627370496.0;
  SrcHead h;
  h.state = finite ? (prm[0] == 0.0 ? 1 : 0) : 2;
  h.q = finite ? (int64_t)floor(f0T) : 0;
  return h;
}

// Source decode from the parameters (A, f0, fdot, phi0, iota, psi, lambda,
// beta) and the sines and cosines of lambda, beta, iota and 2 psi, in three
// groups of outputs: a = 0..2 the k.x_r/c coefficients of receiver r = a,
// a = 3..8 the arm m = (a-3)/3 projection coefficients of k, q or p, a = 9
// carrier bin, phases, polarisation amplitudes, delay factor and state.
struct SrcTrig {
  double sl, cl, sb, cb, ci, s2p, c2p;
};

__device__ __forceinline__ void decode_group(int a, const double* __restrict__ prm, const SrcTrig& tr,
                                             const Geo& g, Src& s) {
  // propagation direction k = -(sky direction) and polarisation basis p, q
  const double kh[3] = {-tr.cb * tr.cl, -tr.cb * tr.sl, -tr.sb};
  const double pv[2] = {tr.sl, -tr.cl};
  const double qv[3] = {-tr.sb * tr.cl, -tr.sb * tr.sl, tr.cb};
  constexpr double cbs[3] = {1.0, -0.5, -0.5};
  constexpr double sbs[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
  if (a < 3) {
    // craft r at orientation 2 pi r/3 (cos/sin br):
    //   x_r = AU (cos a, sin a, 0) + eh (cos 2a cbr + sin 2a sbr - 3 cbr,
    //         sin 2a cbr - cos 2a sbr - 3 sbr, 0) - ez (0, 0, cos a cbr + sin a sbr)
    const int r = a;
    const double cbr = r == 0 ? cbs[0] : r == 1 ? cbs[1] : cbs[2];
    const double sbr = r == 0 ? sbs[0] : r == 1 ? sbs[1] : sbs[2];
    const double kc[3] = {kh[0] / kC, kh[1] / kC, kh[2] / kC};
    double* c = s.xr[r];
    c[0] = kc[0] * kAU - kc[2] * g.ez * cbr;
    c[1] = kc[1] * kAU - kc[2] * g.ez * sbr;
    c[2] = g.eh * (kc[0] * cbr - kc[1] * sbr);
    c[3] = g.eh * (kc[0] * sbr + kc[1] * cbr);
    c[4] = -3.0 * g.eh * (kc[0] * cbr + kc[1] * sbr);
  } else if (a < 9) {
    // arm m = craft m -> m+1: n_m = (x_{m+1} - x_m) / L; projection of v = k, q or p
    const int m = (a - 3) / 3, w = (a - 3) % 3;
    const double dcb = m == 0 ? cbs[1] - cbs[0] : cbs[2] - cbs[1];
    const double dsb = m == 0 ? sbs[1] - sbs[0] : sbs[2] - sbs[1];
    const double v0 = w == 0 ? kh[0] : w == 1 ? qv[0] : pv[0];
    const double v1 = w == 0 ? kh[1] : w == 1 ? qv[1] : pv[1];
    const double v2 = w == 0 ? kh[2] : w == 1 ? qv[2] : 0.0;
    const double sh = g.inv_L * g.eh, sz = g.inv_L * g.ez;
    const double c2 = sh * (v0 * dcb - v1 * dsb);
    const double c3 = sh * (v0 * dsb + v1 * dcb);
    const double c4 = -3.0 * sh * (v0 * dcb + v1 * dsb);
    if (w == 2) {
      s.pn[m][0] = c2;
      s.pn[m][1] = c3;
      s.pn[m][2] = c4;
    } else {
      double* c = w == 0 ? s.kn[m] : s.qn[m];
      c[0] = -sz * v2 * dcb;
      c[1] = -sz * v2 * dsb;
      c[2] = c2;
      c[3] = c3;
      c[4] = c4;
    }
  } else if (a == 9) {
    double A = prm[0], f0 = prm[1], fdot = prm[2], phi0 = prm[3];
    bool finite = isfinite(A) && isfinite(f0) && isfinite(fdot) && isfinite(phi0) && isfinite(prm[4]) &&
                  isfinite(prm[5]) && isfinite(prm[6]) && isfinite(prm[7]) && fabs(f0 * g.T) < 4503599627370496.0;
    s.state = finite ? (A == 0.0 ? 1 : 0) : 2;
    if (!finite) f0 = 0.0;  // keep the arithmetic below well defined
    s.f0 = f0;
    s.fdot = fdot;
    s.phi0_cyc = phi0 / kTwoPi;
    const double qd = floor(f0 * g.T);
    s.q = (int64_t)qd;
    s.dfq = f0 - qd / g.T;
    const double ap = A * (1.0 + tr.ci * tr.ci);
    const double ax = 2.0 * A * tr.ci;
    s.cp = {ap * tr.c2p, -ax * tr.s2p};
    s.cx2 = {2.0 * ap * tr.s2p, 2.0 * ax * tr.c2p};
    s.dq = expi_cycles(-(double)s.q * (g.Lc / g.T));
  }
}

// the angle whose sine and cosine slot a = 0..3 of SrcTrig needs
__device__ __forceinline__ double decode_angle(int a, const double* __restrict__ prm) {
  return a == 0 ? prm[6] : a == 1 ? prm[7] : a == 2 ? prm[4] : 2.0 * prm[5];
}

// Full decode of NSRC (1 or 2) sources by one whole wave (every lane must
// take part) into LDS, spread over the lanes so that the wave issues about one
// trigonometric evaluation and one group of outputs instead of all of them:
// lanes 32 t + a of source t evaluate the sine and cosine of angle a = 0..3
// (then shared by shuffles) and write output group a = 0..9.
template <int NSRC>
__device__ __forceinline__ void decode_sources(const double* __restrict__ p0, const double* __restrict__ p1,
                                               const Geo& g, Src* out) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int t = (lane >> 5) < NSRC ? (lane >> 5) : 0;
  const int role = lane & 31;
  const bool writer = (lane >> 5) < NSRC;
  const double* prm = t ? p1 : p0;
  double sv = 0.0, cv = 1.0;
  if (role < 4) sincos(decode_angle(role, prm), &sv, &cv);
  const int l0 = t << 5;
  SrcTrig tr;
  tr.sl = __shfl(sv, l0 + 0);
  tr.cl = __shfl(cv, l0 + 0);
  tr.sb = __shfl(sv, l0 + 1);
  tr.cb = __shfl(cv, l0 + 1);
  tr.ci = __shfl(cv, l0 + 2);
  tr.s2p = __shfl(sv, l0 + 3);
  tr.c2p = __shfl(cv, l0 + 3);
  if (writer && role < 10) decode_group(role, prm, tr, g, out[t]);
}

// The same decode by one thread (all groups in turn), for the decode pass
// that runs one thread per template.
__device__ __forceinline__ void decode_source(const double* __restrict__ prm, const Geo& g, Src& out) {
  SrcTrig tr;
  sincos(decode_angle(0, prm), &tr.sl, &tr.cl);
  sincos(decode_angle(1, prm), &tr.sb, &tr.cb);
  double si;
  sincos(decode_angle(2, prm), &si, &tr.ci);
  sincos(decode_angle(3, prm), &tr.s2p, &tr.c2p);
  for (int a = 0; a < 10; a++) decode_group(a, prm, tr, g, out);
}

// ---------------------------------------------------------------------------
// sin(u)/u and cos(u) for the link phase u = theta/2, which stays below 1.6
// for every frequency in the analysis band (u < pi f (2L/c)): Taylor series in
// v = u^2 by Horner's rule, truncated where the next term is below 5e-18 for
// |u| <= 1.7 (f up to ~32 mHz).  Larger |u| (sources far above the band)
// falls back to the library sincos.  Not inlined: the lockstep version below
// calls it only for sources far above the band, and its constants would
// otherwise be materialised (or hoisted out of loops) in every caller.
// ---------------------------------------------------------------------------
__device__ __noinline__ void sinc_cos(double u, double& sinc, double& cosu) {
  double v = u * u;
  if (v <= 2.89) {
    double s = -1.0 / 51090942171709440000.0;   // -1/21!
    s = s * v + 1.0 / 121645100408832000.0;     // +1/19!
    s = s * v - 1.0 / 355687428096000.0;        // -1/17!
    s = s * v + 1.0 / 1307674368000.0;          // +1/15!
    s = s * v - 1.0 / 6227020800.0;             // -1/13!
    s = s * v + 1.0 / 39916800.0;               // +1/11!
    s = s * v - 1.0 / 362880.0;                 // -1/9!
    s = s * v + 1.0 / 5040.0;                   // +1/7!
    s = s * v - 1.0 / 120.0;                    // -1/5!
    s = s * v + 1.0 / 6.0;                      // +1/3!
    s = 1.0 - s * v;
    double c = 1.0 / 620448401733239439360000.0;  // +1/24!
    c = c * v - 1.0 / 1124000727777607680000.0;   // -1/22!
    c = c * v + 1.0 / 2432902008176640000.0;      // +1/20!
    c = c * v - 1.0 / 6402373705728000.0;         // -1/18!
    c = c * v + 1.0 / 20922789888000.0;           // +1/16!
    c = c * v - 1.0 / 87178291200.0;              // -1/14!
    c = c * v + 1.0 / 479001600.0;                // +1/12!
    c = c * v - 1.0 / 3628800.0;                  // -1/10!
    c = c * v + 1.0 / 40320.0;                    // +1/8!
    c = c * v - 1.0 / 720.0;                      // -1/6!
    c = c * v + 1.0 / 24.0;                       // +1/4!
    c = c * v - 0.5;                              // -1/2!
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

// FP64 coefficients of the Taylor series below (1/n! with alternating signs),
// kept in the constant address space and read through a pointer that an empty
// asm statement makes opaque at every use.  The Horner steps then take them
// from scalar registers (scalar loads, hits in the scalar cache): gfx9-class
// VALU encodings take no 64-bit literal, so a coefficient written in the code
// costs two vector moves per use, or a pair of vector registers held for the
// whole kernel when the compiler hoists it out of a loop.
struct PolyTable {
  double sinc[10];  // sin(u)/u:  -1/21!, +1/19!, ..., +1/3!  (Horner order, v = u^2)
  double cosu[13];  // cos(u):    +1/24!, -1/22!, ..., -1/2!, 1
  double osin[7];   // octant sin(x)/x - 1 over x^2: -1/15!, ..., -1/3!
  double ocos[9];   // octant cos(x): +1/16!, ..., -1/2!, 1
};

__constant__ PolyTable kPolyTable = {
    {-1.0 / 51090942171709440000.0, 1.0 / 121645100408832000.0, -1.0 / 355687428096000.0, 1.0 / 1307674368000.0,
     -1.0 / 6227020800.0, 1.0 / 39916800.0, -1.0 / 362880.0, 1.0 / 5040.0, -1.0 / 120.0, 1.0 / 6.0},
    {1.0 / 620448401733239439360000.0, -1.0 / 1124000727777607680000.0, 1.0 / 2432902008176640000.0,
     -1.0 / 6402373705728000.0, 1.0 / 20922789888000.0, -1.0 / 87178291200.0, 1.0 / 479001600.0,
     -1.0 / 3628800.0, 1.0 / 40320.0, -1.0 / 720.0, 1.0 / 24.0, -0.5, 1.0},
    {-1.0 / 1307674368000.0, 1.0 / 6227020800.0, -1.0 / 39916800.0, 1.0 / 362880.0, -1.0 / 5040.0, 1.0 / 120.0,
     -1.0 / 6.0},
    {1.0 / 20922789888000.0, -1.0 / 87178291200.0, 1.0 / 479001600.0, -1.0 / 3628800.0, 1.0 / 40320.0,
     -1.0 / 720.0, 1.0 / 24.0, -0.5, 1.0}};

using CPoly = const __attribute__((address_space(4))) PolyTable;

// One Horner step a v + c with the coefficient c in a scalar register pair,
// as the three-operand FMA that reads it there.  Written out because the
// compiler otherwise picks the two-operand form, whose addend is also its
// destination: two vector moves copy the coefficient in before every step
// of every lane's polynomial.  The rounding is that of fma(a, v, c).
__device__ __forceinline__ double fma_sc(double a, double v, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(v), "s"(c));
  return r;
}

__device__ __forceinline__ CPoly* poly_table() {
  CPoly* p = (CPoly*)&kPolyTable;
  asm volatile("" : "+s"(p));
  return p;
}

// The same Taylor polynomials evaluated for K arguments in lockstep, each
// coefficient read once per step and reused K times.  The float versions
// (mixed precision) use the shortest truncations whose next term is below
// 2.5e-10 on the same ranges.
// UC = 1: any |u| in band (above, with the library fallback); UC = 0: the
// caller guarantees |u| <= 0.25 (templates below ~4.7 mHz), where sinc through
// u^10 and cos through u^12 leave next terms below 1e-17 (u^12/13!, u^14/14!).
// check = false: the caller guarantees |u| < 1.7 for every lane (no range
// test; the result is the same, as the fallback would not be taken).
template <int K, int UC = 1>
__device__ __forceinline__ void sinc_cos_k(const double* u, double* sinc, double* cosu, bool check = true) {
  CPoly* const tp = poly_table();
  const auto& cs_ = tp->sinc;
  const auto& cc_ = tp->cosu;
  constexpr int S0 = UC == 0 ? 5 : 0;  // first sinc coefficient used
  constexpr int C0 = UC == 0 ? 6 : 0;  // first cos coefficient used
  double v[K], a[K], c[K];
#pragma unroll
  for (int i = 0; i < K; i++) {
    v[i] = u[i] * u[i];
    a[i] = cs_[S0];
    c[i] = cc_[C0];
  }
#pragma unroll
  for (int k = S0 + 1; k < 10; k++) {
#pragma unroll
    for (int i = 0; i < K; i++) a[i] = fma_sc(a[i], v[i], cs_[k]);
  }
#pragma unroll
  for (int k = C0 + 1; k < 13; k++) {
#pragma unroll
    for (int i = 0; i < K; i++) c[i] = fma_sc(c[i], v[i], cc_[k]);
  }
#pragma unroll
  for (int i = 0; i < K; i++) {
    sinc[i] = 1.0 - a[i] * v[i];
    cosu[i] = c[i];
  }
  if (UC != 0 && check) {
    bool in_range = true;
#pragma unroll
    for (int i = 0; i < K; i++) in_range = in_range && (v[i] <= 2.89);
    if (!in_range) {
      // sources far above the band: exact library evaluation
#pragma unroll
      for (int i = 0; i < K; i++) sinc_cos(u[i], sinc[i], cosu[i]);
    }
  }
}

template <int K, int UC = 1>
__device__ __forceinline__ void sinc_cos_k(const float* u, float* sinc, float* cosu, bool check = true) {
  // sinc through u^14 (next 1.7^16/17! < 1.4e-11), cos through u^14 (next < 2.3e-10)
  constexpr float cs_[7] = {-1.0f / 1307674368000.0f, 1.0f / 6227020800.0f, -1.0f / 39916800.0f,
                            1.0f / 362880.0f,         -1.0f / 5040.0f,      1.0f / 120.0f,
                            -1.0f / 6.0f};
  constexpr float cc_[8] = {-1.0f / 87178291200.0f, 1.0f / 479001600.0f, -1.0f / 3628800.0f, 1.0f / 40320.0f,
                            -1.0f / 720.0f,         1.0f / 24.0f,        -0.5f,              1.0f};
  float v[K], a[K], c[K];
#pragma unroll
  for (int i = 0; i < K; i++) {
    v[i] = u[i] * u[i];
    a[i] = cs_[0];
    c[i] = cc_[0];
  }
#pragma unroll
  for (int k = 1; k < 7; k++) {
#pragma unroll
    for (int i = 0; i < K; i++) a[i] = a[i] * v[i] + cs_[k];
  }
#pragma unroll
  for (int k = 1; k < 8; k++) {
#pragma unroll
    for (int i = 0; i < K; i++) c[i] = c[i] * v[i] + cc_[k];
  }
#pragma unroll
  for (int i = 0; i < K; i++) {
    sinc[i] = a[i] * v[i] + 1.0f;
    cosu[i] = c[i];
  }
  bool in_range = true;
  if (check) {
#pragma unroll
    for (int i = 0; i < K; i++) in_range = in_range && (v[i] <= 2.89f);
  }
  if (!in_range) {
#pragma unroll
    for (int i = 0; i < K; i++) {
      float su, cu;
      sincosf(u[i], &su, &cu);
      sinc[i] = su / u[i];
      cosu[i] = cu;
    }
  }
}

// Octant polynomials of exp(i x), x in [-pi/4, pi/4], per precision:
// double: sin through x^15, cos through x^16 (next terms < 5e-17);
// float:  sin through x^9,  cos through x^10 (next terms < 2e-9).
template <typename F>
struct OctantPoly;
template <>
struct OctantPoly<double> {
  static constexpr int NS = 7, NC = 9;  // coefficients: PolyTable::osin, PolyTable::ocos
};
template <>
struct OctantPoly<float> {
  static constexpr int NS = 4, NC = 6;
  static constexpr float ps[NS] = {1.0f / 362880.0f, -1.0f / 5040.0f, 1.0f / 120.0f, -1.0f / 6.0f};
  static constexpr float pc[NC] = {-1.0f / 3628800.0f, 1.0f / 40320.0f, -1.0f / 720.0f,
                                   1.0f / 24.0f,       -0.5f,           1.0f};
};

// exp(2 pi i c) for K phases c given in cycles (double); the exact reduction
// is done in double, the octant polynomial in F.
template <int K, typename F>
__device__ __forceinline__ void expi_cycles_k(const double* c, cx<F>* out) {
  using P = OctantPoly<F>;
  // FP64: the coefficients from the constant table (the same values)
  constexpr bool kTbl = std::is_same<F, double>::value;
  CPoly* const tp = kTbl ? poly_table() : nullptr;
  auto ps = [&](int k) -> F { if constexpr (kTbl) return tp->osin[k]; else return P::ps[k]; };
  auto pc = [&](int k) -> F { if constexpr (kTbl) return tp->ocos[k]; else return P::pc[k]; };
  F x[K], v[K], sn[K], cs[K];
  int q[K];
#pragma unroll
  for (int i = 0; i < K; i++) {
    double r = c[i] - rint(c[i]);
    double n4 = rint(4.0 * r);
    x[i] = (F)(kTwoPi * (r - 0.25 * n4));
    v[i] = x[i] * x[i];
    q[i] = ((int)n4) & 3;
    sn[i] = ps(0);
    cs[i] = pc(0);
  }
  // FP64: the coefficients stay in scalar registers (fma_sc)
  auto step = [&](F a, F x2, F c) -> F {
    if constexpr (kTbl) return fma_sc(a, x2, c); else return a * x2 + c;
  };
#pragma unroll
  for (int k = 1; k < P::NS; k++) {
#pragma unroll
    for (int i = 0; i < K; i++) sn[i] = step(sn[i], v[i], ps(k));
  }
#pragma unroll
  for (int k = 1; k < P::NC; k++) {
#pragma unroll
    for (int i = 0; i < K; i++) cs[i] = step(cs[i], v[i], pc(k));
  }
#pragma unroll
  for (int i = 0; i < K; i++) {
    F s_ = (sn[i] * v[i]) * x[i] + x[i];
    F c_ = cs[i];
    // rotate by q quarter turns
    F re = (q[i] & 1) ? -s_ : c_;
    F im = (q[i] & 1) ? c_ : s_;
    if (q[i] & 2) {
      re = -re;
      im = -im;
    }
    out[i] = {re, im};
  }
}

// ---------------------------------------------------------------------------
// Slow part: the A, E (and T) TDI pieces U, V at one midpoint sample.
// Spacecraft i = 0, 1, 2 sit at orientation angle 2 pi i/3 of the rigid
// equal-arm orbit; arm m joins craft m -> (m+1) mod 3.
// out[0..5] = U_A, V_A, U_E, V_E, U_T, V_T  (T only when NSER == 6).
// The spacecraft positions, k.x/c and the receiver phases are always formed
// in double; arm projections, link amplitudes and the TDI algebra in F.
// ---------------------------------------------------------------------------
// S is Src, or Src in the constant address space (decoded sources read
// through the scalar cache)
template <int NSER, typename F, int UC = 1, typename S = Src>
__device__ __forceinline__ void slow_sample(const S& s, const Geo& g, const double* __restrict__ basis, int n,
                                            double t, cx<F>* out, bool check = true) {
  const double ca = basis[4 * n + 0], sa = basis[4 * n + 1];
  const double c2a = basis[4 * n + 2], s2a = basis[4 * n + 3];
  auto affine = [&](const auto* c) { return c[4] + c[0] * ca + c[1] * sa + c[2] * c2a + c[3] * s2a; };

  const F fca = (F)ca, fsa = (F)sa, fc2a = (F)c2a, fs2a = (F)s2a;
  auto affine_f = [&](const auto* c) {
    return (F)c[4] + (F)c[0] * fca + (F)c[1] * fsa + (F)c[2] * fc2a + (F)c[3] * fs2a;
  };
  // arm projections k.n (the arms close the triangle, n_0 + n_1 + n_2 = 0,
  // so the third arm's projections are minus the sum of the first two)
  F kn[3];
  kn[0] = affine_f(s.kn[0]);
  kn[1] = affine_f(s.kn[1]);
  kn[2] = -(kn[0] + kn[1]);

  // phases in cycles: phi_r / (2 pi) = phi0/(2 pi) + dfq t + fdot t^2/2
  //                                    - (f0 + fdot t) k.x_r/c + fdot (k.x_r/c)^2 / 2
  const double base = s.phi0_cyc + s.dfq * t + 0.5 * s.fdot * t * t;
  const double fwd = s.f0 + s.fdot * t;

  // receivers: k.x_r/c, phase in cycles, instantaneous frequency
  double cyc[3];
  F fr[3];
#pragma unroll
  for (int r = 0; r < 3; r++) {
    const double kx = affine(s.xr[r]);
    cyc[r] = base - fwd * kx + 0.5 * s.fdot * kx * kx;
    fr[r] = (F)(fwd - s.fdot * kx);
  }
  // the six links, ordered by receiver: (arm, direction, receiver)
  //   l21 = (0,-1,0)  l31 = (2,+1,0)  l12 = (0,+1,1)  l32 = (1,-1,1)
  //   l23 = (1,+1,2)  l13 = (2,-1,2)
  constexpr int arm_[6] = {0, 2, 0, 1, 1, 2};
  constexpr double sgn_[6] = {-1.0, 1.0, 1.0, -1.0, 1.0, -1.0};
  const F piLc = (F)(kPi * g.Lc);
  const F dterm = (F)(0.5 * kPi * s.fdot * g.Lc * g.Lc);
  F amp[6], u[6], sc[6], cu[6];
#pragma unroll
  for (int l = 0; l < 6; l++) {
    F om = (F)1 - (F)sgn_[l] * kn[arm_[l]];
    amp[l] = piLc * fr[l / 2] - dterm * om;
    u[l] = om * amp[l];
  }
  sinc_cos_k<6, UC>(u, sc, cu, check);
  // w exp(-i u) with w = amp sinc(u)
  cx<F> wz[6];
#pragma unroll
  for (int l = 0; l < 6; l++) {
    const F w = amp[l] * sc[l];
    wz[l] = {w * cu[l], -(w * u[l]) * sc[l]};
  }
  // arm factors G = n^T H n and receiver phase factors P, formed only now so
  // that neither they nor their inputs occupy registers across the series
  cx<F> G[3];
  {
    F pn[3], qn[3];
#pragma unroll
    for (int m = 0; m < 2; m++) {
      qn[m] = affine_f(s.qn[m]);
      pn[m] = (F)s.pn[m][2] + (F)s.pn[m][0] * fc2a + (F)s.pn[m][1] * fs2a;
    }
    pn[2] = -(pn[0] + pn[1]);
    qn[2] = -(qn[0] + qn[1]);
    const cx<F> cp = load_cx<F>(s.cp), cx2 = load_cx<F>(s.cx2);
#pragma unroll
    for (int m = 0; m < 3; m++) {
      F ep = pn[m] * pn[m] - qn[m] * qn[m];
      F ex = pn[m] * qn[m];
      G[m] = {cp.re * ep + cx2.re * ex, cp.im * ep + cx2.im * ex};
    }
  }
  cx<F> P[3];
  if constexpr (UC == 0) {
    // FP64 with every phase small: P_1, P_2 follow from P_0 through the
    // offsets x_r = 2 pi (cyc_r - cyc_0), which the caller's bound keeps
    // within |x| <= 0.25 like the link phases, so they take the same short
    // series: exp(i x) = cos x + i x sinc x
    expi_cycles_k<1, F>(cyc, P);
    F x[2], sx[2], cxr[2];
    x[0] = (F)(kTwoPi * (cyc[1] - cyc[0]));
    x[1] = (F)(kTwoPi * (cyc[2] - cyc[0]));
    sinc_cos_k<2, 0>(x, sx, cxr);
#pragma unroll
    for (int r = 1; r < 3; r++) P[r] = P[0] * cx<F>{cxr[r - 1], x[r - 1] * sx[r - 1]};
  } else {
    expi_cycles_k<3, F>(cyc, P);
  }
  // s_{snd->rcv} = -i G w exp(-i u) P_rcv
  cx<F> lk[6];
#pragma unroll
  for (int l = 0; l < 6; l++) lk[l] = mul_negi(G[arm_[l]] * (P[l / 2] * wz[l]));
  // TDI pieces: U_X = s21 - s31, V_X = s12 - s13, U_Y = s32 - s12,
  //             V_Y = s23 - s21, U_Z = s13 - s23, V_Z = s31 - s32
  // and the A, E (T) combinations without their normalisations 1/sqrt 2,
  // 1/sqrt 6 (1/sqrt 3), which bin_spectrum applies per bin
  const cx<F> UX = lk[0] - lk[1], VX = lk[2] - lk[5];
  const cx<F> UY = lk[3] - lk[2], VY = lk[4] - lk[0];
  const cx<F> UZ = lk[5] - lk[4], VZ = lk[1] - lk[3];
  out[0] = UZ - UX;
  out[1] = VZ - VX;
  out[2] = UX - (F)2 * UY + UZ;
  out[3] = VX - (F)2 * VY + VZ;
  if constexpr (NSER == 6) {
    out[4] = UX + UY + UZ;
    out[5] = VX + VY + VZ;
  }
}

// ---------------------------------------------------------------------------
// Small in-register DFTs (forward sign), natural-order output.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void dft2(cx<F>* x) {
  cx<F> a = x[0], b = x[1];
  x[0] = a + b;
  x[1] = a - b;
}

template <typename F>
__device__ __forceinline__ void dft4(cx<F>* x) {
  cx<F> a0 = x[0], a1 = x[1], a2 = x[2], a3 = x[3];
  cx<F> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
  x[0] = t0 + t2;
  x[2] = t0 - t2;
  x[1] = t1 + mul_negi(t3);
  x[3] = t1 + mul_posi(t3);
}

// ---------------------------------------------------------------------------
// Block-level in-place decimation-in-frequency FFT over NSER series of length
// N held in LDS, with radix-4 passes and a final radix-2 pass when log2 N is
// odd, so that every pass offers NSER * N / 4 butterflies to the NT threads of
// the block.  Output X[k] sits at the digit-reversed position fft_pos<N>(k).
//
// LDS layout of element e of a series (against bank conflicts of the 16-byte
// accesses): an XOR swizzle e ^ X(e >> 3) with X linear over GF(2), chosen so
// that the butterfly reads/writes of every pass, the sample writes and the
// digit-reversed read-out hit distinct banks within 8-lane groups.  Linearity
// lets a butterfly address its four elements as lds_pad(base) ^ lds_pad(ST r)
// with the second term a constant.
// ---------------------------------------------------------------------------
template <int N>
struct LdsSwizzle {
  static constexpr int LB = 3;
  static constexpr int NBITS = (N == 128 ? 7 : N == 256 ? 8 : N == 512 ? 9 : 10) - LB;
  static constexpr int col(int j) {
    constexpr int c128[] = {7, 5, 2, 4}, c256[] = {1, 6, 7, 1, 2}, c512[] = {3, 7, 3, 0, 6, 2},
                  c1024[] = {1, 6, 5, 6, 6, 7, 2};
    return N == 128 ? c128[j] : N == 256 ? c256[j] : N == 512 ? c512[j] : c1024[j];
  }
};

template <int N>
__device__ __forceinline__ constexpr int lds_pad(int e) {
  using S = LdsSwizzle<N>;
  int x = 0;
#pragma unroll
  for (int j = 0; j < S::NBITS; j++) x ^= ((e >> (S::LB + j)) & 1) ? S::col(j) : 0;
  return e ^ x;
}

// address of element base + off where off's bits are clear in base (off a constant)
template <int N>
__device__ __forceinline__ int lds_pad_add(int base, int base_addr, int off) {
  (void)base;
  return base_addr ^ lds_pad<N>(off);
}

template <int N>
constexpr int series_pitch() {
  return N;
}

// threads per block for template width N: one sample and one bin per thread
// at N = 256, up to 4 of each at N = 1024
template <int N>
constexpr int block_threads() {
  return N < 256 ? N : 256;
}

template <int N>
__device__ __forceinline__ int fft_pos(int k) {
  int pos = 0, mult = N, m = N;
#pragma unroll
  for (int p = 0; p < 6; p++) {
    if (m >= 4) {
      mult >>= 2;
      pos += (k & 3) * mult;
      k >>= 2;
      m >>= 2;
    } else if (m == 2) {
      mult >>= 1;
      pos += (k & 1) * mult;
      k >>= 1;
      m = 1;
    }
  }
  return pos;
}

// Each wave owns whole series when the series divide evenly over the waves of
// the block (4 series on 1, 2 or 4 waves): a pass then only reads what the
// same wave wrote in the pass before, and the passes are ordered by a
// wavefront-scope fence instead of a block barrier.
template <int NSER, int NT>
constexpr bool fft_wave_local() {
  return NSER % (NT / kWave) == 0;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N, int R, int ST, typename F>
__device__ __forceinline__ void fft_butterfly(cx<F>* b, const cx<F>* __restrict__ tw, int beta) {
  constexpr int TWS = N / (R * ST);
  int grp = beta / ST, i = beta % ST;
  int base = grp * R * ST + i;
  const int base_addr = lds_pad<N>(base);
  cx<F> x[R];
#pragma unroll
  for (int r = 0; r < R; r++) x[r] = b[lds_pad_add<N>(base, base_addr, ST * r)];
  if constexpr (R == 4) dft4(x);
  if constexpr (R == 2) dft2(x);
  if constexpr (ST > 1) {
#pragma unroll
    for (int r = 1; r < R; r++) x[r] = x[r] * tw[TWS * i * r];
  }
#pragma unroll
  for (int r = 0; r < R; r++) b[lds_pad_add<N>(base, base_addr, ST * r)] = x[r];
}

template <int N, int R, int ST, int NSER, int NT, typename F>
__device__ __forceinline__ void fft_pass(cx<F>* buf, const cx<F>* __restrict__ tw, int tid) {
  constexpr int NB = N / R;  // butterflies per series
  constexpr int SP = series_pitch<N>();
  // where the butterflies divide evenly over the lanes, every lane runs the
  // same number of them: a uniform loop without per-lane exit masks
  if constexpr (fft_wave_local<NSER, NT>()) {
    constexpr int SPW = NSER / (NT / kWave);  // series per wave
    const int w = tid / kWave, lane = tid % kWave;
    if constexpr ((SPW * NB) % kWave == 0) {
#pragma unroll 1
      for (int it = 0; it < SPW * NB / kWave; it++) {
        const int item = lane + it * kWave;
        fft_butterfly<N, R, ST>(buf + (w * SPW + item / NB) * SP, tw, item % NB);
      }
    } else {
#pragma unroll 1
      for (int item = lane; item < SPW * NB; item += kWave)
        fft_butterfly<N, R, ST>(buf + (w * SPW + item / NB) * SP, tw, item % NB);
    }
    wave_sync();
  } else {
    if constexpr ((NSER * NB) % NT == 0) {
#pragma unroll 1
      for (int it = 0; it < NSER * NB / NT; it++) {
        const int item = tid + it * NT;
        fft_butterfly<N, R, ST>(buf + (item / NB) * SP, tw, item % NB);
      }
    } else {
#pragma unroll 1
      for (int item = tid; item < NSER * NB; item += NT)
        fft_butterfly<N, R, ST>(buf + (item / NB) * SP, tw, item % NB);
    }
    __syncthreads();
  }
}

// all passes; ends with a block barrier, so every thread may read every series
template <int N, int NT, int NSER, int M, typename F>
__device__ __forceinline__ void fft_stages(cx<F>* buf, const cx<F>* __restrict__ tw, int tid) {
  if constexpr (M >= 4) {
    fft_pass<N, 4, M / 4, NSER, NT>(buf, tw, tid);
    fft_stages<N, NT, NSER, M / 4>(buf, tw, tid);
  } else if constexpr (M == 2) {
    fft_pass<N, 2, 1, NSER, NT>(buf, tw, tid);
  }
  if constexpr (M == N && fft_wave_local<NSER, NT>()) __syncthreads();
}

// ---------------------------------------------------------------------------
// One template: slow part -> FFT.  Afterwards bin_spectrum() reads the
// spectrum at any window bin j from the transformed U/V series in LDS.
// Ends with a barrier, so the caller may read the workspace immediately.
// ---------------------------------------------------------------------------
template <int N, int NSER, typename F, int NT = block_threads<N>(), bool kUniform = false, typename S = Src>
__device__ __forceinline__ void template_transform(const S& s, const Geo& g, const WaveTables<F>& tb,
                                                   cx<F>* buf, int tid) {
  constexpr int SP = series_pitch<N>();
  // kUniform: where N divides evenly over the block, every thread runs the
  // same number of samples (a loop without per-lane exit masks; the FFT
  // passes already take every thread id below NT).  It pays in the sampler's
  // band loops; the fused likelihood kernel runs faster with the per-lane
  // loop, which the compiler schedules differently.
  constexpr bool kEven = kUniform && N % NT == 0;
  constexpr int NIT = (N + NT - 1) / NT;
  // link phases u = (1 -+ k.n) (pi f L/c - ...) stay below 2 pi (L/c) f_max plus
  // a tiny fdot term, and so do the receiver phase offsets
  // 2 pi (cyc_r - cyc_0) = 2 pi (k.x_r - k.x_0)/c (-f + fdot (k.x_r + k.x_0)/(2c))
  // with |k.x_r - k.x_0| <= L and |k.x_r| <= AU + 2L: block-uniform choice of
  // the short series for both (FP64 only; the FP32 series are short already)
  const double f_max = fabs(s.f0) + fabs(s.fdot) * (g.T + 1100.0);
  const double u_max = 2.0 * kPi * g.Lc * (f_max + fabs(s.fdot) * (kAU / kC + 2.0 * g.Lc));
  const bool small_u = std::is_same<F, double>::value && u_max <= 0.25;
  // every link phase below 1.7 (sources in band): no per-lane range test
  const bool check = !(u_max <= 1.69);
  if constexpr (!std::is_same<F, double>::value) {
#pragma unroll 1
    for (int it = 0, n = tid; kEven ? it < NIT : n < N; it++, n += NT) {
      double t = ((double)n + 0.5) * g.T / (double)N;
      cx<F> v[6];
      slow_sample<NSER, F, 1, S>(s, g, tb.basis, n, t, v, check);
      const int a = lds_pad<N>(n);
#pragma unroll
      for (int c = 0; c < NSER; c++) buf[c * SP + a] = v[c];
    }
  } else if (small_u) {
#pragma unroll 1
    for (int it = 0, n = tid; kEven ? it < NIT : n < N; it++, n += NT) {
      double t = ((double)n + 0.5) * g.T / (double)N;
      cx<F> v[6];
      slow_sample<NSER, F, 0, S>(s, g, tb.basis, n, t, v);
      const int a = lds_pad<N>(n);
#pragma unroll
      for (int c = 0; c < NSER; c++) buf[c * SP + a] = v[c];
    }
  } else {
#pragma unroll 1
    for (int it = 0, n = tid; kEven ? it < NIT : n < N; it++, n += NT) {
      double t = ((double)n + 0.5) * g.T / (double)N;
      cx<F> v[6];
      slow_sample<NSER, F, 1, S>(s, g, tb.basis, n, t, v, check);
      const int a = lds_pad<N>(n);
#pragma unroll
      for (int c = 0; c < NSER; c++) buf[c * SP + a] = v[c];
    }
  }
  __syncthreads();
  fft_stages<N, NT, NSER, N>(buf, tb.fft_tw, tid);
}

// Spectra of channels 0..NCH-1 (A, E[, T]) at window bin j, from the
// transformed U/V series in LDS: C = c_A,E,T (1 - D^2) F (U + D V) with
// D = exp(-i x), x = 2 pi (q + k) L/(c T), F = (1/2)(T/N) exp(-i pi k/N),
// k = j - N/2, and the channel normalisations c = 1/sqrt 2, 1/sqrt 6, 1/sqrt 3.
// D is the carrier's factor exp(-2 pi i q L/(c T)) times the bin's table
// entry (the relative error of sin x stays within a few ulp wherever
// q + k >= N/2, since |k| <= N/2); 1 - D^2 = 2 sin x (sin x, cos x) is formed
// without cancellation (at 0.1 mHz x ~ 5e-3, where 1 - cos 2x would lose
// three digits in single precision).
template <int N, int NCH, typename F, typename S = Src>
__device__ __forceinline__ void bin_spectrum(const S& s, const Geo& g, const WaveTables<F>& tb, const cx<F>* buf,
                                             int j, cx<F>* out) {
  constexpr int SP = series_pitch<N>();
  constexpr double norm[3] = {kInvSqrt2, kInvSqrt6, kInvSqrt3};
  const int kk = (j + N / 2) & (N - 1);
  const int pos = lds_pad<N>(fft_pos<N>(kk));
  const cx<F> D = load_cx<F>(s.dq) * tb.bin_W[j];
  // D = (cos x, -sin x):  1 - D^2 = (2 sin^2 x, 2 sin x cos x)
  const F two_s = (F)2 * D.im;
  const cx<F> Fj = tb.bin_F[j];
#pragma unroll
  for (int c = 0; c < NCH; c++) {
    const F h = (F)norm[c] * two_s;
    const cx<F> one_m = {h * D.im, -h * D.re};
    cx<F> U = buf[(2 * c) * SP + pos];
    cx<F> V = buf[(2 * c + 1) * SP + pos];
    out[c] = one_m * (Fj * (U + D * V));
  }
}

}  // namespace gbl
