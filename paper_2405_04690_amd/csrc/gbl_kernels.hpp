// gbl_kernels.hpp -- HIP kernels of the GB likelihood library (gfx950).
#pragma once

#include <type_traits>

#include "gbl_device.hpp"

namespace gbl {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double qnan() { return __builtin_nan(""); }

// ---------------------------------------------------------------------------
// Table construction (once per context)
// ---------------------------------------------------------------------------
__global__ void k_init_wave_tables(int N, double T, double Lc, double* basis, cd* fft_tw, cd* bin_F, cd* bin_W,
                                   cf* fft_tw32, cf* bin_F32, cf* bin_W32) {
  int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double t = ((double)n + 0.5) * T / (double)N;
  double a = kTwoPi * t / kYear;
  double sa, ca, s2a, c2a;
  sincos(a, &sa, &ca);
  sincos(2.0 * a, &s2a, &c2a);
  basis[4 * n + 0] = ca;
  basis[4 * n + 1] = sa;
  basis[4 * n + 2] = c2a;
  basis[4 * n + 3] = s2a;
  double s, c;
  sincospi(-2.0 * (double)n / (double)N, &s, &c);
  fft_tw[n] = {c, s};
  int k = n - N / 2;
  sincospi(-(double)k / (double)N, &s, &c);
  double h = 0.5 * T / (double)N;
  bin_F[n] = {h * c, h * s};
  bin_W[n] = expi_cycles(-(double)k * (Lc / T));
  fft_tw32[n] = cvt<float>(fft_tw[n]);
  bin_F32[n] = cvt<float>(bin_F[n]);
  bin_W32[n] = cvt<float>(bin_W[n]);
}

// PSD basis of eq. psd, linear in (S_oms, S_acc):  S_n = S_oms P1 + S_acc P2,
//   P1 = 8 sin^2 x (2 + cos x) (2 pi f/c)^2 [1 + (2 mHz/f)^4]
//   P2 = 16 sin^2 x (3 + 2 cos x + cos 2x) (2 pi c f)^-2 [1 + (0.4 mHz/f)^2][1 + (f/8 mHz)^4]
// and the parameter-free factors of the Galactic foreground (Sec. 3):
//   S_fg = 6 x^2 sin^2 x h_fg(f),  h_fg = 1/2 A_fg f^(-7/3) exp(-s1 f^alpha) [1 + tanh(-s2 (f - f_k))]
//   P3 = 3 x^2 sin^2 x f^(-7/3),   LF = ln f
__global__ void k_init_psd_basis(int64_t k_min, int64_t nb, double T, double L, double* P1, double* P2, double* P3,
                                 double* LF) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  double f = (double)(k_min + i) / T;
  double x = kTwoPi * f * L / kC;
  double sx, cx;
  sincos(x, &sx, &cx);
  double c2x = cx * cx - sx * sx;
  double s2 = sx * sx;
  double r_oms = 2e-3 / f;
  double r_acc = 0.4e-3 / f;
  double r_hi = f / 8e-3;
  double wo = kTwoPi * f / kC;
  double wa = kTwoPi * kC * f;
  P1[i] = 8.0 * s2 * (2.0 + cx) * wo * wo * (1.0 + r_oms * r_oms * r_oms * r_oms);
  P2[i] = 16.0 * s2 * (3.0 + 2.0 * cx + c2x) / (wa * wa) * (1.0 + r_acc * r_acc) * (1.0 + r_hi * r_hi * r_hi * r_hi);
  P3[i] = 3.0 * x * x * s2 * pow(f, -7.0 / 3.0);
  LF[i] = log(f);
}

// Galactic-foreground term of one bin: P3 = 3 x^2 sin^2 x f^(-7/3), lf = ln f,
// fg = (A_fg, alpha, f_k, s1, s2)
__device__ __forceinline__ double foreground_term(double f, double p3, double lf, const double* fg) {
  const double fa = exp(fg[1] * lf);  // f^alpha
  return fg[0] * p3 * exp(-fg[3] * fa) * (1.0 + tanh(-fg[4] * (f - fg[2])));
}

// Sum over the block (NT threads, NT/64 waves); valid in thread 0 only.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / kWave; i++) t += red[i];
  }
  return t;
}

// ---------------------------------------------------------------------------
// gb_waveform: one block per template; writes A, E (and T) band slices of
// width N starting at element `off` of each output array.
// ---------------------------------------------------------------------------
template <int N, int NSER, typename F>
struct WaveSmem {
  cx<F> buf[NSER * series_pitch<N>()];
  Src src;
};

template <int N, int NSER, typename F>
__device__ __forceinline__ void waveform_one(const Geo& g, const WaveTables<F>& tb, const double* __restrict__ prm,
                                             int64_t off, cd* __restrict__ A, cd* __restrict__ E,
                                             cd* __restrict__ Tc, int64_t* __restrict__ start,
                                             WaveSmem<N, NSER, F>& sm) {
  constexpr int NT = block_threads<N>();
  const int tid = threadIdx.x;
  if (tid < kWave) decode_sources<1>(prm, prm, g, &sm.src);  // one wave decodes, the block shares it
  __syncthreads();
  const Src& s = sm.src;
  if (s.state == 0) template_transform<N, NSER, F>(s, g, tb, sm.buf, tid);
  cd* outs[3] = {A, E, Tc};
  constexpr int NCH = NSER / 2;
  for (int j = tid; j < N; j += NT) {
    cx<F> v[NCH];
    if (s.state == 0) bin_spectrum<N, NCH, F>(s, g, tb, sm.buf, j, v);
#pragma unroll
    for (int c = 0; c < NCH; c++) {
      cd o;
      if (s.state == 0)
        o = cvt<double>(v[c]);
      else if (s.state == 1)
        o = {0.0, 0.0};
      else
        o = {qnan(), qnan()};
      outs[c][off + j] = o;
    }
  }
  if (tid == 0) *start = (s.state == 2) ? 0 : s.q - N / 2;
  __syncthreads();  // the shared decode may be overwritten afterwards
}

template <int N, int NSER, typename F>
__global__ __launch_bounds__(block_threads<N>()) void k_waveform(Geo g, WaveTables<F> tb,
                                                                 const double* __restrict__ params, int64_t b0,
                                                                 cd* __restrict__ A, cd* __restrict__ E,
                                                                 cd* __restrict__ Tc, int64_t* __restrict__ start) {
  __shared__ WaveSmem<N, NSER, F> sm;
  const int64_t b = b0 + blockIdx.x;
  waveform_one<N, NSER, F>(g, tb, params + 8 * b, b * N, A, E, Tc, start + b, sm);
}

// ---------------------------------------------------------------------------
// gb_delta_loglike (FP64): one block per (old, new) pair.  The old template r
// goes into an LDS window, the new template a through the FFT workspace, then
//   dlogl = 4 df [ sum Re(conj R) d / S - 1/2 sum |d|^2 / S ],  d = a - r,
// over the union of the two windows clipped to the band (channels A, E).
// The residual and PSD values of a's window are fetched before the templates
// are built, so their HBM latency overlaps the arithmetic.
// ---------------------------------------------------------------------------
struct DeltaArgs {
  const cd* residual;
  int n_res;
  const double* psd;
  int n_psd;
  int psd_inv;
  const double* p_old;
  const double* p_new;
  const int32_t* res_idx;
  const int32_t* psd_idx;
  double* out;
  // mixed precision: pairs whose FP32 error estimate exceeds route_tol are
  // queued (index - route_b0) on route_list / route_count for an FP64 pass
  int32_t* route_list;
  int* route_count;
  double route_tol;
  int64_t route_b0;
  // decoded sources of pairs [src_b0, src_b0 + chunk): old at 2 (b - src_b0),
  // new at 2 (b - src_b0) + 1 (k_decode_pairs)
  const Src* srcs;
  int64_t src_b0;
};

// Decode pass: one thread per template of pairs [b0, b0 + nb) into out
// (old, new interleaved).  The fused kernels then read the decoded sources
// through the scalar cache: per template a wave loads each coefficient once
// into scalar registers instead of every lane reading it from LDS, and no
// wave of the fused kernel spends time on the decode.
// (decoded into LDS first, then copied out in 16-byte pieces by consecutive
// lanes, so that the stores to the workspace are contiguous)
constexpr int kDecodeBlock = 64;

__global__ __launch_bounds__(kDecodeBlock) void k_decode_pairs(Geo g, const double* __restrict__ p_old,
                                                               const double* __restrict__ p_new, int64_t b0,
                                                               int64_t nb, Src* __restrict__ out) {
  static_assert(sizeof(Src) % 16 == 0, "decoded sources are copied in 16-byte pieces");
  __shared__ Src stage[kDecodeBlock];
  const int64_t first = (int64_t)blockIdx.x * kDecodeBlock;
  const int64_t i = first + threadIdx.x;
  if (i < 2 * nb) decode_source(((i & 1) ? p_new : p_old) + 8 * (b0 + (i >> 1)), g, stage[threadIdx.x]);
  __syncthreads();
  const int64_t count = (2 * nb - first) < kDecodeBlock ? (2 * nb - first) : kDecodeBlock;
  const int pieces = (int)(count * (int64_t)(sizeof(Src) / 16));
  const uint4* src = reinterpret_cast<const uint4*>(stage);
  uint4* dst = reinterpret_cast<uint4*>(out + first);
  for (int k = threadIdx.x; k < pieces; k += kDecodeBlock) dst[k] = src[k];
}

// a decoded source in the constant address space: loads of its fields are
// scalar loads
using ConstSrc = const __attribute__((address_space(4))) Src;

// Wide templates (N >= 512) keep the old template's spectrum in registers
// and hand it over through the FFT buffer once the new template's bins are
// taken, instead of holding it in an LDS array of its own: 64 instead of
// 96 KB at N = 1024, so that two blocks share a CU and one block's barriers
// are filled by the other's work.
template <int N>
constexpr bool delta_rwin_in_buf() {
  return N >= 512;
}

// threads per block of the fused likelihood kernels: one per sample and bin
// up to N = 256, two per thread above (8 waves at N = 1024, two blocks per CU)
template <int N>
constexpr int delta_threads() {
  return N <= 256 ? N : N / 2;
}

// FP64 templates from N = 512 on read the pair's decoded sources from LDS:
// with two samples and bins per thread they hold more values at once, and
// read through the scalar cache the sources then spill several hundred
// scalar registers; up to N = 256, and in FP32, the scalar cache is faster
template <int N, typename F>
constexpr bool delta_lds_src() {
  return N >= 512 && std::is_same<F, double>::value;
}

template <int N, typename F>
struct DeltaSmem {
  cx<F> buf[4 * series_pitch<N>()];
  cx<F> rwin[delta_rwin_in_buf<N>() ? 1 : 2 * N];
  double red[6 * (delta_threads<N>() / kWave)];
};

template <int N, typename F>
__device__ __forceinline__ void delta_one(const Geo& g, const WaveTables<F>& tb, const DeltaArgs& da, int64_t b,
                                          DeltaSmem<N, F>& sm) {
  constexpr int NT = delta_threads<N>();
  constexpr int BPT = N / NT;  // window bins per thread
  const int tid = threadIdx.x;
  // validity and carrier bins first; the decoded sources come from the
  // decode pass
  const SrcHead ho = source_head(da.p_old + 8 * b, g);
  const SrcHead hn = source_head(da.p_new + 8 * b, g);
  const int ri = da.res_idx[b];
  const int pi = da.psd_idx[b];
  if (ho.state == 2 || hn.state == 2 || ri < 0 || ri >= da.n_res || pi < 0 || pi >= da.n_psd) {
    if (tid == 0) da.out[b] = qnan();
    return;  // uniform over the block
  }
  const int64_t nb = g.n_bins;
  const cd* RA = da.residual + (int64_t)ri * 2 * nb;
  const cd* RE = RA + nb;
  const double* SA = da.psd + (int64_t)pi * 2 * nb;
  const double* SE = SA + nb;
  const int64_t ka = hn.q - N / 2;
  const int64_t kr = ho.q - N / 2;
  const int psd_inv = da.psd_inv;

  auto weight = [&](const double* Sc, int64_t idx) { return psd_inv ? Sc[idx] : 1.0 / Sc[idx]; };

  using SrcRef = std::conditional_t<delta_lds_src<N, F>(), Src, ConstSrc>;
  SrcRef* cs;
  if constexpr (delta_lds_src<N, F>()) {
    // the pair's two decoded sources into LDS, 16 bytes per thread
    __shared__ Src lds_src[2];
    static_assert(sizeof(Src) % 16 == 0, "Src is copied in 16-byte pieces");
    constexpr int kPieces = 2 * (int)sizeof(Src) / 16;
    static_assert(kPieces <= NT, "one piece per thread");
    const int4* src16 = reinterpret_cast<const int4*>(da.srcs + 2 * (b - da.src_b0));
    if (tid < kPieces) reinterpret_cast<int4*>(lds_src)[tid] = src16[tid];
    __syncthreads();
    cs = lds_src;
  } else {
    cs = (ConstSrc*)da.srcs + 2 * (b - da.src_b0);
  }

  // old template r: its spectrum over its window, in LDS (rw) or, for the
  // wide templates, in registers until the new template's bins are taken
  constexpr bool kRegR = delta_rwin_in_buf<N>();
  cx<F> rr[BPT][2];
  cx<F> aa[BPT][2];
  cx<F>* rw = kRegR ? sm.buf : sm.rwin;
  if (ho.state == 0) {
    SrcRef& so = cs[0];
    template_transform<N, 4, F, NT>(so, g, tb, sm.buf, tid);
#pragma unroll
    for (int m = 0; m < BPT; m++) {
      const int j = tid + NT * m;
      bin_spectrum<N, 2, F>(so, g, tb, sm.buf, j, rr[m]);
      if constexpr (!kRegR) {
        sm.rwin[j] = rr[m][0];
        sm.rwin[N + j] = rr[m][1];
      }
    }
  }
  __syncthreads();
  if constexpr (kRegR) {
    // new template a: bins into registers, then r's spectrum into the buffer
    if (hn.state == 0) {
      SrcRef& sn = cs[1];
      template_transform<N, 4, F, NT>(sn, g, tb, sm.buf, tid);
#pragma unroll
      for (int m = 0; m < BPT; m++) bin_spectrum<N, 2, F>(sn, g, tb, sm.buf, tid + NT * m, aa[m]);
    }
    __syncthreads();
    if (ho.state == 0) {
#pragma unroll
      for (int m = 0; m < BPT; m++) {
        rw[tid + NT * m] = rr[m][0];
        rw[N + tid + NT * m] = rr[m][1];
      }
    }
    __syncthreads();
  }

  double acc_rd = 0.0, acc_dd = 0.0;
  auto accumulate = [&](cd R0, cd R1, double w0, double w1, cd d0, cd d1) {
    acc_rd += (R0.re * d0.re + R0.im * d0.im) * w0 + (R1.re * d1.re + R1.im * d1.im) * w1;
    acc_dd += (d0.re * d0.re + d0.im * d0.im) * w0 + (d1.re * d1.re + d1.im * d1.im) * w1;
  };
  // FP32 templates: magnitudes of the inner-product terms <a|a>, <r|r>,
  // <R|a>, <R|r> for the error estimate (<a|r> is at most max(<a|a>, <r|r>))
  constexpr bool kEst = std::is_same<F, float>::value;
  double m_aa = 0.0, m_rr = 0.0, m_Ra = 0.0, m_Rr = 0.0;
  // x = a: adds to <a|a>, <R|a>; else to <r|r>, <R|r>
  auto magnitude = [&](cd R0, cd R1, double w0, double w1, cd x0, cd x1, bool is_a) {
    const double xx = (x0.re * x0.re + x0.im * x0.im) * w0 + (x1.re * x1.re + x1.im * x1.im) * w1;
    const double Rx = (R0.re * x0.re + R0.im * x0.im) * w0 + (R1.re * x1.re + R1.im * x1.im) * w1;
    if (is_a) {
      m_aa += xx;
      m_Ra += Rx;
    } else {
      m_rr += xx;
      m_Rr += Rx;
    }
  };

  if (hn.state == 0) {
    SrcRef& sn = cs[1];
    if constexpr (!kRegR) template_transform<N, 4, F, NT>(sn, g, tb, sm.buf, tid);
    // a's window, one bin per iteration: residual and weights are loaded at
    // the top of the iteration (not earlier: at four waves per SIMD the other
    // waves hide the latency, and no registers stay occupied across the
    // template builds or across the bins of the wider templates)
#pragma unroll
    for (int m = 0; m < BPT; m++) {
      const int j = tid + NT * m;
      int64_t k = ka + j;
      if (k < g.k_min || k >= g.k_min + nb) continue;
      const int64_t idx = k - g.k_min;
      const cd R0 = RA[idx], R1 = RE[idx];
      const double W0 = weight(SA, idx), W1 = weight(SE, idx);
      cx<F> v[2];
      if constexpr (kRegR) {
        v[0] = aa[m][0];
        v[1] = aa[m][1];
      } else {
        bin_spectrum<N, 2, F>(sn, g, tb, sm.buf, j, v);
      }
      cd a0 = cvt<double>(v[0]);
      cd a1 = cvt<double>(v[1]);
      int64_t jr = k - kr;
      const bool has_r = ho.state == 0 && jr >= 0 && jr < N;
      if constexpr (kEst) {
        if (da.route_list) {
          magnitude(R0, R1, W0, W1, a0, a1, true);
          if (has_r) magnitude(R0, R1, W0, W1, cvt<double>(rw[jr]), cvt<double>(rw[N + jr]), false);
        }
      }
      if (has_r) {
        a0 = a0 - cvt<double>(rw[jr]);
        a1 = a1 - cvt<double>(rw[N + jr]);
      }
      accumulate(R0, R1, W0, W1, a0, a1);
    }
  }
  if (ho.state == 0) {
    // bins of r's window not already covered by a's window
#pragma unroll
    for (int m = 0; m < BPT; m++) {
      const int j = tid + NT * m;
      int64_t k = kr + j;
      if (hn.state == 0 && k >= ka && k < ka + N) continue;
      if (k < g.k_min || k >= g.k_min + nb) continue;
      int64_t idx = k - g.k_min;
      cd r0 = cvt<double>(kRegR ? rr[m][0] : sm.rwin[j]), r1 = cvt<double>(kRegR ? rr[m][1] : sm.rwin[N + j]);
      const cd R0 = RA[idx], R1 = RE[idx];
      const double w0 = weight(SA, idx), w1 = weight(SE, idx);
      if constexpr (kEst) {
        if (da.route_list) magnitude(R0, R1, w0, w1, r0, r1, false);
      }
      accumulate(R0, R1, w0, w1, cd{-r0.re, -r0.im}, cd{-r1.re, -r1.im});
    }
  }
  acc_rd = block_sum<NT>(acc_rd, sm.red);
  acc_dd = block_sum<NT>(acc_dd, sm.red + NT / kWave);
  if (tid == 0) da.out[b] = g.df4 * acc_rd - 0.5 * g.df4 * acc_dd;
  if constexpr (kEst) {
    if (da.route_list) {
      m_aa = block_sum<NT>(m_aa, sm.red + 2 * (NT / kWave));
      m_rr = block_sum<NT>(m_rr, sm.red + 3 * (NT / kWave));
      m_Ra = block_sum<NT>(m_Ra, sm.red + 4 * (NT / kWave));
      m_Rr = block_sum<NT>(m_Rr, sm.red + 5 * (NT / kWave));
      if (tid == 0) {
        // error estimate of the FP32 path: 20 * 2^-24 * the largest term
        const double M = g.df4 * fmax(fmax(m_aa, m_rr), fmax(fabs(m_Ra), fabs(m_Rr)));
        if (20.0 * 5.9604644775390625e-8 * M > da.route_tol) {
          const int pos = atomicAdd(da.route_count, 1);
          da.route_list[pos] = (int32_t)(b - da.route_b0);
        }
      }
    }
  }
}

// occupancy target of the fused kernel: four waves per SIMD at every width
// (at most 128 VGPRs; the kernels fit in 112 without spills)
template <int N>
constexpr int delta_min_waves() {
  return 4;
}

template <int N, typename F>
__global__ __launch_bounds__(delta_threads<N>(), delta_min_waves<N>()) void k_delta_loglike(Geo g, WaveTables<F> tb,
                                                                                            DeltaArgs da, int64_t b0) {
  __shared__ DeltaSmem<N, F> sm;
  delta_one<N, F>(g, tb, da, b0 + blockIdx.x, sm);
}

// FP64 pass over a list of pairs (the mixed-precision pairs whose error
// estimate is too large): block i takes entry i, blocks past the count exit.
template <int N>
__global__ __launch_bounds__(delta_threads<N>(), delta_min_waves<N>()) void k_delta_loglike_list(
    Geo g, WaveTables<double> tb, DeltaArgs da, int64_t b0, const int* __restrict__ count,
    const int32_t* __restrict__ list) {
  __shared__ DeltaSmem<N, double> sm;
  if ((int)blockIdx.x >= *count) return;
  delta_one<N, double>(g, tb, da, b0 + list[blockIdx.x], sm);
}

// ---------------------------------------------------------------------------
// Uneven template widths in one call: bucket the templates by N on the
// device (atomic position counters, no host round trip), then one launch per
// width whose grid covers the whole batch; block i takes the i-th template of
// its bucket and blocks past the bucket's count exit at once, so the hardware
// dispatcher balances the work and the host never waits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int width_bucket(int N) {
  return N == 128 ? 0 : N == 256 ? 1 : N == 512 ? 2 : N == 1024 ? 3 : -1;
}

__global__ void k_bucket_reset(int* counts, int n) {
  if (threadIdx.x < n) counts[threadIdx.x] = 0;
}

// Templates whose width is not supported are not queued; they get a NaN
// output (bad_out) or the start-bin sentinel INT64_MIN (bad_start).
// Positions are taken per block: LDS atomics give each pair its place among
// the block's pairs of the same width, and one global atomic per width and
// block reserves the block's run in the bucket (a global atomic per pair
// would serialise on the four counters).  The order inside a bucket follows
// the order in which blocks reserve; every pair is queued exactly once.
constexpr int kBucketWidths = 4;

__global__ __launch_bounds__(256) void k_bucket_by_width(const int32_t* __restrict__ widths, int64_t b0, int64_t nb,
                                                         int cap, int* __restrict__ counts,
                                                         int32_t* __restrict__ perm, double* __restrict__ bad_out,
                                                         int64_t* __restrict__ bad_start) {
  __shared__ int local_count[kBucketWidths], block_base[kBucketWidths];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
  if (tid < kBucketWidths) local_count[tid] = 0;
  __syncthreads();
  int slot = -1, local = 0;
  if (i < nb) {
    slot = width_bucket(widths[b0 + i]);
    if (slot < 0) {
      if (bad_out) bad_out[b0 + i] = qnan();
      if (bad_start) bad_start[b0 + i] = INT64_MIN;
    } else {
      local = atomicAdd(&local_count[slot], 1);
    }
  }
  __syncthreads();
  if (tid < kBucketWidths && local_count[tid] > 0) block_base[tid] = atomicAdd(&counts[tid], local_count[tid]);
  __syncthreads();
  if (slot >= 0) perm[(int64_t)slot * cap + block_base[slot] + local] = (int32_t)i;
}

template <int N, typename F>
__global__ __launch_bounds__(delta_threads<N>(), delta_min_waves<N>()) void k_delta_loglike_bucket(Geo g,
                                                                                                   WaveTables<F> tb,
                                                                                                   DeltaArgs da,
                                                                             int64_t b0, const int* __restrict__ count,
                                                                             const int32_t* __restrict__ perm) {
  __shared__ DeltaSmem<N, F> sm;
  if ((int)blockIdx.x >= *count) return;
  delta_one<N, F>(g, tb, da, b0 + perm[blockIdx.x], sm);
}

template <int N, int NSER, typename F>
__global__ __launch_bounds__(block_threads<N>()) void k_waveform_bucket(Geo g, WaveTables<F> tb,
                                                                        const double* __restrict__ params, int64_t b0,
                                                                        const int64_t* __restrict__ out_offset,
                                                                        cd* A, cd* E, cd* Tc, int64_t* start,
                                                                        const int* __restrict__ count,
                                                                        const int32_t* __restrict__ perm) {
  __shared__ WaveSmem<N, NSER, F> sm;
  if ((int)blockIdx.x >= *count) return;
  const int64_t b = b0 + perm[blockIdx.x];
  waveform_one<N, NSER, F>(g, tb, params + 8 * b, out_offset[b], A, E, Tc, start + b, sm);
}

// ---------------------------------------------------------------------------
// gb_scatter_add: residual[res_idx[b]] += sign * template b (A, E), FP64 atomics.
// ---------------------------------------------------------------------------
template <int N, typename F>
__global__ __launch_bounds__(block_threads<N>()) void k_scatter_add(Geo g, WaveTables<F> tb,
                                                                    const double* __restrict__ params, int64_t b0,
                                                                    double sign, cd* residual, int n_res,
                                                                    const int32_t* __restrict__ res_idx) {
  constexpr int NT = block_threads<N>();
  __shared__ cx<F> buf[4 * series_pitch<N>()];
  __shared__ Src s_sh;
  const int64_t b = b0 + blockIdx.x;
  const int tid = threadIdx.x;
  const SrcHead h = source_head(params + 8 * b, g);
  const int ri = res_idx[b];
  if (h.state != 0 || ri < 0 || ri >= n_res) return;  // zero or invalid templates add nothing
  if (tid < kWave) decode_sources<1>(params + 8 * b, params + 8 * b, g, &s_sh);
  __syncthreads();
  const Src& s = s_sh;
  template_transform<N, 4, F>(s, g, tb, buf, tid);
  const int64_t nb = g.n_bins;
  const int64_t k0 = s.q - N / 2;
  cd* R = residual + (int64_t)ri * 2 * nb;
  for (int j = tid; j < N; j += NT) {
    int64_t k = k0 + j;
    if (k < g.k_min || k >= g.k_min + nb) continue;
    int64_t idx = k - g.k_min;
    cx<F> v[2];
    bin_spectrum<N, 2, F>(s, g, tb, buf, j, v);
#pragma unroll
    for (int c = 0; c < 2; c++) {
      double* dst = reinterpret_cast<double*>(R + c * nb + idx);
      atomicAdd(dst, sign * (double)v[c].re);
      atomicAdd(dst + 1, sign * (double)v[c].im);
    }
  }
}

// ---------------------------------------------------------------------------
// PSD evaluation and the noise-parameter log-likelihood
// ---------------------------------------------------------------------------
// rows pc = p * 2 + c over blockIdx.y, bins over blockIdx.x (both grid-stride);
// noise sets of NP = 4 (instrument) or 9 (with the foreground) parameters
struct PsdBasis {
  const double* P1;
  const double* P2;
  const double* P3;
  const double* LF;
  int64_t k_min;
  double T;
};

template <int NP>
__global__ void k_psd_eval(int64_t nb, PsdBasis pb, const double* __restrict__ noise, int64_t P, int inverse,
                           double* __restrict__ S) {
  for (int64_t pc = blockIdx.y; pc < 2 * P; pc += gridDim.y) {
    const double* th = noise + NP * (pc >> 1);
    const double so = th[2 * (pc & 1)], sa = th[2 * (pc & 1) + 1];
    double* Sr = S + pc * nb;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += (int64_t)gridDim.x * blockDim.x) {
      double v = so * so * pb.P1[k] + sa * sa * pb.P2[k];
      if constexpr (NP == 9) v += foreground_term((double)(pb.k_min + k) / pb.T, pb.P3[k], pb.LF[k], th + 4);
      Sr[k] = inverse ? 1.0 / v : v;
    }
  }
}

// grid of the row kernels: bins of a row over x, rows over y
__host__ inline dim3 row_grid(int64_t n, int64_t rows) {
  const int64_t bx = (n + 255) / 256, cap = 1024;
  return dim3((unsigned)(bx < cap ? (bx > 0 ? bx : 1) : cap), (unsigned)(rows < cap ? (rows > 0 ? rows : 1) : cap));
}

constexpr int kPsdChunks = 256;
constexpr int kPsdBlock = 256;
constexpr int kPsdSets = 4;  // parameter sets per block of the PSD likelihood
constexpr double kLn2 = 0.69314718055994530942;

// partial sums over one chunk of bins for G parameter sets
// (sets p = p1st + blockIdx.y * G + s, s < G; p0 = first set of the workspace):
// work[p - p0][chunk] = (sum |R|^2/S, sum ln S) over both channels.  The sets of a
// block share each bin's PSD basis load; every set's sums run in the same order
// whatever G is, so the result does not depend on the grouping.
// Each S is split as m 2^e (m in [1/2, 1)): a bin's two quadratic terms take one
// division of m_A m_E, and a thread's ln S terms are one logarithm of the running
// mantissa product (renormalised every bin) plus ln 2 times the exponent sum.
// NP = 4 (instrument noise) or 9 (with the Galactic foreground, shared by A and E:
// one foreground evaluation per bin and set serves both channels).
template <int G, int NP>
__global__ __launch_bounds__(kPsdBlock) void k_psd_partial(int64_t nb, PsdBasis pb, const cd* __restrict__ residual,
                                                           int n_res, const double* __restrict__ noise,
                                                           const int32_t* __restrict__ res_idx, int64_t p0,
                                                           int64_t p1st, double* __restrict__ work, int map_nt,
                                                           int map_nw) {
  const int64_t pg = p1st + (int64_t)blockIdx.y * G;
  // set of slot s: pg + s, or with map_nt > 0 the batch's sets taken
  // walker-major (the batch holds map_nt x map_nw sets, temperature-major),
  // so that a block's sets share one residual row and read it once
  auto set_of = [&](int s) -> int64_t {
    const int64_t q = pg + s - p0;
    return map_nt > 0 ? p0 + (q % map_nt) * map_nw + q / map_nt : pg + s;
  };
  const int chunk = blockIdx.x;
  const int64_t cs = (nb + kPsdChunks - 1) / kPsdChunks;
  const int64_t lo = chunk * cs;
  const int64_t hi = lo + cs < nb ? lo + cs : nb;
  const cd* R[G];
  double oA[G], aA[G], oE[G], aE[G], quad[G], lm[G];
  double fg[NP == 9 ? G : 1][5];
  int le[G];
#pragma unroll
  for (int s = 0; s < G; s++) {
    const int64_t p = set_of(s);
    const int ri = res_idx[p];
    R[s] = residual + (int64_t)(ri >= 0 && ri < n_res ? ri : 0) * 2 * nb;  // a bad index reports NaN below
    oA[s] = noise[NP * p] * noise[NP * p];
    aA[s] = noise[NP * p + 1] * noise[NP * p + 1];
    oE[s] = noise[NP * p + 2] * noise[NP * p + 2];
    aE[s] = noise[NP * p + 3] * noise[NP * p + 3];
    if constexpr (NP == 9) {
#pragma unroll
      for (int i = 0; i < 5; i++) fg[s][i] = noise[NP * p + 4 + i];
    }
    quad[s] = 0.0;
    lm[s] = 1.0;
    le[s] = 0;
  }
  for (int64_t k = lo + threadIdx.x; k < hi; k += kPsdBlock) {
    const double p1 = pb.P1[k], p2 = pb.P2[k];
    double f = 0.0, p3 = 0.0, lf = 0.0;
    if constexpr (NP == 9) {
      f = (double)(pb.k_min + k) / pb.T;
      p3 = pb.P3[k];
      lf = pb.LF[k];
    }
#pragma unroll
    for (int s = 0; s < G; s++) {
      // explicit fma: the same rounding in every instance of G
      double SAv = fma(oA[s], p1, aA[s] * p2);
      double SEv = fma(oE[s], p1, aE[s] * p2);
      if constexpr (NP == 9) {
        const double gfg = foreground_term(f, p3, lf, fg[s]);
        SAv += gfg;
        SEv += gfg;
      }
      const cd r0 = R[s][k], r1 = R[s][nb + k];
      const double qa = fma(r0.re, r0.re, r0.im * r0.im), qe = fma(r1.re, r1.re, r1.im * r1.im);
      int eA, eE, eM;
      const double mA = frexp(SAv, &eA), mE = frexp(SEv, &eE);
      const double m = mA * mE;  // in [1/4, 1)
      quad[s] += fma(ldexp(qa, -eA), mE, ldexp(qe, -eE) * mA) / m;
      lm[s] = frexp(lm[s] * m, &eM);
      le[s] += eA + eE + eM;
    }
  }
  __shared__ double sq[G][kPsdBlock / kWave], sl[G][kPsdBlock / kWave];
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int s = 0; s < G; s++) {
    const double q = wave_sum(quad[s]), l = wave_sum(fma((double)le[s], kLn2, log(lm[s])));
    if ((threadIdx.x & (kWave - 1)) == 0) {
      sq[s][w] = q;
      sl[s][w] = l;
    }
  }
  __syncthreads();
  if (threadIdx.x < G) {
    const int s = threadIdx.x;
    const int64_t p = set_of(s);
    const int ri = res_idx[p];
    double a = 0.0, c = 0.0;
    for (int i = 0; i < kPsdBlock / kWave; i++) {
      a += sq[s][i];
      c += sl[s][i];
    }
    double* dst = work + 2 * ((p - p0) * kPsdChunks + chunk);
    dst[0] = ri >= 0 && ri < n_res ? a : qnan();
    dst[1] = c;
  }
}

__global__ __launch_bounds__(64) void k_psd_final(double df, const double* __restrict__ work, int64_t p0,
                                                  double* __restrict__ logl) {
  const int64_t pl = blockIdx.x;
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < kPsdChunks; i += kWave) {
    a += work[2 * (pl * kPsdChunks + i)];
    c += work[2 * (pl * kPsdChunks + i) + 1];
  }
  a = wave_sum(a);
  c = wave_sum(c);
  if (threadIdx.x == 0) logl[p0 + pl] = -2.0 * df * a - c;
}

__global__ void k_make_noise(int64_t total, double scale, const double* __restrict__ S,
                             const cd* __restrict__ normals, cd* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    double a = sqrt(S[i] * scale);
    cd gv = normals[i];
    out[i] = {a * gv.re, a * gv.im};
  }
}


// ---------------------------------------------------------------------------
// XCD-aware block order: the dispatcher deals workgroups round-robin to the
// eight XCDs, each with its own L2, so consecutive blocks run on different
// L2s.  The logical block index below gives each XCD one contiguous run of
// the grid instead (XCD x takes blocks x, x + 8, ...; with G = 8q + r blocks
// the first r XCDs take q + 1), so templates that are close in the batch, and
// share residual and PSD windows, also share an L2.  A bijection on [0, G).
// ---------------------------------------------------------------------------
constexpr unsigned kXcds = 8;

__device__ __forceinline__ unsigned xcd_block() {
  const unsigned G = gridDim.x, x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
  const unsigned q = G / kXcds, r = G % kXcds;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---------------------------------------------------------------------------
// gb_inner: PSD-weighted inner products of stored band slices (Sec. 2 eq.
// inner over channels A, E):
//   out[b] = (<h|h>, <R|h>) = 4 df sum_{c,k} (|h|^2, Re(conj(R) h)) / S
// over the slice's bins inside the band.  One wave per template: consecutive
// lanes read consecutive bins (16-byte loads of the slices and the residual,
// 8-byte loads of S), the sums stay in FP64 registers and one wave reduction
// finishes them.  Bound by HBM: 2 N (16 + 16 + 8) + 16 bytes per template.
// ---------------------------------------------------------------------------
constexpr int kInnerWaves = 4;  // templates per block

__global__ __launch_bounds__(kInnerWaves * kWave) void k_inner(Geo g, const cd* __restrict__ A,
                                                               const cd* __restrict__ E,
                                                               const int64_t* __restrict__ start, int N,
                                                               const cd* __restrict__ residual, int n_res,
                                                               const double* __restrict__ psd, int n_psd, int psd_inv,
                                                               const int32_t* __restrict__ res_idx,
                                                               const int32_t* __restrict__ psd_idx, int64_t B,
                                                               double* __restrict__ out) {
  const int64_t b = (int64_t)xcd_block() * kInnerWaves + threadIdx.x / kWave;
  if (b >= B) return;  // uniform over the wave
  const int lane = threadIdx.x & (kWave - 1);
  const int ri = res_idx[b], pi = psd_idx[b];
  if (ri < 0 || ri >= n_res || pi < 0 || pi >= n_psd) {
    if (lane == 0) out[2 * b] = out[2 * b + 1] = qnan();
    return;
  }
  const int64_t nb = g.n_bins;
  const int64_t s0 = start[b];
  // slice element j sits at band index s0 - k_min + j; only j in [jlo, jhi) is inside the band
  int64_t sb = 0, jlo = 0, jhi = 0;
  if (s0 > g.k_min - N && s0 < g.k_min + nb) {
    sb = s0 - g.k_min;
    jlo = sb < 0 ? -sb : 0;
    jhi = nb - sb < (int64_t)N ? nb - sb : (int64_t)N;
  }
  const cd* hA = A + b * N;
  const cd* hE = E + b * N;
  const cd* RA = residual + (int64_t)ri * 2 * nb;
  const cd* RE = RA + nb;
  const double* SA = psd + (int64_t)pi * 2 * nb;
  const double* SE = SA + nb;
  double hh = 0.0, rh = 0.0;
#pragma unroll 4
  for (int64_t j = jlo + lane; j < jhi; j += kWave) {
    const int64_t k = sb + j;
    const cd a = hA[j], e = hE[j], ra = RA[k], re = RE[k];
    const double sa = SA[k], se = SE[k];
    const double wa = psd_inv ? sa : 1.0 / sa;
    const double we = psd_inv ? se : 1.0 / se;
    hh += fma(a.re, a.re, a.im * a.im) * wa + fma(e.re, e.re, e.im * e.im) * we;
    rh += fma(ra.re, a.re, ra.im * a.im) * wa + fma(re.re, e.re, re.im * e.im) * we;
  }
  hh = wave_sum(hh);
  rh = wave_sum(rh);
  if (lane == 0) {
    out[2 * b] = g.df4 * hh;
    out[2 * b + 1] = g.df4 * rh;
  }
}

// ---------------------------------------------------------------------------
// gb_snr: optimal SNR sqrt(<h|h>) and observed SNR <d|h>/sqrt(<h|h>) of
// templates built on the fly (one block per template, FP64 response; the
// template never leaves LDS).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_snr(Geo g, WaveTables<double> tb,
                                                            const double* __restrict__ params, int64_t b0,
                                                            const double* __restrict__ psd, int n_psd, int psd_inv,
                                                            const int32_t* __restrict__ psd_idx,
                                                            const cd* __restrict__ data, int n_data,
                                                            const int32_t* __restrict__ data_idx,
                                                            double* __restrict__ snr_opt,
                                                            double* __restrict__ snr_obs) {
  constexpr int NT = block_threads<N>();
  constexpr int NW = NT / kWave;
  __shared__ cd buf[4 * series_pitch<N>()];
  __shared__ Src s_sh;
  __shared__ double red[2][NW];
  const int64_t b = b0 + blockIdx.x;
  const int tid = threadIdx.x;
  const SrcHead h = source_head(params + 8 * b, g);
  const int pi = psd_idx[b];
  const int di = data ? data_idx[b] : 0;
  if (h.state == 2 || pi < 0 || pi >= n_psd || (data && (di < 0 || di >= n_data))) {
    if (tid == 0) {
      snr_opt[b] = qnan();
      if (data) snr_obs[b] = qnan();
    }
    return;  // uniform over the block
  }
  double hh = 0.0, dh = 0.0;
  if (h.state == 0) {
    if (tid < kWave) decode_sources<1>(params + 8 * b, params + 8 * b, g, &s_sh);
    __syncthreads();
    const Src& s = s_sh;
    template_transform<N, 4, double>(s, g, tb, buf, tid);
    const int64_t nb = g.n_bins;
    const int64_t k0 = s.q - N / 2;
    const double* S = psd + (int64_t)pi * 2 * nb;
    const cd* D = data ? data + (int64_t)di * 2 * nb : nullptr;
    for (int j = tid; j < N; j += NT) {
      const int64_t k = k0 + j;
      if (k < g.k_min || k >= g.k_min + nb) continue;
      const int64_t idx = k - g.k_min;
      cd v[2];
      bin_spectrum<N, 2, double>(s, g, tb, buf, j, v);
#pragma unroll
      for (int c = 0; c < 2; c++) {
        const double sv = S[c * nb + idx];
        const double w = psd_inv ? sv : 1.0 / sv;
        hh += fma(v[c].re, v[c].re, v[c].im * v[c].im) * w;
        if (D) {
          const cd dv = D[c * nb + idx];
          dh += fma(dv.re, v[c].re, dv.im * v[c].im) * w;
        }
      }
    }
  }
  // state 1 (zero amplitude): both sums are exactly zero
  hh = wave_sum(hh);
  dh = wave_sum(dh);
  if ((tid & (kWave - 1)) == 0) {
    red[0][tid / kWave] = hh;
    red[1][tid / kWave] = dh;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      a += red[0][i];
      c += red[1][i];
    }
    a *= g.df4;
    c *= g.df4;
    const double so = sqrt(a);
    snr_opt[b] = so;
    if (data) snr_obs[b] = c / so;
  }
}

// ---------------------------------------------------------------------------
// gb_overlap: (<a|a>, <b|b>, <a|b>, <a|b> / sqrt(<a|a> <b|b>)) of template
// pairs (the overlaps that group sources in the cataloging operation of
// Sec. 4).  One block per pair, FP64: a's spectrum is kept in LDS, b is built
// in the FFT workspace and every bin of b's window adds to <b|b> and, where
// a's window covers it, to <a|b>; a's own bins give <a|a>.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_overlap(Geo g, WaveTables<double> tb,
                                                                const double* __restrict__ pa,
                                                                const double* __restrict__ pb, int64_t b0,
                                                                const double* __restrict__ psd, int n_psd,
                                                                int psd_inv, const int32_t* __restrict__ psd_idx,
                                                                double* __restrict__ out) {
  constexpr int NT = block_threads<N>();
  constexpr int NW = NT / kWave;
  __shared__ cd buf[4 * series_pitch<N>()];
  __shared__ cd aw[2 * N];
  __shared__ Src src;
  __shared__ double red[3][NW];
  const int64_t b = b0 + blockIdx.x;
  const int tid = threadIdx.x;
  const double* prm_a = pa + 8 * b;
  const double* prm_b = pb + 8 * b;
  const SrcHead ha = source_head(prm_a, g), hb = source_head(prm_b, g);
  const int pi = psd_idx[b];
  if (ha.state == 2 || hb.state == 2 || pi < 0 || pi >= n_psd) {
    if (tid == 0) out[4 * b] = out[4 * b + 1] = out[4 * b + 2] = out[4 * b + 3] = qnan();
    return;  // uniform over the block
  }
  const int64_t nb = g.n_bins;
  const double* S = psd + (int64_t)pi * 2 * nb;
  const int64_t ka = ha.q - N / 2, kb = hb.q - N / 2;
  // template a into aw (zeros for a zero-amplitude template)
  if (ha.state == 0) {
    if (tid < kWave) decode_sources<1>(prm_a, prm_a, g, &src);
    __syncthreads();
    template_transform<N, 4, double>(src, g, tb, buf, tid);
    for (int j = tid; j < N; j += NT) {
      cd v[2];
      bin_spectrum<N, 2, double>(src, g, tb, buf, j, v);
      aw[j] = v[0];
      aw[N + j] = v[1];
    }
  } else {
    for (int j = tid; j < 2 * N; j += NT) aw[j] = cd{0.0, 0.0};
  }
  __syncthreads();  // aw complete; the workspace and the decode are free again
  double aa = 0.0, bb = 0.0, ab = 0.0;
  for (int j = tid; j < N; j += NT) {
    const int64_t k = ka + j;
    if (k < g.k_min || k >= g.k_min + nb) continue;
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const double sv = S[c * nb + (k - g.k_min)];
      const double w = psd_inv ? sv : 1.0 / sv;
      const cd x = aw[c * N + j];
      aa += fma(x.re, x.re, x.im * x.im) * w;
    }
  }
  if (hb.state == 0) {
    if (tid < kWave) decode_sources<1>(prm_b, prm_b, g, &src);
    __syncthreads();
    template_transform<N, 4, double>(src, g, tb, buf, tid);
    for (int j = tid; j < N; j += NT) {
      const int64_t k = kb + j;
      if (k < g.k_min || k >= g.k_min + nb) continue;
      cd v[2];
      bin_spectrum<N, 2, double>(src, g, tb, buf, j, v);
      const int64_t ja = k - ka;
      const bool in_a = ja >= 0 && ja < N;
#pragma unroll
      for (int c = 0; c < 2; c++) {
        const double sv = S[c * nb + (k - g.k_min)];
        const double w = psd_inv ? sv : 1.0 / sv;
        bb += fma(v[c].re, v[c].re, v[c].im * v[c].im) * w;
        if (in_a) {
          const cd x = aw[c * N + ja];
          ab += fma(x.re, v[c].re, x.im * v[c].im) * w;
        }
      }
    }
  }
  aa = wave_sum(aa);
  bb = wave_sum(bb);
  ab = wave_sum(ab);
  if ((tid & (kWave - 1)) == 0) {
    red[0][tid / kWave] = aa;
    red[1][tid / kWave] = bb;
    red[2][tid / kWave] = ab;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      s0 += red[0][i];
      s1 += red[1][i];
      s2 += red[2][i];
    }
    s0 *= g.df4;
    s1 *= g.df4;
    s2 *= g.df4;
    out[4 * b] = s0;
    out[4 * b + 1] = s1;
    out[4 * b + 2] = s2;
    out[4 * b + 3] = s2 / sqrt(s0 * s1);
  }
}

// ---------------------------------------------------------------------------
// Deterministic scatter-add (GBL_DETERMINISTIC contexts).  A chunk of
// templates is built into a workspace, sorted by (residual, start bin) with a
// stable radix sort (ties keep template order), and every band bin is
// written by exactly one thread: the first sorted template that covers it
// sums, in sorted order, every template covering the bin and adds the total
// with a plain read-modify-write.  No atomics, so the residual does not
// depend on scheduling.
// ---------------------------------------------------------------------------
constexpr uint64_t kDetInvalid = ~0ull;

// key = res_idx << 32 | (start - k_min + N): templates that miss the band,
// zero or undefined templates and bad indices get kDetInvalid (sorted last)
__global__ void k_det_keys(Geo g, const double* __restrict__ params, int64_t b0, int64_t nb, int N,
                           const int32_t* __restrict__ res_idx, int n_res, uint64_t* __restrict__ keys,
                           int32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int64_t b = b0 + i;
  const SrcHead h = source_head(params + 8 * b, g);
  const int ri = res_idx[b];
  const int64_t start = h.q - N / 2;
  const bool ok = h.state == 0 && ri >= 0 && ri < n_res && start + N > g.k_min && start < g.k_min + g.n_bins;
  keys[i] = ok ? ((uint64_t)ri << 32) | (uint64_t)(start - g.k_min + N) : kDetInvalid;
  vals[i] = (int32_t)i;
}

// template b0 + blockIdx.x into workspace slot blockIdx.x (A at ws, E at ws + cap)
template <int N, typename F>
__global__ __launch_bounds__(block_threads<N>()) void k_det_slices(Geo g, WaveTables<F> tb,
                                                                   const double* __restrict__ params, int64_t b0,
                                                                   cd* __restrict__ ws, int64_t cap,
                                                                   int64_t* __restrict__ ws_start) {
  __shared__ WaveSmem<N, 4, F> sm;
  const int64_t i = blockIdx.x;
  waveform_one<N, 4, F>(g, tb, params + 8 * (b0 + i), i * N, ws, ws + cap, nullptr, ws_start + i, sm);
}

template <int N>
__global__ __launch_bounds__(256) void k_det_gather(Geo g, const uint64_t* __restrict__ keys,
                                                    const int32_t* __restrict__ vals, int64_t nb,
                                                    const cd* __restrict__ ws, int64_t cap, double sign,
                                                    cd* __restrict__ residual) {
  const int64_t i = blockIdx.x;
  const uint64_t key = keys[i];
  if (key == kDetInvalid) return;
  const uint64_t ri = key >> 32;
  const int64_t start = (int64_t)(key & 0xffffffffull) + g.k_min - N;
  const bool first_of_row = i == 0 || (keys[i - 1] >> 32) != ri;
  const int64_t prev_end = first_of_row ? INT64_MIN : (int64_t)(keys[i - 1] & 0xffffffffull) + g.k_min;  // start + N
  cd* R = residual + (int64_t)ri * 2 * g.n_bins;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const int64_t k = start + j;
    if (k < g.k_min || k >= g.k_min + g.n_bins) continue;
    if (prev_end > k) continue;  // an earlier sorted template covers k and owns it
    cd sa = {0.0, 0.0}, se = {0.0, 0.0};
    for (int64_t i2 = i; i2 < nb; i2++) {
      const uint64_t k2 = keys[i2];
      if ((k2 >> 32) != ri) break;  // also stops at kDetInvalid (ri < 2^31)
      const int64_t s2 = (int64_t)(k2 & 0xffffffffull) + g.k_min - N;
      if (s2 > k) break;
      const int64_t slot = vals[i2];
      const cd a = ws[slot * N + (k - s2)], e = ws[cap + slot * N + (k - s2)];
      sa.re += a.re;
      sa.im += a.im;
      se.re += e.re;
      se.im += e.im;
    }
    const int64_t idx = k - g.k_min;
    cd ra = R[idx], re = R[g.n_bins + idx];
    ra.re += sign * sa.re;
    ra.im += sign * sa.im;
    re.re += sign * se.re;
    re.im += sign * se.im;
    R[idx] = ra;
    R[g.n_bins + idx] = re;
  }
}

}  // namespace gbl
