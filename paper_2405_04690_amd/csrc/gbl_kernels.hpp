// gbl_kernels.hpp -- HIP kernels of the GB likelihood library (gfx950).
#pragma once

#include "gbl_device.hpp"

namespace gbl {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double qnan() { return __builtin_nan(""); }

// ---------------------------------------------------------------------------
// Table construction (once per context)
// ---------------------------------------------------------------------------
__global__ void k_init_wave_tables(int N, double T, double Lc, double* basis, cd* fft_tw, cd* bin_F, cd* bin_E) {
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
  sincos(-kTwoPi * (double)k * Lc / T, &s, &c);
  bin_E[n] = {c, s};
}

// PSD basis of eq. psd, linear in (S_oms, S_acc):  S_n = S_oms P1 + S_acc P2,
//   P1 = 8 sin^2 x (2 + cos x) (2 pi f/c)^2 [1 + (2 mHz/f)^4]
//   P2 = 16 sin^2 x (3 + 2 cos x + cos 2x) (2 pi c f)^-2 [1 + (0.4 mHz/f)^2][1 + (f/8 mHz)^4]
__global__ void k_init_psd_basis(int64_t k_min, int64_t nb, double T, double L, double* P1, double* P2) {
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
// gb_waveform: one block per template; writes A, E (and T) band slices.
// ---------------------------------------------------------------------------
template <int N, int NSER>
__global__ __launch_bounds__(block_threads<N>()) void k_waveform(Geo g, WaveTables tb,
                                                                 const double* __restrict__ params, int64_t b0,
                                                                 cd* __restrict__ A, cd* __restrict__ E,
                                                                 cd* __restrict__ Tc, int64_t* __restrict__ start) {
  constexpr int NT = block_threads<N>();
  __shared__ cd buf[NSER * series_pitch<N>()];
  __shared__ Src s_sh;
  const int64_t b = b0 + blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < kWave) {  // one wave decodes, the block shares the result
    Src d = decode_source(params + 8 * b, g);
    if (tid == 0) s_sh = d;
  }
  __syncthreads();
  const Src& s = s_sh;
  if (s.state == 0) template_transform<N, NSER>(s, g, tb, buf, tid);
  cd* outs[3] = {A, E, Tc};
#pragma unroll
  for (int c = 0; c < NSER / 2; c++) {
    for (int j = tid; j < N; j += NT) {
      cd v;
      if (s.state == 0)
        v = bin_value<N>(s, tb, buf, c, j);
      else if (s.state == 1)
        v = {0.0, 0.0};
      else
        v = {qnan(), qnan()};
      outs[c][b * N + j] = v;
    }
  }
  if (tid == 0) start[b] = (s.state == 2) ? 0 : s.q - N / 2;
}

// ---------------------------------------------------------------------------
// gb_delta_loglike (FP64): one block per (old, new) pair.  The old template r
// goes into an LDS window, the new template a through the FFT workspace, then
//   dlogl = 4 df [ sum Re(conj R) d / S - 1/2 sum |d|^2 / S ],  d = a - r,
// over the union of the two windows clipped to the band (channels A, E).
// The residual and PSD values of a's window are fetched before the templates
// are built, so their HBM latency overlaps the arithmetic.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_delta_loglike(
    Geo g, WaveTables tb, const cd* __restrict__ residual, int n_res, const double* __restrict__ psd, int n_psd,
    int psd_inv, const double* __restrict__ p_old, const double* __restrict__ p_new,
    const int32_t* __restrict__ res_idx, const int32_t* __restrict__ psd_idx, int64_t b0, double* __restrict__ out) {
  constexpr int NT = block_threads<N>();
  constexpr int BPT = N / NT;  // window bins per thread
  constexpr int SP = series_pitch<N>();
  __shared__ cd buf[4 * SP];
  __shared__ cd rwin[2 * N];
  __shared__ double red[2 * (NT / kWave)];
  __shared__ Src src_sh[2];  // 0: old, 1: new
  const int64_t b = b0 + blockIdx.x;
  const int tid = threadIdx.x;
  // validity and carrier bins first; each source is fully decoded only when
  // its template is built, which keeps one decoded source live at a time
  const SrcHead ho = source_head(p_old + 8 * b, g);
  const SrcHead hn = source_head(p_new + 8 * b, g);
  const int ri = res_idx[b];
  const int pi = psd_idx[b];
  if (ho.state == 2 || hn.state == 2 || ri < 0 || ri >= n_res || pi < 0 || pi >= n_psd) {
    if (tid == 0) out[b] = qnan();
    return;  // uniform over the block
  }
  const int64_t nb = g.n_bins;
  const cd* RA = residual + (int64_t)ri * 2 * nb;
  const cd* RE = RA + nb;
  const double* SA = psd + (int64_t)pi * 2 * nb;
  const double* SE = SA + nb;
  const int64_t ka = hn.q - N / 2;
  const int64_t kr = ho.q - N / 2;

  auto weight = [&](const double* Sc, int64_t idx) { return psd_inv ? Sc[idx] : 1.0 / Sc[idx]; };

  // wave 0 decodes the old source, wave 1 the new one; the block shares them
  if (tid < 2 * kWave) {
    const int which = tid / kWave;
    Src d = decode_source((which ? p_new : p_old) + 8 * b, g);
    if ((tid & (kWave - 1)) == 0) src_sh[which] = d;
  }

  // prefetch residual and weights over a's window
  cd pR0[BPT], pR1[BPT];
  double pW0[BPT], pW1[BPT];
  if (hn.state == 0) {
#pragma unroll
    for (int m = 0; m < BPT; m++) {
      int64_t k = ka + tid + NT * m;
      if (k >= g.k_min && k < g.k_min + nb) {
        int64_t idx = k - g.k_min;
        pR0[m] = RA[idx];
        pR1[m] = RE[idx];
        pW0[m] = weight(SA, idx);
        pW1[m] = weight(SE, idx);
      }
    }
  }

  __syncthreads();

  // old template into the LDS window
  if (ho.state == 0) {
    const Src& so = src_sh[0];
    template_transform<N, 4>(so, g, tb, buf, tid);
    for (int j = tid; j < N; j += NT) {
      rwin[j] = bin_value<N>(so, tb, buf, 0, j);
      rwin[N + j] = bin_value<N>(so, tb, buf, 1, j);
    }
  }
  __syncthreads();

  double acc_rd = 0.0, acc_dd = 0.0;
  auto accumulate = [&](cd R0, cd R1, double w0, double w1, cd d0, cd d1) {
    acc_rd += (R0.re * d0.re + R0.im * d0.im) * w0 + (R1.re * d1.re + R1.im * d1.im) * w1;
    acc_dd += (d0.re * d0.re + d0.im * d0.im) * w0 + (d1.re * d1.re + d1.im * d1.im) * w1;
  };

  if (hn.state == 0) {
    const Src& sn = src_sh[1];
    template_transform<N, 4>(sn, g, tb, buf, tid);
#pragma unroll
    for (int m = 0; m < BPT; m++) {
      const int j = tid + NT * m;
      int64_t k = ka + j;
      if (k < g.k_min || k >= g.k_min + nb) continue;
      cd a0 = bin_value<N>(sn, tb, buf, 0, j);
      cd a1 = bin_value<N>(sn, tb, buf, 1, j);
      int64_t jr = k - kr;
      if (ho.state == 0 && jr >= 0 && jr < N) {
        a0 = a0 - rwin[jr];
        a1 = a1 - rwin[N + jr];
      }
      accumulate(pR0[m], pR1[m], pW0[m], pW1[m], a0, a1);
    }
  }
  if (ho.state == 0) {
    // bins of r's window not already covered by a's window
    for (int j = tid; j < N; j += NT) {
      int64_t k = kr + j;
      if (hn.state == 0 && k >= ka && k < ka + N) continue;
      if (k < g.k_min || k >= g.k_min + nb) continue;
      int64_t idx = k - g.k_min;
      cd r0 = rwin[j], r1 = rwin[N + j];
      accumulate(RA[idx], RE[idx], weight(SA, idx), weight(SE, idx), cd{-r0.re, -r0.im}, cd{-r1.re, -r1.im});
    }
  }
  acc_rd = block_sum<NT>(acc_rd, red);
  acc_dd = block_sum<NT>(acc_dd, red + NT / kWave);
  if (tid == 0) out[b] = g.df4 * acc_rd - 0.5 * g.df4 * acc_dd;
}

// ---------------------------------------------------------------------------
// gb_scatter_add: residual[res_idx[b]] += sign * template b (A, E), FP64 atomics.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_scatter_add(Geo g, WaveTables tb,
                                                                    const double* __restrict__ params, int64_t b0,
                                                                    double sign, cd* residual, int n_res,
                                                                    const int32_t* __restrict__ res_idx) {
  constexpr int NT = block_threads<N>();
  __shared__ cd buf[4 * series_pitch<N>()];
  __shared__ Src s_sh;
  const int64_t b = b0 + blockIdx.x;
  const int tid = threadIdx.x;
  const SrcHead h = source_head(params + 8 * b, g);
  const int ri = res_idx[b];
  if (h.state != 0 || ri < 0 || ri >= n_res) return;  // zero or invalid templates add nothing
  if (tid < kWave) {
    Src d = decode_source(params + 8 * b, g);
    if (tid == 0) s_sh = d;
  }
  __syncthreads();
  const Src& s = s_sh;
  template_transform<N, 4>(s, g, tb, buf, tid);
  const int64_t nb = g.n_bins;
  const int64_t k0 = s.q - N / 2;
  cd* R = residual + (int64_t)ri * 2 * nb;
  for (int j = tid; j < N; j += NT) {
    int64_t k = k0 + j;
    if (k < g.k_min || k >= g.k_min + nb) continue;
    int64_t idx = k - g.k_min;
#pragma unroll
    for (int c = 0; c < 2; c++) {
      cd v = bin_value<N>(s, tb, buf, c, j);
      double* dst = reinterpret_cast<double*>(R + c * nb + idx);
      atomicAdd(dst, sign * v.re);
      atomicAdd(dst + 1, sign * v.im);
    }
  }
}

// ---------------------------------------------------------------------------
// PSD evaluation and the noise-parameter log-likelihood
// ---------------------------------------------------------------------------
__global__ void k_psd_eval(int64_t nb, const double* __restrict__ P1, const double* __restrict__ P2,
                           const double* __restrict__ noise, int64_t P, int inverse, double* __restrict__ S) {
  int64_t total = P * 2 * nb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = i % nb;
    int64_t pc = i / nb;  // p * 2 + c
    double so = noise[2 * pc], sa = noise[2 * pc + 1];
    double v = so * so * P1[k] + sa * sa * P2[k];
    S[i] = inverse ? 1.0 / v : v;
  }
}

constexpr int kPsdChunks = 256;
constexpr int kPsdBlock = 256;

// partial sums over one chunk of bins for one parameter set:
// work[p][chunk] = (sum |R|^2/S, sum ln S) over both channels
__global__ __launch_bounds__(kPsdBlock) void k_psd_partial(int64_t nb, const double* __restrict__ P1,
                                                           const double* __restrict__ P2,
                                                           const cd* __restrict__ residual, int n_res,
                                                           const double* __restrict__ noise,
                                                           const int32_t* __restrict__ res_idx, int64_t p0,
                                                           double* __restrict__ work) {
  const int64_t p = p0 + blockIdx.y;
  const int chunk = blockIdx.x;
  const int64_t cs = (nb + kPsdChunks - 1) / kPsdChunks;
  const int64_t lo = chunk * cs;
  const int64_t hi = lo + cs < nb ? lo + cs : nb;
  const int ri = res_idx[p];
  double quad = 0.0, lg = 0.0;
  if (ri >= 0 && ri < n_res) {
    const cd* R = residual + (int64_t)ri * 2 * nb;
    const double oA = noise[4 * p] * noise[4 * p], aA = noise[4 * p + 1] * noise[4 * p + 1];
    const double oE = noise[4 * p + 2] * noise[4 * p + 2], aE = noise[4 * p + 3] * noise[4 * p + 3];
    for (int64_t k = lo + threadIdx.x; k < hi; k += kPsdBlock) {
      double p1 = P1[k], p2 = P2[k];
      double SAv = oA * p1 + aA * p2;
      double SEv = oE * p1 + aE * p2;
      cd r0 = R[k], r1 = R[nb + k];
      quad += (r0.re * r0.re + r0.im * r0.im) / SAv + (r1.re * r1.re + r1.im * r1.im) / SEv;
      lg += log(SAv) + log(SEv);
    }
  } else {
    quad = qnan();
  }
  __shared__ double sq[kPsdBlock / kWave], sl[kPsdBlock / kWave];
  quad = wave_sum(quad);
  lg = wave_sum(lg);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sq[w] = quad;
    sl[w] = lg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < kPsdBlock / kWave; i++) {
      a += sq[i];
      c += sl[i];
    }
    double* dst = work + 2 * ((p - p0) * kPsdChunks + chunk);
    dst[0] = a;
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

}  // namespace gbl
