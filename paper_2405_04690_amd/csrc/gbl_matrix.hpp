// gbl_matrix.hpp -- correlated A/E channels (Sec. 2: with unequal noise in
// the links the A and E channels correlate, and the likelihood needs the
// noise matrix across channels).
//
// Noise model: twelve independent noises, the metrology noise of each of the
// six links and the Doppler noise of each of the six test masses, with the
// spectral shapes of eq. psd; a link y_{s->r} carries o_{sr} + delta_{rs} +
// D delta_{sr} (D = exp(-i x), x = 2 pi f L / c); the first-generation
// Michelson combinations X, Y, Z and A = (Z - X)/sqrt 2, E = (X - 2Y + Z)/sqrt 6
// carry each noise with a coefficient, and C = sum_j c_j c_j^H S_j.
// Per bin the kernels store K = C^-1 as (K_AA, K_EE, Re K_AE, Im K_AE) and
// ln det C; the inner product is 4 df Re sum a^H K b.
#pragma once

#include "gbl_kernels.hpp"

namespace gbl {

struct NoiseLevels {
  double v[12];  // sqrt S_oms of links 0->1, 0->2, 1->0, 1->2, 2->0, 2->1; sqrt S_acc of masses (0,1) .. (2,1)
};

// index of the directed pair (s, r), s != r, in the order above
__device__ __forceinline__ int pair_index(int s, int r) { return 2 * s + (r > s ? r - 1 : r); }

// coefficient of noise j in the Michelson combination at vertex v with arms
// to b1 and b2: (1 - D^2)[(y_{b1->v} + D y_{v->b1}) - (y_{b2->v} + D y_{v->b2})]
__device__ __forceinline__ void michelson_coefs(int v, int b1, int b2, cd D, cd* c /*[12]*/) {
#pragma unroll
  for (int j = 0; j < 12; j++) c[j] = cd{0.0, 0.0};
  const cd D2 = D * D;
  const cd f = cd{1.0 - D2.re, -D2.im};
  // y_{s->r} contributes (metrology o_{sr}: 1, mass delta_{rs}: 1, mass delta_{sr}: D) times w
  auto add_link = [&](int s, int r, cd w) {
    c[pair_index(s, r)] = c[pair_index(s, r)] + w;
    c[6 + pair_index(r, s)] = c[6 + pair_index(r, s)] + w;
    c[6 + pair_index(s, r)] = c[6 + pair_index(s, r)] + w * D;
  };
  add_link(b1, v, f);
  add_link(v, b1, f * D);
  add_link(b2, v, cd{-f.re, -f.im});
  add_link(v, b2, cd{-(f * D).re, -(f * D).im});
}

// rows pc = p over blockIdx.y, bins over blockIdx.x (grid-stride)
__global__ void k_noise_matrix(int64_t nb, int64_t k_min, double T, double L, const NoiseLevels* __restrict__ lv,
                               int64_t P, double* __restrict__ out) {
  for (int64_t p = blockIdx.y; p < P; p += gridDim.y) {
    const NoiseLevels lev = lv[p];
    double* o = out + p * 5 * nb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
      const double f = (double)(k_min + i) / T;
      double sx, cx_;
      sincos(kTwoPi * f * L / kC, &sx, &cx_);
      const cd D{cx_, -sx};
      cd X[12], Y[12], Z[12];
      michelson_coefs(0, 1, 2, D, X);
      michelson_coefs(1, 2, 0, D, Y);
      michelson_coefs(2, 0, 1, D, Z);
      const double wo = kTwoPi * f / kC, wa = kTwoPi * kC * f;
      const double ro = 2e-3 / f, ra = 0.4e-3 / f, rh = f / 8e-3;
      const double shape_o = wo * wo * (1.0 + ro * ro * ro * ro);
      const double shape_a = (1.0 + ra * ra) * (1.0 + rh * rh * rh * rh) / (wa * wa);
      double caa = 0.0, cee = 0.0;
      cd cae{0.0, 0.0};
#pragma unroll
      for (int j = 0; j < 12; j++) {
        const double S = lev.v[j] * lev.v[j] * (j < 6 ? shape_o : shape_a);
        const cd a{(Z[j].re - X[j].re) * kInvSqrt2, (Z[j].im - X[j].im) * kInvSqrt2};
        const cd e{(X[j].re - 2.0 * Y[j].re + Z[j].re) * kInvSqrt6, (X[j].im - 2.0 * Y[j].im + Z[j].im) * kInvSqrt6};
        caa += (a.re * a.re + a.im * a.im) * S;
        cee += (e.re * e.re + e.im * e.im) * S;
        // a conj(e)
        cae.re += (a.re * e.re + a.im * e.im) * S;
        cae.im += (a.im * e.re - a.re * e.im) * S;
      }
      const double det = caa * cee - (cae.re * cae.re + cae.im * cae.im);
      o[i] = cee / det;
      o[nb + i] = caa / det;
      o[2 * nb + i] = -cae.re / det;
      o[3 * nb + i] = -cae.im / det;
      o[4 * nb + i] = log(det);
    }
  }
}

// Re(x^H K y) for two-channel values at one bin, K = (kaa, kee, kae)
__device__ __forceinline__ double mat_form(const cd x0, const cd x1, double kaa, double kee, cd kae, const cd y0,
                                           const cd y1) {
  // K y = (kaa y0 + kae y1, conj(kae) y0 + kee y1)
  const cd k0{kaa * y0.re + kae.re * y1.re - kae.im * y1.im, kaa * y0.im + kae.re * y1.im + kae.im * y1.re};
  const cd k1{kae.re * y0.re + kae.im * y0.im + kee * y1.re, kae.re * y0.im - kae.im * y0.re + kee * y1.im};
  return x0.re * k0.re + x0.im * k0.im + x1.re * k1.re + x1.im * k1.im;
}

// ---------------------------------------------------------------------------
// Swap likelihood with the channel matrix (eq. swapsource in the matrix inner
// product): dlogl = <R|a - r>_K - 1/2 <a - r|a - r>_K.  One block per pair,
// FP64: r's spectrum parked in LDS, a built in the FFT workspace, the sums over
// the union of the two windows clipped to the band.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_delta_loglike_mat(
    Geo g, WaveTables<double> tb, const cd* __restrict__ residual, int n_res, const double* __restrict__ Kmat, int n_K,
    const double* __restrict__ p_old, const double* __restrict__ p_new, const int32_t* __restrict__ res_idx,
    const int32_t* __restrict__ k_idx, int64_t b0, double* __restrict__ out) {
  constexpr int NT = block_threads<N>();
  constexpr int NW = NT / kWave;
  __shared__ cd buf[4 * series_pitch<N>()];
  __shared__ cd rw[2 * N];
  __shared__ Src src;
  __shared__ double red[2][NW];
  const int64_t b = b0 + blockIdx.x;
  const int tid = threadIdx.x;
  const double* po = p_old + 8 * b;
  const double* pn = p_new + 8 * b;
  const SrcHead ho = source_head(po, g), hn = source_head(pn, g);
  const int ri = res_idx[b], ki = k_idx[b];
  if (ho.state == 2 || hn.state == 2 || ri < 0 || ri >= n_res || ki < 0 || ki >= n_K) {
    if (tid == 0) out[b] = qnan();
    return;  // uniform over the block
  }
  const int64_t nb = g.n_bins;
  const cd* R = residual + (int64_t)ri * 2 * nb;
  const double* K = Kmat + (int64_t)ki * 5 * nb;
  const int64_t kr = ho.q - N / 2, ka = hn.q - N / 2;
  // r into rw (zeros for a zero-amplitude template)
  if (ho.state == 0) {
    if (tid < kWave) decode_sources<1>(po, po, g, &src);
    __syncthreads();
    template_transform<N, 4, double>(src, g, tb, buf, tid);
    for (int j = tid; j < N; j += NT) {
      cd v[2];
      bin_spectrum<N, 2, double>(src, g, tb, buf, j, v);
      rw[j] = v[0];
      rw[N + j] = v[1];
    }
  } else {
    for (int j = tid; j < 2 * N; j += NT) rw[j] = cd{0.0, 0.0};
  }
  __syncthreads();
  double rd = 0.0, dd = 0.0;
  auto acc = [&](int64_t k, cd d0, cd d1) {
    const int64_t i = k - g.k_min;
    const double kaa = K[i], kee = K[nb + i];
    const cd kae{K[2 * nb + i], K[3 * nb + i]};
    rd += mat_form(R[i], R[nb + i], kaa, kee, kae, d0, d1);
    dd += mat_form(d0, d1, kaa, kee, kae, d0, d1);
  };
  if (hn.state == 0) {
    if (tid < kWave) decode_sources<1>(pn, pn, g, &src);
    __syncthreads();
    template_transform<N, 4, double>(src, g, tb, buf, tid);
    for (int j = tid; j < N; j += NT) {
      const int64_t k = ka + j;
      if (k < g.k_min || k >= g.k_min + nb) continue;
      cd v[2];
      bin_spectrum<N, 2, double>(src, g, tb, buf, j, v);
      const int64_t jr = k - kr;
      if (jr >= 0 && jr < N) {
        v[0] = v[0] - rw[jr];
        v[1] = v[1] - rw[N + jr];
      }
      acc(k, v[0], v[1]);
    }
  }
  // r's bins outside a's window
  for (int j = tid; j < N; j += NT) {
    const int64_t k = kr + j;
    if (hn.state == 0 && k >= ka && k < ka + N) continue;
    if (k < g.k_min || k >= g.k_min + nb) continue;
    acc(k, cd{-rw[j].re, -rw[j].im}, cd{-rw[N + j].re, -rw[N + j].im});
  }
  rd = wave_sum(rd);
  dd = wave_sum(dd);
  if ((tid & (kWave - 1)) == 0) {
    red[0][tid / kWave] = rd;
    red[1][tid / kWave] = dd;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      a += red[0][i];
      c += red[1][i];
    }
    out[b] = g.df4 * a - 0.5 * g.df4 * c;
  }
}

// ---------------------------------------------------------------------------
// Log-likelihood with the channel matrix: -1/2 <R|R>_K - sum ln det C, as
// fixed-order partial sums per (set, chunk of bins) and a final sum per set.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPsdBlock) void k_loglike_mat_partial(int64_t nb, const cd* __restrict__ residual,
                                                                   int n_res, const double* __restrict__ Kmat,
                                                                   int n_K, const int32_t* __restrict__ res_idx,
                                                                   const int32_t* __restrict__ k_idx, int64_t p0,
                                                                   double* __restrict__ work) {
  const int64_t p = p0 + blockIdx.y;
  const int chunk = blockIdx.x;
  const int ri = res_idx[p], ki = k_idx[p];
  const bool ok = ri >= 0 && ri < n_res && ki >= 0 && ki < n_K;
  const cd* R = residual + (int64_t)(ok ? ri : 0) * 2 * nb;
  const double* K = Kmat + (int64_t)(ok ? ki : 0) * 5 * nb;
  const int64_t cs = (nb + kPsdChunks - 1) / kPsdChunks;
  const int64_t lo = chunk * cs;
  const int64_t hi = lo + cs < nb ? lo + cs : nb;
  double q = 0.0, l = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPsdBlock) {
    const cd kae{K[2 * nb + i], K[3 * nb + i]};
    q += mat_form(R[i], R[nb + i], K[i], K[nb + i], kae, R[i], R[nb + i]);
    l += K[4 * nb + i];
  }
  __shared__ double sq[kPsdBlock / kWave], sl[kPsdBlock / kWave];
  q = wave_sum(q);
  l = wave_sum(l);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sq[threadIdx.x / kWave] = q;
    sl[threadIdx.x / kWave] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < kPsdBlock / kWave; i++) {
      a += sq[i];
      c += sl[i];
    }
    double* dst = work + 2 * ((p - p0) * kPsdChunks + chunk);
    dst[0] = ok ? a : qnan();
    dst[1] = c;
  }
}

}  // namespace gbl
