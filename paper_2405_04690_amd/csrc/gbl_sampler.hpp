// gbl_sampler.hpp -- the GB sampler sweep on the GPU (Sec. 4; appendix
// algorithms gb1 "Galaxy sampling" and gb2 "Galaxy tempering").
//
// State (caller-owned device arrays):
//   u       [n_t][n_w][n_b][n_slot][8] sampling coordinates (log10 A, f0, fdot,
//           phi0, cos iota, psi, lambda, sin beta)
//   exists  [n_t][n_w][n_b][n_slot]    slot occupancy (reversible jump)
//   betas   [n_b][n_t]                  inverse temperatures per sub-band
//   resid   [2][n_w][2][n_bins]         cold-chain buffers: parity p holds the
//           data minus the cold-chain sources of the sub-bands with b % 2 == p
//   inv_psd [n_w][2][n_bins]            1/S per walker
//   group   [n_b][n_w * n_slot][8], group_count [n_b]: stationary groups
//   stats   [8] proposal / acceptance counters; sweep_ctr: sweep index
// Sub-band b covers bins [k_band0 + b N, k_band0 + (b+1) N); its analysis
// window is sub-bands b-1..b+1, read from the opposite-parity buffer, so the
// neighbours' sources stay fixed while band b's sources move.
#pragma once

#include "gbl_kernels.hpp"

namespace gbl {

constexpr int kMaxSlots = 64;
static_assert((kMaxSlots & (kMaxSlots - 1)) == 0, "slot and draw rows are indexed with a mask");

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) from its definition.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                           uint64_t k1, uint64_t* o) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t y0 = hi1 ^ c1 ^ k0, y2 = hi0 ^ c3 ^ k1;
    c0 = y0;
    c1 = lo1;
    c2 = y2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  o[0] = c0;
  o[1] = c1;
  o[2] = c2;
  o[3] = c3;
}

// uniform in (0, 1): counter (sweep, move << 40 | unit, idx / 4, 0), word idx % 4
__device__ __forceinline__ double rng_uniform(uint64_t seed, int64_t sweep, int move, uint64_t unit, uint64_t idx) {
  uint64_t o[4];
  philox4x64((uint64_t)sweep, ((uint64_t)move << 40) | unit, idx >> 2, 0, seed, 0, o);
  return ((double)(o[idx & 3] >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

enum { kMoveInModel = 0, kMoveRJ = 1, kMovePT = 2, kMovePTPerm = 3 };

struct SweepArgs {
  int n_t, n_w, n_b, n_slot, n_prop, n_friends;
  int64_t k_band0;
  double stretch_a;
  uint64_t seed;
  double lo[8], hi[8];
  double* u;
  int32_t* exists;
  const double* betas;
  cd* resid;
  const double* inv_psd;
  double* group;
  int32_t* group_count;
  unsigned long long* stats;
  const int64_t* sweep_ctr;
  const double* prop_u;   // RJ birth candidates (nullptr: prior draws)
  const double* rj_logq;  // ln q per slot (with prop_u)
  double* cold_logl;      // [n_w][n_b] cold-chain band logL after tempering (optional)
  int32_t* swap_acc;      // [n_b][n_t] accepted swaps of rungs (t-1, t) since the last ladder adaptation (optional)
  cd* spec_pool;          // optional pool of per-slot spectra, pool_size entries of n_slot x 2N
  int32_t* pool_flags;    // [pool_size], 0 = free
  int pool_size;
};

__device__ __forceinline__ int64_t uidx(const SweepArgs& a, int t, int w, int b, int s) {
  return (((int64_t)t * a.n_w + w) * a.n_b + b) * a.n_slot + s;
}

__device__ __forceinline__ double period_of(int i) {
  return i == 3 ? kTwoPi : i == 5 ? kPi : i == 6 ? kTwoPi : 0.0;
}

__device__ __forceinline__ double wrap_p(double x, double P) {
  double y = fmod(x, P);
  return y < 0 ? y + P : y;
}

template <int N>
__device__ __forceinline__ void band_f0_range(const Geo& g, const SweepArgs& a, int b, double& lo, double& hi) {
  lo = ((double)a.k_band0 + ((double)b - 0.5) * N) / g.T;
  hi = ((double)a.k_band0 + ((double)b + 1.5) * N) / g.T;
}

// ln of the prior box volume of band b in sampling coordinates
template <int N>
__device__ __forceinline__ double log_box_volume(const Geo& g, const SweepArgs& a, int b) {
  double flo, fhi, v = 0.0;
  band_f0_range<N>(g, a, b, flo, fhi);
  for (int k = 0; k < 8; k++) {
    double w = a.hi[k] - a.lo[k];
    if (k == 1)
      w = fhi - flo;
    else if (period_of(k) > 0)
      w = period_of(k);
    v += log(w);
  }
  return v;
}

template <int N>
__device__ __forceinline__ bool in_prior(const Geo& g, const SweepArgs& a, int b, const double* u) {
  double flo, fhi;
  band_f0_range<N>(g, a, b, flo, fhi);
  if (!(u[1] >= flo && u[1] < fhi)) return false;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    if (i == 1 || period_of(i) > 0) continue;
    if (!(u[i] >= a.lo[i] && u[i] <= a.hi[i])) return false;
  }
  return true;
}

// LDS of one band loop
template <int N>
struct BandSmem {
  cd win[2][3 * N];         // residual window r' (channels A, E)
  double wts[2][3 * N];     // 1/S over the window (0 outside the analysis band)
  cd buf[4 * series_pitch<N>()];
  cd rwin[2 * N];           // spectrum of the template being removed
  double red[2 * (block_threads<N>() / kWave)];
  double u_old[8], u_new[8], prm[8];
  Src src;
  double su[kMaxSlots][8];  // the band's slot coordinates during the loop
  int32_t ex[kMaxSlots];
  int32_t order[kMaxSlots];  // RJ: the slots' flip order; in-model: the occupied slots
  int32_t draw[kMaxSlots];   // the slot-order draws of the reversible-jump pass
  double rdraw[kMaxSlots][9];  // RJ, per flip: acceptance draw, prior birth's coordinates;
                               // in-model, per proposal: its four draws
  int n_occ;                 // in-model: number of occupied slots
  int64_t sq[kMaxSlots];    // carrier bin of each slot's cached spectrum
  int entry;                // spectrum pool entry held by the block (-1: none)
};

// Build the template of sampling coordinates u (shared) into the FFT workspace;
// sm.src holds its decode afterwards.  Block-uniform; contains barriers.
// Not inlined: the band loops call it from several places, and one shared
// body keeps the kernels' register allocation at two waves per SIMD (measured
// 1.6x faster sweeps than the inlined copies at one wave per SIMD).
template <int N>
__device__ __noinline__ void band_template(const Geo& g, const WaveTables<double>& tb, const double* u,
                                           BandSmem<N>& sm) {
  const int tid = threadIdx.x;
  // sampling -> physical coordinates: the three transcendental maps on lane 0
  // of different waves, so that they run side by side
  static_assert(block_threads<N>() >= kWave, "band loops use whole waves");
  if ((tid & (kWave - 1)) == 0) {
    for (int r = tid / kWave; r < 4; r += block_threads<N>() / kWave) {
      if (r == 0) {
        sm.prm[0] = exp10(u[0]);
      } else if (r == 1) {
        sm.prm[4] = acos(u[4]);
      } else if (r == 2) {
        sm.prm[7] = asin(u[7]);
      } else {
        sm.prm[1] = u[1];
        sm.prm[2] = u[2];
        sm.prm[3] = u[3];
        sm.prm[5] = u[5];
        sm.prm[6] = u[6];
      }
    }
  }
  __syncthreads();
  if (tid < kWave) decode_sources<1>(sm.prm, sm.prm, g, &sm.src);
  __syncthreads();
  template_transform<N, 4, double>(sm.src, g, tb, sm.buf, tid);
}

// sums over the block of K values per thread, returned to every thread: wave
// sums, then every thread adds the per-wave partials in wave order (red holds
// K x NT/64 values; the closing barrier frees it for the next reduction)
template <int NT, int K>
__device__ __forceinline__ void block_allsum(double (&v)[K], double* red) {
  constexpr int NW = NT / kWave;
#pragma unroll
  for (int k = 0; k < K; k++) v[k] = wave_sum(v[k]);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) red[k * NW + w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; i++) t += red[k * NW + i];
    v[k] = t;
  }
  __syncthreads();
}

// window += s * (template in the FFT workspace), bins inside the window;
// with `global_buf`, the same change also goes (atomically) to the cold-chain
// buffer of the band's own parity.
// With `store`, the template's spectrum (all N bins, A then E) is also kept
// there for later reuse.
template <int N>
__device__ __forceinline__ void band_add_template(const Geo& g, const WaveTables<double>& tb, BandSmem<N>& sm,
                                                  int64_t k0w, double s, cd* global_buf, cd* store = nullptr) {
  constexpr int NT = block_threads<N>();
  const int64_t ks = sm.src.q - N / 2;
  for (int j = threadIdx.x; j < N; j += NT) {
    int64_t i = ks + j - k0w;
    if (!store && (i < 0 || i >= 3 * N)) continue;
    cd v[2];
    bin_spectrum<N, 2, double>(sm.src, g, tb, sm.buf, j, v);
    if (store) {
      store[j] = v[0];
      store[N + j] = v[1];
      if (i < 0 || i >= 3 * N) continue;
    }
#pragma unroll
    for (int c = 0; c < 2; c++) {
      sm.win[c][i] = sm.win[c][i] + cd{s * v[c].re, s * v[c].im};
      if (global_buf) {
        int64_t k = k0w + i - g.k_min;
        if (k >= 0 && k < g.n_bins) {
          double* dst = reinterpret_cast<double*>(global_buf + c * g.n_bins + k);
          atomicAdd(dst, s * v[c].re);
          atomicAdd(dst + 1, s * v[c].im);
        }
      }
    }
  }
  __syncthreads();
}

// same for the spectrum held in sm.rwin (start bin kr)
template <int N>
__device__ __forceinline__ void band_add_rwin(const Geo& g, BandSmem<N>& sm, int64_t k0w, int64_t kr, double s,
                                              cd* global_buf) {
  constexpr int NT = block_threads<N>();
  for (int j = threadIdx.x; j < N; j += NT) {
    int64_t i = kr + j - k0w;
    if (i < 0 || i >= 3 * N) continue;
#pragma unroll
    for (int c = 0; c < 2; c++) {
      cd v = sm.rwin[c * N + j];
      sm.win[c][i] = sm.win[c][i] + cd{s * v.re, s * v.im};
      if (global_buf) {
        int64_t k = k0w + i - g.k_min;
        if (k >= 0 && k < g.n_bins) {
          double* dst = reinterpret_cast<double*>(global_buf + c * g.n_bins + k);
          atomicAdd(dst, s * v.re);
          atomicAdd(dst + 1, s * v.im);
        }
      }
    }
  }
  __syncthreads();
}

// dlnL = 4 df [<R|d> - 1/2 <d|d>], d = a - r, R = window; a = template in the
// FFT workspace (if has_a), r = sm.rwin (if has_r).  Block-uniform result.
template <int N>
__device__ __forceinline__ double band_dlogl(const Geo& g, const WaveTables<double>& tb, BandSmem<N>& sm,
                                             int64_t k0w, bool has_a, int64_t ka, bool has_r, int64_t kr) {
  constexpr int NT = block_threads<N>();
  double rd = 0.0, dd = 0.0;
  auto acc = [&](int64_t i, cd d0, cd d1) {
    if (i < 0 || i >= 3 * N) return;
    double w0 = sm.wts[0][i], w1 = sm.wts[1][i];
    cd R0 = sm.win[0][i], R1 = sm.win[1][i];
    rd += (R0.re * d0.re + R0.im * d0.im) * w0 + (R1.re * d1.re + R1.im * d1.im) * w1;
    dd += (d0.re * d0.re + d0.im * d0.im) * w0 + (d1.re * d1.re + d1.im * d1.im) * w1;
  };
  if (has_a) {
    for (int j = threadIdx.x; j < N; j += NT) {
      cd v[2];
      bin_spectrum<N, 2, double>(sm.src, g, tb, sm.buf, j, v);
      int64_t k = ka + j;
      int64_t jr = k - kr;
      if (has_r && jr >= 0 && jr < N) {
        v[0] = v[0] - sm.rwin[jr];
        v[1] = v[1] - sm.rwin[N + jr];
      }
      acc(k - k0w, v[0], v[1]);
    }
  }
  if (has_r) {
    for (int j = threadIdx.x; j < N; j += NT) {
      int64_t k = kr + j;
      if (has_a && k >= ka && k < ka + N) continue;
      cd r0 = sm.rwin[j], r1 = sm.rwin[N + j];
      acc(k - k0w, cd{-r0.re, -r0.im}, cd{-r1.re, -r1.im});
    }
  }
  double sums[2] = {rd, dd};
  block_allsum<NT>(sums, sm.red);
  rd = sums[0];
  dd = sums[1];
  return g.df4 * rd - 0.5 * g.df4 * dd;
}

// spectrum of the template in the workspace into sm.rwin
template <int N>
__device__ __forceinline__ void band_store_rwin(const Geo& g, const WaveTables<double>& tb, BandSmem<N>& sm) {
  constexpr int NT = block_threads<N>();
  for (int j = threadIdx.x; j < N; j += NT) {
    cd v[2];
    bin_spectrum<N, 2, double>(sm.src, g, tb, sm.buf, j, v);
    sm.rwin[j] = v[0];
    sm.rwin[N + j] = v[1];
  }
  __syncthreads();
}

// a cached spectrum into sm.rwin
template <int N>
__device__ __forceinline__ void band_load_rwin(BandSmem<N>& sm, const cd* spec) {
  constexpr int NT = block_threads<N>();
  for (int j = threadIdx.x; j < 2 * N; j += NT) sm.rwin[j] = spec[j];
  __syncthreads();
}

// load walker w's window from the opposite-parity buffer, and its weights
template <int N>
__device__ __forceinline__ void band_load_window(const Geo& g, const SweepArgs& a, int w, int b, int64_t k0w,
                                                 BandSmem<N>& sm) {
  constexpr int NT = block_threads<N>();
  const int par = b & 1;
  const cd* opp = a.resid + ((int64_t)(1 - par) * a.n_w + w) * 2 * g.n_bins;
  const double* ip = a.inv_psd + (int64_t)w * 2 * g.n_bins;
  for (int i = threadIdx.x; i < 3 * N; i += NT) {
    int64_t k = k0w + i - g.k_min;
    bool inb = k >= 0 && k < g.n_bins;
#pragma unroll
    for (int c = 0; c < 2; c++) {
      sm.win[c][i] = inb ? opp[c * g.n_bins + k] : cd{0.0, 0.0};
      sm.wts[c][i] = inb ? ip[c * g.n_bins + k] : 0.0;
    }
  }
  __syncthreads();
}

// entry size of the spectrum pool (complex values): the band loops keep n_slot
// spectra of 2N bins, the tempering kernel n_t window sums of 2 x 3N bins
__host__ __device__ __forceinline__ int64_t pool_entry(int n_slot, int n_t, int N) {
  const int64_t e1 = (int64_t)n_slot * 2 * N, e2 = (int64_t)n_t * 6 * N;
  return e1 > e2 ? e1 : e2;
}

// a free pool entry for the block (bounded scan), or -1
__device__ __forceinline__ int pool_acquire(const SweepArgs& a) {
  if (!a.spec_pool) return -1;
  const int P = a.pool_size;
  const int start = (int)(((uint64_t)blockIdx.x * 2654435761ull) % (uint64_t)P);
  for (int k = 0; k < P; k++) {
    const int e = (start + k) % P;
    if (atomicCAS(&a.pool_flags[e], 0, 1) == 0) return e;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Alg. gb1 for every (t, w, b) of one parity: in-model group-stretch moves
// (move 0) or the reversible-jump pass that flips every slot (move 1).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_sweep_band(Geo g, WaveTables<double> tb, SweepArgs a,
                                                                   int move, int parity) {
  __shared__ BandSmem<N> sm;
  const int nbp = (a.n_b - parity + 1) / 2;  // bands of this parity
  const int bi = blockIdx.x % nbp;
  const int tw = blockIdx.x / nbp;
  const int w = tw % a.n_w;
  const int t = tw / a.n_w;
  const int b = parity + 2 * bi;
  const int tid = threadIdx.x;
  const int S = a.n_slot;
  const int64_t sweep = *a.sweep_ctr;
  const int64_t k0w = a.k_band0 + (int64_t)(b - 1) * N;
  const double beta = a.betas[(int64_t)b * a.n_t + t];
  const uint64_t unit = ((uint64_t)t * a.n_w + w) * a.n_b + b;
  cd* own = (t == 0) ? a.resid + ((int64_t)(b & 1) * a.n_w + w) * 2 * g.n_bins : nullptr;

  band_load_window<N>(g, a, w, b, k0w, sm);
  for (int s = tid; s < S; s += block_threads<N>()) {
    sm.ex[s] = a.exists[uidx(a, t, w, b, s)];
    for (int k = 0; k < 8; k++) sm.su[s][k] = a.u[8 * uidx(a, t, w, b, s) + k];
  }
  // a pool entry for the slots' spectra (a bounded scan; without one the
  // spectra are recomputed)
  if (tid == 0) sm.entry = pool_acquire(a);
  __syncthreads();
  cd* const spec = sm.entry >= 0 ? a.spec_pool + (int64_t)sm.entry * pool_entry(S, a.n_t, N) : nullptr;
  // the band's residual: remove its current sources (keeping their spectra)
  for (int s = 0; s < S; s++) {
    if (!sm.ex[s]) continue;
    band_template<N>(g, tb, sm.su[s], sm);
    band_add_template<N>(g, tb, sm, k0w, -1.0, nullptr, spec ? spec + (int64_t)s * 2 * N : nullptr);
    if (tid == 0) sm.sq[s] = sm.src.q;
  }
  __syncthreads();

  unsigned long long n_prop = 0, n_acc = 0, n_bprop = 0, n_bacc = 0, n_dprop = 0, n_dacc = 0;
  if (move == kMoveInModel) {
    const double* grp = a.group + (int64_t)b * a.n_w * S * 8;
    const int G = a.group_count[b];
    // the occupied slots in slot order (in-model moves keep the occupancy)
    if (tid == 0) {
      int c = 0;
      for (int s = 0; s < S; s++)
        if (sm.ex[s]) sm.order[c++] = s;
      sm.n_occ = c;
    }
    __syncthreads();
    const int gcount = sm.n_occ;
    for (int p = 0; p < a.n_prop; p++) {
      if ((p & (kMaxSlots - 1)) == 0) {
        // the next kMaxSlots proposals' four draws (words 8 p + k), one per
        // thread, into the RJ draw rows (free during in-model moves)
        const int pe = a.n_prop - p < kMaxSlots ? a.n_prop - p : kMaxSlots;
        __syncthreads();
        for (int q = tid; q < 4 * pe; q += block_threads<N>())
          sm.rdraw[q >> 2][q & 3] = rng_uniform(a.seed, sweep, move, unit, 8 * (uint64_t)(p + (q >> 2)) + (q & 3));
        __syncthreads();
      }
      const double* rp = sm.rdraw[p & (kMaxSlots - 1)];
      const double r_pick = rp[0], r_friend = rp[1], r_z = rp[2], r_acc = rp[3];
      if (gcount == 0) continue;
      const int sk = sm.order[(int)floor(r_pick * gcount)];
      const double* uk = sm.su[sk];
      n_prop++;
      if (G <= 0) continue;
      // friend: the n_friends sorted group entries around the current f0.
      // Lower bound of f0 among the group keys by a 64-way search of each
      // wave: lane l tests the key at lo + l n / 64, and the ballot (a prefix,
      // the keys being sorted) narrows [lo, hi] 64-fold per step.
      int lo = 0, hi = G;
      {
        const int lane = tid & (kWave - 1);
        while (lo < hi) {
          const int n = hi - lo;
          const int pl = n >= kWave ? lo + (int)(((int64_t)lane * n) / kWave) : lo + lane;
          const bool less = (n >= kWave || lane < n) && grp[8 * (int64_t)pl + 1] < uk[1];
          const int c = __popcll(__ballot(less));
          if (n < kWave) {
            lo += c;
            break;
          }
          if (c == 0) break;  // key[lo] >= f0
          const int lo2 = lo + (int)(((int64_t)(c - 1) * n) / kWave) + 1;
          hi = c < kWave ? lo + (int)(((int64_t)c * n) / kWave) : hi;
          lo = lo2;
        }
      }
      const int nf = a.n_friends < G ? a.n_friends : G;
      int start = lo - nf / 2;
      if (start < 0) start = 0;
      if (start > G - nf) start = G - nf;
      const double* X = grp + 8 * (start + (int)floor(r_friend * nf));
      const double am = a.stretch_a;
      const double z = ((am - 1.0) * r_z + 1.0) * ((am - 1.0) * r_z + 1.0) / am;
      // periodic angles move on the circle: the difference to the friend is
      // taken in (-P/2, P/2] and the stretched difference must stay inside
      // (-P/2, P/2), so that the reverse move (same friend, 1/z) returns to
      // the start; otherwise the proposal is rejected (the pair of moves is
      // then an exact involution with Jacobian z^8)
      double un[8];
      bool reversible = true;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        double diff = uk[i] - X[i];
        double P = period_of(i);
        if (P > 0) {
          diff = wrap_p(diff + 0.5 * P, P) - 0.5 * P;
          const double zd = z * diff;
          if (!(fabs(zd) < 0.5 * P)) reversible = false;
          un[i] = wrap_p(X[i] + zd, P);
        } else {
          un[i] = X[i] + z * diff;
        }
      }
      if (!reversible || !in_prior<N>(g, a, b, un)) continue;
      const double lr = 7.0 * log(z);
      if (tid < 8) {
        sm.u_old[tid] = uk[tid];
        sm.u_new[tid] = un[tid];
      }
      __syncthreads();
      int64_t kr;
      if (spec) {
        band_load_rwin<N>(sm, spec + (int64_t)sk * 2 * N);
        kr = sm.sq[sk] - N / 2;
      } else {
        band_template<N>(g, tb, sm.u_old, sm);
        band_store_rwin<N>(g, tb, sm);
        kr = sm.src.q - N / 2;
      }
      band_template<N>(g, tb, sm.u_new, sm);
      const int64_t ka = sm.src.q - N / 2;
      const double dl = band_dlogl<N>(g, tb, sm, k0w, true, ka, true, kr);
      if (log(r_acc) < beta * dl + lr) {
        band_add_template<N>(g, tb, sm, k0w, -1.0, own, spec ? spec + (int64_t)sk * 2 * N : nullptr);
        band_add_rwin<N>(g, sm, k0w, kr, 1.0, own);
        if (tid < 8) sm.su[sk][tid] = sm.u_new[tid];
        if (tid == 0) sm.sq[sk] = sm.src.q;
        n_acc++;
      }
      __syncthreads();
    }
  } else {
    // flip every slot once in a random order (Fisher-Yates from the top:
    // position j swaps with r_j <= j); the draws in parallel, the swaps on one
    // thread
    for (int j = tid; j < S; j += block_threads<N>())
      sm.draw[j] = j ? (int)floor(rng_uniform(a.seed, sweep, move, unit, (uint64_t)j) * (j + 1)) : 0;
    __syncthreads();
    if (tid == 0) {
      for (int s = 0; s < S; s++) sm.order[s] = s;
      for (int j = S - 1; j >= 1; j--) {
        const int r = sm.draw[j];
        const int tmp = sm.order[j];
        sm.order[j] = sm.order[r];
        sm.order[r] = tmp;
      }
    }
    // every flip's uniform draws (words 64 + 16 i + k: k = 0 acceptance,
    // k = 1..8 a prior birth's coordinates) one per thread ahead of the loop
    for (int q = tid; q < S * 9; q += block_threads<N>()) {
      const int i = q / 9, k = q - 9 * (q / 9);
      sm.rdraw[i][k] = rng_uniform(a.seed, sweep, move, unit, 64 + 16 * (uint64_t)i + k);
    }
    __syncthreads();
    double flo, fhi;
    band_f0_range<N>(g, a, b, flo, fhi);
    const double lvol = a.prop_u ? log_box_volume<N>(g, a, b) : 0.0;
    for (int i = 0; i < S; i++) {
      const int s = sm.order[i];
      const double r_acc = sm.rdraw[i][0];
      const int64_t ui = uidx(a, t, w, b, s);
      double* us = sm.su[s];
      if (sm.ex[s]) {
        // death: the new template is zero; with the prior proposal (q = p) only
        // the likelihood enters, otherwise ln q - ln p as well
        n_dprop++;
        int64_t kr;
        if (spec) {
          band_load_rwin<N>(sm, spec + (int64_t)s * 2 * N);
          kr = sm.sq[s] - N / 2;
        } else {
          if (tid < 8) sm.u_old[tid] = us[tid];
          __syncthreads();
          band_template<N>(g, tb, sm.u_old, sm);
          band_store_rwin<N>(g, tb, sm);
          kr = sm.src.q - N / 2;
        }
        const double dl = band_dlogl<N>(g, tb, sm, k0w, false, 0, true, kr);
        const double lpq = a.prop_u ? a.rj_logq[ui] + lvol : 0.0;
        if (log(r_acc) < beta * dl + lpq) {
          band_add_rwin<N>(g, sm, k0w, kr, 1.0, own);
          if (tid == 0) sm.ex[s] = 0;
          n_dacc++;
        }
      } else if (a.prop_u) {
        // birth from the given proposal: ln p - ln q enters
        n_bprop++;
        if (tid < 8) sm.u_new[tid] = a.prop_u[8 * ui + tid];
        __syncthreads();
        if (in_prior<N>(g, a, b, sm.u_new)) {
          band_template<N>(g, tb, sm.u_new, sm);
          const int64_t ka = sm.src.q - N / 2;
          const double dl = band_dlogl<N>(g, tb, sm, k0w, true, ka, false, 0);
          if (log(r_acc) < beta * dl - lvol - a.rj_logq[ui]) {
            band_add_template<N>(g, tb, sm, k0w, -1.0, own, spec ? spec + (int64_t)s * 2 * N : nullptr);
            if (tid < 8) us[tid] = sm.u_new[tid];
            if (tid == 0) {
              sm.ex[s] = 1;
              sm.sq[s] = sm.src.q;
            }
            n_bacc++;
          }
        }
      } else {
        // birth drawn from the prior
        n_bprop++;
        if (tid < 8) {
          const int k = tid;
          const double r = sm.rdraw[i][1 + k];
          double lo = a.lo[k], hi = a.hi[k];
          if (k == 1) {
            lo = flo;
            hi = fhi;
          } else if (period_of(k) > 0) {
            lo = 0.0;
            hi = period_of(k);
          }
          sm.u_new[k] = lo + (hi - lo) * r;
        }
        __syncthreads();
        band_template<N>(g, tb, sm.u_new, sm);
        const int64_t ka = sm.src.q - N / 2;
        const double dl = band_dlogl<N>(g, tb, sm, k0w, true, ka, false, 0);
        if (log(r_acc) < beta * dl) {
          band_add_template<N>(g, tb, sm, k0w, -1.0, own, spec ? spec + (int64_t)s * 2 * N : nullptr);
          if (tid < 8) us[tid] = sm.u_new[tid];
          if (tid == 0) {
            sm.ex[s] = 1;
            sm.sq[s] = sm.src.q;
          }
          n_bacc++;
        }
      }
      __syncthreads();
    }
  }
  for (int s = tid; s < S; s += block_threads<N>()) {
    a.exists[uidx(a, t, w, b, s)] = sm.ex[s];
    for (int k = 0; k < 8; k++) a.u[8 * uidx(a, t, w, b, s) + k] = sm.su[s][k];
  }
  if (tid == 0 && sm.entry >= 0) atomicExch(&a.pool_flags[sm.entry], 0);
  if (tid == 0) {
    if (n_prop) atomicAdd(&a.stats[0], n_prop);
    if (n_acc) atomicAdd(&a.stats[1], n_acc);
    if (n_bprop) atomicAdd(&a.stats[2], n_bprop);
    if (n_bacc) atomicAdd(&a.stats[3], n_bacc);
    if (n_dprop) atomicAdd(&a.stats[4], n_dprop);
    if (n_dacc) atomicAdd(&a.stats[5], n_dacc);
  }
}

// ---------------------------------------------------------------------------
// Alg. gb2: residual-aware tempering for every band of one parity and every
// ensemble index i; the walker at temperature t is perm_t[i] with perm_t a
// random permutation per (band, temperature).  Swaps run from the hottest
// pair down and are accepted with eq. temp-final.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ double band_set_loglike(const Geo& g, const WaveTables<double>& tb, const SweepArgs& a,
                                                   int t, int w_src, int b, int w_res, int64_t k0w,
                                                   BandSmem<N>& sm) {
  constexpr int NT = block_threads<N>();
  // the set's occupancy flags into LDS in parallel (the window load's barrier
  // covers them)
  for (int s = threadIdx.x; s < a.n_slot; s += NT) sm.ex[s] = a.exists[uidx(a, t, w_src, b, s)];
  band_load_window<N>(g, a, w_res, b, k0w, sm);
  for (int s = 0; s < a.n_slot; s++) {
    if (!sm.ex[s]) continue;
    band_template<N>(g, tb, a.u + 8 * uidx(a, t, w_src, b, s), sm);
    band_add_template<N>(g, tb, sm, k0w, -1.0, nullptr);
  }
  double rr = 0.0;
  for (int i = threadIdx.x; i < 3 * N; i += NT) {
    cd r0 = sm.win[0][i], r1 = sm.win[1][i];
    rr += (r0.re * r0.re + r0.im * r0.im) * sm.wts[0][i] + (r1.re * r1.re + r1.im * r1.im) * sm.wts[1][i];
  }
  double sums[1] = {rr};
  block_allsum<NT>(sums, sm.red);
  rr = sums[0];
  return -0.5 * g.df4 * rr;
}

// H [2][3N] = sum of the templates of source set (t, w_src) over band b's
// window (the templates of band b lie inside it); block-exclusive memory
template <int N>
__device__ __forceinline__ void band_set_sum(const Geo& g, const WaveTables<double>& tb, const SweepArgs& a, int t,
                                             int w_src, int b, int64_t k0w, BandSmem<N>& sm, cd* H) {
  constexpr int NT = block_threads<N>();
  for (int i = threadIdx.x; i < 6 * N; i += NT) H[i] = cd{0.0, 0.0};
  for (int s = threadIdx.x; s < a.n_slot; s += NT) sm.ex[s] = a.exists[uidx(a, t, w_src, b, s)];
  __syncthreads();
  for (int s = 0; s < a.n_slot; s++) {
    if (!sm.ex[s]) continue;
    band_template<N>(g, tb, a.u + 8 * uidx(a, t, w_src, b, s), sm);
    const int64_t ks = sm.src.q - N / 2;
    for (int j = threadIdx.x; j < N; j += NT) {
      const int64_t i = ks + j - k0w;
      if (i < 0 || i >= 3 * N) continue;
      cd v[2];
      bin_spectrum<N, 2, double>(sm.src, g, tb, sm.buf, j, v);
      H[i] = H[i] + v[0];
      H[3 * N + i] = H[3 * N + i] + v[1];
    }
    __syncthreads();
  }
}

// band log-likelihood -1/2 <R - H | R - H> over band b's window, R = walker
// w_res's opposite-parity buffer, weights 1/S of w_res
template <int N>
__device__ __forceinline__ double band_set_loglike_h(const Geo& g, const SweepArgs& a, int b, int w_res, int64_t k0w,
                                                     const cd* H, BandSmem<N>& sm) {
  constexpr int NT = block_threads<N>();
  const cd* opp = a.resid + ((int64_t)(1 - (b & 1)) * a.n_w + w_res) * 2 * g.n_bins;
  const double* ip = a.inv_psd + (int64_t)w_res * 2 * g.n_bins;
  double rr = 0.0;
  for (int i = threadIdx.x; i < 3 * N; i += NT) {
    const int64_t k = k0w + i - g.k_min;
    if (k < 0 || k >= g.n_bins) continue;
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const cd r = opp[c * g.n_bins + k] - H[c * 3 * N + i];
      rr += (r.re * r.re + r.im * r.im) * ip[c * g.n_bins + k];
    }
  }
  double sums[1] = {rr};
  block_allsum<NT>(sums, sm.red);
  rr = sums[0];
  return -0.5 * g.df4 * rr;
}

template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_sweep_pt(Geo g, WaveTables<double> tb, SweepArgs a,
                                                                 int parity) {
  __shared__ BandSmem<N> sm;
  __shared__ int wt[256];
  __shared__ double Lc[256];
  __shared__ int hidx[256];  // window sum of the set at temperature t: entry slot hidx[t]
  const int nbp = (a.n_b - parity + 1) / 2;
  const int bi = blockIdx.x % nbp;
  const int i = blockIdx.x / nbp;
  const int b = parity + 2 * bi;
  const int tid = threadIdx.x;
  const int nt = a.n_t;
  const int64_t sweep = *a.sweep_ctr;
  const int64_t k0w = a.k_band0 + (int64_t)(b - 1) * N;
  // walker of pairing i at temperature t: entry i of a uniform permutation of
  // the walkers (Fisher-Yates from the top: position j swaps with r_j <= j).
  // Each temperature's thread follows position i back through the swaps
  // (j = 1, 2, ...) instead of building the whole permutation.
  for (int t = tid; t < nt; t += block_threads<N>()) {
    const uint64_t unit = (uint64_t)b * nt + t;
    int p = i;
    for (int j = 1; j < a.n_w; j++) {
      const int r = (int)floor(rng_uniform(a.seed, sweep, kMovePTPerm, unit, (uint64_t)j) * (j + 1));
      if (p == j)
        p = r;
      else if (p == r)
        p = j;
    }
    wt[t] = p;
  }
  if (tid == 0) sm.entry = pool_acquire(a);
  for (int t = tid; t < nt; t += block_threads<N>()) hidx[t] = t;
  __syncthreads();
  cd* const Hs = sm.entry >= 0 ? a.spec_pool + (int64_t)sm.entry * pool_entry(a.n_slot, nt, N) : nullptr;
  auto Hof = [&](int t) { return Hs + (int64_t)hidx[t] * 6 * N; };
  for (int t = 0; t < nt; t++) {
    double L;
    if (Hs) {
      band_set_sum<N>(g, tb, a, t, wt[t], b, k0w, sm, Hof(t));
      L = band_set_loglike_h<N>(g, a, b, wt[t], k0w, Hof(t), sm);
    } else {
      L = band_set_loglike<N>(g, tb, a, t, wt[t], b, wt[t], k0w, sm);
    }
    if (tid == 0) Lc[t] = L;
  }
  __syncthreads();
  const double* bt = a.betas + (int64_t)b * nt;
  unsigned long long n_prop = 0, n_acc = 0;
  for (int t = nt - 1; t >= 1; t--) {
    const double L1 = Hs ? band_set_loglike_h<N>(g, a, b, wt[t], k0w, Hof(t - 1), sm)
                         : band_set_loglike<N>(g, tb, a, t - 1, wt[t - 1], b, wt[t], k0w, sm);
    const double L2 = Hs ? band_set_loglike_h<N>(g, a, b, wt[t - 1], k0w, Hof(t), sm)
                         : band_set_loglike<N>(g, tb, a, t, wt[t], b, wt[t - 1], k0w, sm);
    const double la = bt[t] * (L1 - Lc[t]) + bt[t - 1] * (L2 - Lc[t - 1]);
    const double r = rng_uniform(a.seed, sweep, kMovePT, (uint64_t)b * a.n_w + i, (uint64_t)t);
    n_prop++;
    if (log(r) < la) {
      n_acc++;
      if (tid == 0 && a.swap_acc) atomicAdd(&a.swap_acc[(int64_t)b * nt + t], 1);
      if (t == 1 && Hs) {
        // the cold chain of walker w_0 changes: own-parity buffer += old - new
        cd* own = a.resid + ((int64_t)(b & 1) * a.n_w + wt[0]) * 2 * g.n_bins;
        const cd* H0 = Hof(0);
        const cd* H1 = Hof(1);
        for (int i2 = tid; i2 < 3 * N; i2 += block_threads<N>()) {
          const int64_t k = k0w + i2 - g.k_min;
          if (k < 0 || k >= g.n_bins) continue;
#pragma unroll
          for (int c = 0; c < 2; c++) {
            const cd d = H0[c * 3 * N + i2] - H1[c * 3 * N + i2];
            double* dst = reinterpret_cast<double*>(own + c * g.n_bins + k);
            atomicAdd(dst, d.re);
            atomicAdd(dst + 1, d.im);
          }
        }
        __syncthreads();
      } else if (t == 1) {
        // the cold chain of walker w_0 changes: own-parity buffer += old - new
        cd* own = a.resid + ((int64_t)(b & 1) * a.n_w + wt[0]) * 2 * g.n_bins;
        for (int s = 0; s < a.n_slot; s++) {
          if (a.exists[uidx(a, 0, wt[0], b, s)]) {
            band_template<N>(g, tb, a.u + 8 * uidx(a, 0, wt[0], b, s), sm);
            band_add_template<N>(g, tb, sm, k0w, 1.0, own);
          }
          if (a.exists[uidx(a, 1, wt[1], b, s)]) {
            band_template<N>(g, tb, a.u + 8 * uidx(a, 1, wt[1], b, s), sm);
            band_add_template<N>(g, tb, sm, k0w, -1.0, own);
          }
        }
      }
      // exchange the source sets of (t, w_t) and (t-1, w_(t-1))
      for (int s = tid; s < a.n_slot; s += block_threads<N>()) {
        int64_t i1 = uidx(a, t, wt[t], b, s), i2 = uidx(a, t - 1, wt[t - 1], b, s);
        for (int k = 0; k < 8; k++) {
          double tmp = a.u[8 * i1 + k];
          a.u[8 * i1 + k] = a.u[8 * i2 + k];
          a.u[8 * i2 + k] = tmp;
        }
        int32_t e = a.exists[i1];
        a.exists[i1] = a.exists[i2];
        a.exists[i2] = e;
      }
      __threadfence_block();
      __syncthreads();
      if (tid == 0) {
        Lc[t] = L1;
        Lc[t - 1] = L2;
        const int h = hidx[t];
        hidx[t] = hidx[t - 1];
        hidx[t - 1] = h;
      }
      __syncthreads();
    }
  }
  if (tid == 0 && sm.entry >= 0) atomicExch(&a.pool_flags[sm.entry], 0);
  if (tid == 0) {
    atomicAdd(&a.stats[6], n_prop);
    if (n_acc) atomicAdd(&a.stats[7], n_acc);
    if (a.cold_logl) a.cold_logl[(int64_t)wt[0] * a.n_b + b] = Lc[0];
  }
}

// ---------------------------------------------------------------------------
// Stationary groups: the cold-chain sources of every walker in each band,
// sorted by f0 (ties keep walker-major, slot-minor order).
// ---------------------------------------------------------------------------
// every > 0: rebuild only on sweeps that are multiples of `every` (the check
// runs on the device so that captured sweeps stay replayable)
__global__ __launch_bounds__(256) void k_sweep_group(SweepArgs a, int every) {
  if (every > 0 && (*a.sweep_ctr % every) != 0) return;
  constexpr int kChunk = 4096;
  __shared__ double fv[kChunk];  // f0 of a chunk of entries, NaN where the slot is empty
  __shared__ int count;
  const int b = blockIdx.x;
  const int S = a.n_slot;
  const int M = a.n_w * S;
  double* grp = a.group + (int64_t)b * M * 8;
  if (threadIdx.x == 0) count = 0;
  for (int m0 = 0; m0 < M; m0 += blockDim.x) {
    const int m = m0 + threadIdx.x;
    bool mine = false;
    double f = 0.0;
    int64_t ui = 0;
    if (m < M) {
      ui = uidx(a, 0, m / S, b, m % S);
      mine = a.exists[ui] != 0;
      f = a.u[8 * ui + 1];
    }
    // rank = number of entries ordered before this one (f0, then entry index)
    int rank = 0;
    for (int c0 = 0; c0 < M; c0 += kChunk) {
      const int n = min(kChunk, M - c0);
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int m2 = c0 + i;
        const int64_t u2 = uidx(a, 0, m2 / S, b, m2 % S);
        fv[i] = a.exists[u2] ? a.u[8 * u2 + 1] : qnan();
      }
      __syncthreads();
      if (mine)
        for (int i = 0; i < n; i++) {
          const double f2 = fv[i];
          rank += (f2 < f) || (f2 == f && c0 + i < m);
        }
    }
    if (mine) {
      for (int k = 0; k < 8; k++) grp[8 * rank + k] = a.u[8 * ui + k];
      atomicAdd(&count, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) a.group_count[b] = count;
}

// RJ candidates of the flow-and-prior mixture proposal.  Per slot (unit
// (t, w, b), move RJ, draws 2048 + 16 s + k): an occupied slot gets mode 0
// (density at its source); an empty slot draws c = U(2048 + 16 s + 8) and,
// if c < prior_weight, a prior point from the uniforms k = 0..7 (mode 2),
// else 8 standard normals by Box-Muller from the same uniforms (mode 1), to be
// pushed through the flow.
template <int N>
__global__ void k_rj_draw(Geo g, SweepArgs a, double prior_weight, double* prop, int32_t* mode) {
  const int64_t n = (int64_t)a.n_t * a.n_w * a.n_b * a.n_slot;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (a.exists[i]) {
    mode[i] = 0;
    return;
  }
  const int s = (int)(i % a.n_slot);
  const uint64_t unit = (uint64_t)(i / a.n_slot);
  const int b = (int)(unit % a.n_b);
  const int64_t sweep = *a.sweep_ctr;
  const uint64_t d0 = 2048 + 16 * (uint64_t)s;
  double uu[8];
  for (int k = 0; k < 8; k++) uu[k] = rng_uniform(a.seed, sweep, kMoveRJ, unit, d0 + k);
  const double c = rng_uniform(a.seed, sweep, kMoveRJ, unit, d0 + 8);
  if (c < prior_weight) {
    double flo, fhi;
    band_f0_range<N>(g, a, b, flo, fhi);
    for (int k = 0; k < 8; k++) {
      double lo = a.lo[k], hi = a.hi[k];
      if (k == 1) {
        lo = flo;
        hi = fhi;
      } else if (period_of(k) > 0) {
        lo = 0.0;
        hi = period_of(k);
      }
      prop[8 * i + k] = lo + (hi - lo) * uu[k];
    }
    mode[i] = 2;
  } else {
    for (int p = 0; p < 4; p++) {
      const double r = sqrt(-2.0 * log(uu[2 * p]));
      double sn, cs;
      sincospi(2.0 * uu[2 * p + 1], &sn, &cs);
      prop[8 * i + 2 * p] = r * cs;
      prop[8 * i + 2 * p + 1] = r * sn;
    }
    mode[i] = 1;
  }
}

// rj_logq <- ln[(1 - w) q_flow + w p] with rj_logq holding ln q_flow on entry
// (NaN = outside the flow's support) and p the band's uniform prior density
template <int N>
__global__ void k_rj_mix(Geo g, SweepArgs a, double prior_weight, double* rj_logq) {
  const int64_t n = (int64_t)a.n_t * a.n_w * a.n_b * a.n_slot;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = (int)((i / a.n_slot) % a.n_b);
  const double lp = -log_box_volume<N>(g, a, b);
  const double lf = rj_logq[i];
  if (prior_weight <= 0.0) return;  // pure flow: ln q_flow as it is
  const double x = log(prior_weight) + lp;
  if (!(lf == lf) || prior_weight >= 1.0) {
    rj_logq[i] = x;
    return;
  }
  const double y = log1p(-prior_weight) + lf;
  const double m = fmax(x, y);
  rj_logq[i] = m + log1p(exp(-fabs(x - y)));
}

// ---------------------------------------------------------------------------
// Noise-PSD step: stretch moves of the four noise parameters with vertical
// tempering (one chain per temperature and walker, walker w's residual).
// ---------------------------------------------------------------------------
enum { kMovePsd = 4, kMovePsdPT = 5 };

struct PsdArgs {
  int nt, nw;
  int np;  // parameters per set: 4, or 9 with the Galactic foreground
  double a;
  uint64_t seed;
  double lo[9], hi[9];
  double* theta;
  double* logl;
  const double* betas;
  const int64_t* sweep_ctr;
  unsigned long long* stats;
};

// full residual of walker w: buffer 0 + buffer 1 - data; rows r = w * 2 + c
// over blockIdx.y, bins over blockIdx.x (both grid-stride)
__global__ void k_psd_full_resid(int64_t nb, int nw, const cd* __restrict__ resid, const cd* __restrict__ data,
                                 cd* __restrict__ out) {
  const int64_t total = (int64_t)nw * 2 * nb;
  for (int64_t r = blockIdx.y; r < 2 * (int64_t)nw; r += gridDim.y) {
    const cd* dr = data + (r & 1) * nb;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = r * nb + k;
      out[i] = resid[i] + resid[total + i] - dr[k];
    }
  }
}

// res_idx for all chains (h < 0: set t n_w + w -> w) or the chains of half h
// (set t (n_w/2) + i -> walker 2 i + h)
__global__ void k_psd_res_idx(int nt, int nw, int h, int32_t* res_idx) {
  const int n = h < 0 ? nt * nw : nt * (nw / 2);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  res_idx[s] = h < 0 ? s % nw : 2 * (s % (nw / 2)) + h;
}

// proposals of half h: prop [nt][nw/2][np], lz = (np - 1) ln z, ok = inside the prior box
__global__ void k_psd_propose(PsdArgs p, int h, double* prop, double* lz, double* ok) {
  const int half = p.nw / 2;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.nt * half) return;
  const int t = s / half, w = 2 * (s % half) + h;
  const int64_t sweep = *p.sweep_ctr;
  const uint64_t unit = (uint64_t)t * p.nw + w;
  const double r_pick = rng_uniform(p.seed, sweep, kMovePsd, unit, 4 * (uint64_t)h + 0);
  const double r_z = rng_uniform(p.seed, sweep, kMovePsd, unit, 4 * (uint64_t)h + 1);
  const int j = 2 * (int)floor(r_pick * half) + (1 - h);
  const double z = ((p.a - 1.0) * r_z + 1.0) * ((p.a - 1.0) * r_z + 1.0) / p.a;
  const double* X = p.theta + ((int64_t)t * p.nw + j) * p.np;
  const double* Y = p.theta + ((int64_t)t * p.nw + w) * p.np;
  bool inside = true;
  for (int k = 0; k < p.np; k++) {
    const double v = X[k] + z * (Y[k] - X[k]);
    prop[(int64_t)p.np * s + k] = v;
    inside = inside && (v >= p.lo[k] && v <= p.hi[k]);
  }
  lz[s] = (double)(p.np - 1) * log(z);
  ok[s] = inside ? 1.0 : 0.0;
}

__global__ void k_psd_accept(PsdArgs p, int h, const double* prop, const double* lprop, const double* lz,
                             const double* ok) {
  const int half = p.nw / 2;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.nt * half) return;
  const int t = s / half, w = 2 * (s % half) + h;
  const int64_t c = (int64_t)t * p.nw + w;
  atomicAdd(&p.stats[0], 1ull);
  if (ok[s] == 0.0) return;
  const int64_t sweep = *p.sweep_ctr;
  const double r = rng_uniform(p.seed, sweep, kMovePsd, (uint64_t)c, 4 * (uint64_t)h + 2);
  const double la = p.betas[t] * (lprop[s] - p.logl[c]) + lz[s];
  if (log(r) < la) {
    for (int k = 0; k < p.np; k++) p.theta[p.np * c + k] = prop[(int64_t)p.np * s + k];
    p.logl[c] = lprop[s];
    atomicAdd(&p.stats[1], 1ull);
  }
}

// vertical tempering: per walker, swaps from the hottest pair down
__global__ void k_psd_swap(PsdArgs p) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= p.nw) return;
  const int64_t sweep = *p.sweep_ctr;
  unsigned long long np = 0, na = 0;
  for (int t = p.nt - 1; t >= 1; t--) {
    np++;
    const double r = rng_uniform(p.seed, sweep, kMovePsdPT, (uint64_t)w, (uint64_t)t);
    const int64_t c1 = (int64_t)t * p.nw + w, c0 = (int64_t)(t - 1) * p.nw + w;
    const double la = (p.betas[t - 1] - p.betas[t]) * (p.logl[c1] - p.logl[c0]);
    if (log(r) < la) {
      for (int k = 0; k < p.np; k++) {
        const double tmp = p.theta[p.np * c1 + k];
        p.theta[p.np * c1 + k] = p.theta[p.np * c0 + k];
        p.theta[p.np * c0 + k] = tmp;
      }
      const double tl = p.logl[c1];
      p.logl[c1] = p.logl[c0];
      p.logl[c0] = tl;
      na++;
    }
  }
  if (np) atomicAdd(&p.stats[2], np);
  if (na) atomicAdd(&p.stats[3], na);
}

// ---------------------------------------------------------------------------
// Temperature-ladder adaptation (appendix on parallel tempering; the gap
// dynamics of Vousden, Farr & Mandel 2016): with T = 1/beta and A_j the
// fraction of accepted swaps of rungs (j, j+1) since the last call,
//   T_(j+1) - T_j  <-  (T_(j+1) - T_j) exp(kappa (A_j - A_(j+1))),
//   kappa = t0 / (nu (sweep + t0)),
// the coldest and hottest rungs fixed and the others re-summed from the
// coldest.  One thread per band; the counts are cleared.
// ---------------------------------------------------------------------------
__global__ void k_sweep_adapt(SweepArgs a, double lag, double time_scale) {
#pragma clang fp contract(off)
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_b) return;
  const int nt = a.n_t;
  double* bt = const_cast<double*>(a.betas) + (int64_t)b * nt;
  int32_t* ac = a.swap_acc + (int64_t)b * nt;
  const double kappa = lag / (time_scale * ((double)*a.sweep_ctr + lag));
  if (nt > 2) {
    double T = 1.0 / bt[0];
    double inv_cur = 1.0 / bt[0];
    for (int j = 0; j + 2 < nt; j++) {
      const double inv_next = 1.0 / bt[j + 1];  // still the old rung
      const double A_lo = (double)ac[j + 1] / (double)a.n_w;
      const double A_hi = (double)ac[j + 2] / (double)a.n_w;
      const double gap = (inv_next - inv_cur) * exp(kappa * (A_lo - A_hi));
      T += gap;
      bt[j + 1] = 1.0 / T;
      inv_cur = inv_next;
    }
  }
  for (int t = 0; t < nt; t++) ac[t] = 0;
}

// ---------------------------------------------------------------------------
// Sub-band ownership (Sec. 4): a cold-chain source whose f0 has left its
// band's nominal range [k_band0 + b N, k_band0 + (b+1) N) / T moves to the
// neighbouring band it lies in (lowest free cold-chain slot; it stays if
// there is none); it is added back to the old parity's buffer and removed
// from the new one's.  One block per walker, bands and slots in increasing
// order (the walker's buffers belong to its block alone: plain updates).
// stats[8] counts moved sources, stats[9] sources without a free slot.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(block_threads<N>()) void k_sweep_shift(Geo g, WaveTables<double> tb, SweepArgs a) {
  constexpr int NT = block_threads<N>();
  __shared__ cd buf[4 * series_pitch<N>()];
  __shared__ Src src;
  __shared__ double prm[8];
  const int w = blockIdx.x;
  const int tid = threadIdx.x;
  const int S = a.n_slot;
  unsigned long long moved = 0, stuck = 0;
  for (int b = 0; b < a.n_b; b++) {
    for (int s = 0; s < S; s++) {
      const int64_t ui = uidx(a, 0, w, b, s);
      if (!a.exists[ui]) continue;  // uniform: every thread reads the same flag
      const double f0 = a.u[8 * ui + 1];
      const double lo = (double)(a.k_band0 + (int64_t)b * N) / g.T;
      const double hi = (double)(a.k_band0 + (int64_t)(b + 1) * N) / g.T;
      const int bb = f0 < lo ? b - 1 : (f0 >= hi ? b + 1 : b);
      if (bb == b || bb < 0 || bb >= a.n_b) continue;
      int s2 = -1;
      for (int j = 0; j < S && s2 < 0; j++)
        if (!a.exists[uidx(a, 0, w, bb, j)]) s2 = j;
      if (s2 < 0) {
        stuck++;
        continue;
      }
      const int64_t u2 = uidx(a, 0, w, bb, s2);
      __syncthreads();  // every thread has read the flags before they change
      if (tid < 8) {
        // sampling -> physical coordinates (log10 A, cos iota, sin beta mapped back)
        const double v = a.u[8 * ui + tid];
        a.u[8 * u2 + tid] = v;
        prm[tid] = tid == 0 ? exp10(v) : tid == 4 ? acos(v) : tid == 7 ? asin(v) : v;
      }
      if (tid == 0) {
        a.exists[u2] = 1;
        a.exists[ui] = 0;
      }
      __threadfence_block();
      __syncthreads();
      if (tid < kWave) decode_sources<1>(prm, prm, g, &src);
      __syncthreads();
      template_transform<N, 4, double>(src, g, tb, buf, tid);
      cd* old_buf = a.resid + ((int64_t)(b & 1) * a.n_w + w) * 2 * g.n_bins;
      cd* new_buf = a.resid + ((int64_t)(bb & 1) * a.n_w + w) * 2 * g.n_bins;
      const int64_t k0 = src.q - N / 2;
      for (int j = tid; j < N; j += NT) {
        const int64_t k = k0 + j;
        if (k < g.k_min || k >= g.k_min + g.n_bins) continue;
        const int64_t idx = k - g.k_min;
        cd v[2];
        bin_spectrum<N, 2, double>(src, g, tb, buf, j, v);
#pragma unroll
        for (int c = 0; c < 2; c++) {
          old_buf[c * g.n_bins + idx] = old_buf[c * g.n_bins + idx] + v[c];
          new_buf[c * g.n_bins + idx] = new_buf[c * g.n_bins + idx] - v[c];
        }
      }
      __syncthreads();
      moved++;
    }
  }
  if (tid == 0) {
    if (moved) atomicAdd(&a.stats[8], moved);
    if (stuck) atomicAdd(&a.stats[9], stuck);
  }
}

__global__ void k_sweep_advance(int64_t* sweep_ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *sweep_ctr += 1;
}

}  // namespace gbl
