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
  int band_w;             // sub-band width W (bins)
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
  cd* wsum;               // optional [n_t][n_w][n_b][2][2W + N] window sums of the source sets
};

// Band b's window: every bin a template of the band can reach (f0 ranges over
// [(b - 1/2) W, (b + 3/2) W) past k_band0, a template spans N bins around its
// carrier): [k_band0 + bW - W/2 - N/2, ...), 2W + N bins; bands b-1..b+1 when
// W = N.
template <int N>
__device__ __forceinline__ int64_t win_k0(const SweepArgs& a, int b) {
  return a.k_band0 + (int64_t)b * a.band_w - a.band_w / 2 - N / 2;
}

template <int N>
__host__ __device__ __forceinline__ int win_len(int band_w) {
  return 2 * band_w + N;
}

// window-sum entry of source set (t, w) in band b (A, then E)
template <int N>
__device__ __forceinline__ cd* wsum_entry(const SweepArgs& a, int t, int w, int b) {
  return a.wsum + (((int64_t)t * a.n_w + w) * a.n_b + b) * 2 * win_len<N>(a.band_w);
}

__device__ __forceinline__ int64_t uidx(const SweepArgs& a, int t, int w, int b, int s) {
  return (((int64_t)t * a.n_w + w) * a.n_b + b) * a.n_slot + s;
}

__device__ __forceinline__ double period_of(int i) {
  return i == 3 ? kTwoPi : i == 5 ? kPi : i == 6 ? kTwoPi : 0.0;
}

// x reduced into [0, P).  The remainder is fmod's (exact); for |x| < 2P it
// is formed directly: x itself for |x| < P, and x - P (exact, Sterbenz) for
// P <= x < 2P, which covers every use in the moves.
__device__ __forceinline__ double wrap_p(double x, double P) {
  double y;
  if (fabs(x) < P)
    y = x;
  else if (x >= P && x < 2.0 * P)
    y = x - P;
  else
    y = fmod(x, P);
  return y < 0 ? y + P : y;
}

template <int N>
__device__ __forceinline__ void band_f0_range(const Geo& g, const SweepArgs& a, int b, double& lo, double& hi) {
  const double W = (double)a.band_w;
  lo = ((double)a.k_band0 + ((double)b - 0.5) * W) / g.T;
  hi = ((double)a.k_band0 + ((double)b + 1.5) * W) / g.T;
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

// LDS of the tempering kernel's band likelihoods (the window arrays serve the
// path without window sums or pool entry, which N = 1024 does not take)
template <int N>
constexpr bool pt_lds_window() {
  return N <= 512;
}

template <int N>
struct BandSmem {
  cd win[2][pt_lds_window<N>() ? 3 * N : 1];      // residual window r' (channels A, E)
  double wts[2][pt_lds_window<N>() ? 3 * N : 1];  // 1/S over the window (0 outside the analysis band)
  cd buf[4 * series_pitch<N>()];
  double red[2 * (block_threads<N>() / kWave)];
  double prm[8];
  Src src;
  int32_t ex[kMaxSlots];
  int entry;                // spectrum pool entry held by the block (-1: none)
};

// Build the template of sampling coordinates u (shared) into the FFT workspace;
// sm.src holds its decode afterwards.  Block-uniform; contains barriers.
// Not inlined: the tempering kernel calls it from several places, and one
// shared body keeps its register allocation at two waves per SIMD.
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

// Block order of the per-band kernels (band loops and tempering): each XCD
// takes one contiguous run of the logical grid (xcd_block), and the logical
// grid is band-major, so that the blocks in flight on an XCD share one band's
// group, residual windows and weights in its L2.  Bands are ordered by class
// bi mod 8 (bands 0, 8, 16, ..., then 1, 9, ...), so that every XCD's run
// spreads over the whole frequency range and the XCDs carry similar source
// counts.  Returns the band index bi of this parity (0 <= bi < nbp) and the
// index j of the block within its band (0 <= j < per_band); a bijection from
// the grid of nbp * per_band blocks.
__device__ __forceinline__ void band_block(int nbp, int per_band, int& bi, int& j) {
  const int L = (int)xcd_block();
  const int lb = L / per_band;
  j = L - lb * per_band;
  int off = 0;
  bi = 0;
#pragma unroll
  for (int c = 0; c < (int)kXcds; c++) {
    const int nc = (nbp - c + (int)kXcds - 1) / (int)kXcds;  // bands bi = c mod 8
    if (lb >= off && lb < off + nc) bi = c + (int)kXcds * (lb - off);
    off += nc;
  }
}

// ---------------------------------------------------------------------------
// Alg. gb1 for every (t, w, b) of one parity: in-model group-stretch moves
// (move 0) or the reversible-jump pass that flips every slot (move 1).
//
// The loop body builds at most one template per pass, so that the template
// build has a single call site and is inlined once; with the residual window
// as the only large LDS array the kernel holds three blocks per CU at
// N = 256 (below 168 VGPRs and 54 KB of LDS).  The spectra of the template
// being added (a) and removed (r) stay in registers at the bins each thread
// owns (j = tid + NT m); r goes through the FFT workspace only for the bins
// of a's window that need it at another offset.  The weights 1/S come from
// HBM, fetched while the template is built.
// ---------------------------------------------------------------------------
// threads per block of the band loops: as for the other kernels, except at
// N = 1024, where 512 threads (two bins each) keep the spectra and weights
// of the loop within the register budget
template <int N>
constexpr int loop_threads() {
  return N == 1024 ? 512 : block_threads<N>();
}

// waves per SIMD the band loop is compiled for (the register budget): three
// at one bin per thread (168 VGPRs, three blocks per CU); at two bins per
// thread the loop's spectra need more, and two waves (256 VGPRs) keep them
// out of scratch memory, whose spill stores inside the loop would otherwise
// reach HBM on every pass
template <int N>
constexpr int loop_waves() {
  return N / loop_threads<N>() == 1 ? 3 : 2;
}

// GW: the window lives in global memory (the set's window-sum entry) instead
// of LDS, for sub-bands wider than the template (2W + N bins) or N = 1024
template <int N, bool GW>
struct LoopSmem {
  cd win[2][GW ? 1 : 3 * N];      // residual window r' (channels A, E), W = N in LDS
  cd buf[4 * series_pitch<N>()];  // FFT workspace; afterwards r's spectrum (A at [0, N), E at [N, 2N))
  double su[kMaxSlots][8];        // the band's slot coordinates during the loop
  double rdraw[kMaxSlots][9];     // RJ, per flip: acceptance draw, prior birth's coordinates;
                                  // in-model, per proposal: its four draws
  double red[2 * (loop_threads<N>() / kWave)];
  double u_old[8], u_new[8];
  double blo[8], bhi[8];      // the band's prior box in sampling coordinates (f0: the band's range,
                              // angles: one period)
  Src src;
  int64_t sq[kMaxSlots];      // carrier bin of each slot's cached spectrum
  int32_t ex[kMaxSlots];
  int32_t order[kMaxSlots];   // RJ: the slots' flip order; in-model: the occupied slots
  int32_t draw[kMaxSlots];    // the slot-order draws of the reversible-jump pass
  int32_t fstart[kMaxSlots];  // in-model: first friend of each occupied slot's window in the group
  int n_occ;                  // in-model: number of occupied slots
  int entry;                  // spectrum pool entry held by the block (-1: none)
};

// u inside the band's prior box (kept in LDS rather than in registers across
// the band loop); the same tests as in_prior
template <int N, bool GW>
__device__ __forceinline__ bool loop_in_prior(const LoopSmem<N, GW>& sm, const double* u) {
  if (!(u[1] >= sm.blo[1] && u[1] < sm.bhi[1])) return false;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    if (i == 1 || period_of(i) > 0) continue;
    if (!(u[i] >= sm.blo[i] && u[i] <= sm.bhi[i])) return false;
  }
  return true;
}

// natural logarithm, not inlined: inside the band loop the library
// function's constants would be hoisted out of the loop and held in vector
// registers across it
__device__ __noinline__ double log_ni(double x) { return log(x); }

// first friend of key f in the band's group (G entries sorted by f0, the key
// at word 1 of each): the lower bound of f by a 64-way search of the calling
// wave (every lane takes part: lane l tests the key at lo + l n / 64, and the
// ballot, a prefix since the keys are sorted, narrows [lo, hi] 64-fold per
// step), then the start of the nf entries around it
__device__ __forceinline__ int friend_start(const double* __restrict__ grp, int G, int nf, double f) {
  int lo = 0, hi = G;
  const int lane = threadIdx.x & (kWave - 1);
  while (lo < hi) {
    const int n = hi - lo;
    const int pl = n >= kWave ? lo + (int)(((int64_t)lane * n) / kWave) : lo + lane;
    const bool less = (n >= kWave || lane < n) && grp[8 * (int64_t)pl + 1] < f;
    const int c = __popcll(__ballot(less));
    if (n < kWave) {
      lo += c;
      break;
    }
    if (c == 0) break;  // key[lo] >= f
    const int lo2 = lo + (int)(((int64_t)(c - 1) * n) / kWave) + 1;
    hi = c < kWave ? lo + (int)(((int64_t)c * n) / kWave) : hi;
    lo = lo2;
  }
  int start = lo - nf / 2;
  if (start < 0) start = 0;
  if (start > G - nf) start = G - nf;
  return start;
}

// weights 1/S (0 outside the analysis band) at the thread's bins k0 + j
template <int N, int BPT>
__device__ __forceinline__ void loop_weights(const Geo& g, const double* __restrict__ wts, int64_t k0,
                                             double (&wh)[BPT][2], int tid) {
  constexpr int NT = loop_threads<N>();
#pragma unroll
  for (int m = 0; m < BPT; m++) {
    const int64_t k = k0 + tid + NT * m - g.k_min;
    const bool in = k >= 0 && k < g.n_bins;
    wh[m][0] = in ? wts[k] : 0.0;
    wh[m][1] = in ? wts[g.n_bins + k] : 0.0;
  }
}

// a spectrum (all N bins, A then E) to or from a pool slot
template <int N, int BPT>
__device__ __forceinline__ void loop_store(cd* dst, const cd (&h)[BPT][2], int tid) {
  constexpr int NT = loop_threads<N>();
#pragma unroll
  for (int m = 0; m < BPT; m++) {
    const int j = tid + NT * m;
    dst[j] = h[m][0];
    dst[N + j] = h[m][1];
  }
}

template <int N, int BPT>
__device__ __forceinline__ void loop_load(const cd* src, cd (&h)[BPT][2], int tid) {
  constexpr int NT = loop_threads<N>();
#pragma unroll
  for (int m = 0; m < BPT; m++) {
    const int j = tid + NT * m;
    h[m][0] = src[j];
    h[m][1] = src[N + j];
  }
}

// the window's element i of channel c: in LDS, or in global memory at
// gw + c L + i
// Full decode of one source from its sampling coordinates (log10 A, f0,
// fdot, phi0, cos iota, psi, lambda, sin beta) by the block's first two
// waves side by side (every lane of both takes part).  The sky and
// inclination angles enter the response only through sin beta, cos beta and
// cos iota, so those come from the coordinates themselves (cos beta =
// sqrt((1 - sin beta)(1 + sin beta)) >= 0 on |beta| <= pi/2) instead of
// through acos/asin and back, and the phases lambda, 2 psi and the carrier's
// delay take the exactly reduced polynomial exp(2 pi i c) in cycles.  Wave 0
// writes output groups 0..8 (lane a: group a, the projections, which need
// lambda and beta only); wave 1 the amplitude 10^u0 (the one library call),
// the polarisation amplitudes, carrier, phases, delay factor and state.
__device__ __forceinline__ void decode_sampled(const double* __restrict__ u, const Geo& g, Src& s) {
  const int wid = (int)(threadIdx.x / kWave);
  const int lane = (int)(threadIdx.x & (kWave - 1));
  if (wid == 0) {
    const cd el = expi_cycles(u[6] * (1.0 / kTwoPi));  // (cos lambda, sin lambda)
    SrcTrig tr;
    tr.sl = el.im;
    tr.cl = el.re;
    tr.sb = u[7];
    tr.cb = sqrt((1.0 - u[7]) * (1.0 + u[7]));
    tr.ci = u[4];
    tr.s2p = 0.0;  // (groups 0..8 read neither)
    tr.c2p = 1.0;
    if (lane < 9) decode_group(lane, u, tr, g, s);
  } else if (wid == 1) {
    const bool finite_u = isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(u[3]) &&
                          isfinite(u[4]) && isfinite(u[5]) && isfinite(u[6]) && isfinite(u[7]) &&
                          fabs(u[4]) <= 1.0 && fabs(u[7]) <= 1.0 && fabs(u[1] * g.T) < 4503599627370496.0;
    const double A = exp10(u[0]);
    const bool finite = finite_u && isfinite(A);
    const double f0 = finite ? u[1] : 0.0;  // keep the arithmetic below well defined
    const double qd = floor(f0 * g.T);
    const cd dq = expi_cycles(-qd * (g.Lc / g.T));
    const cd e2p = expi_cycles(u[5] * (1.0 / kPi));  // (cos 2 psi, sin 2 psi)
    if (lane == 0) {
      s.state = finite ? (A == 0.0 ? 1 : 0) : 2;
      s.f0 = f0;
      s.fdot = u[2];
      s.phi0_cyc = u[3] / kTwoPi;
      s.q = (int64_t)qd;
      s.dfq = f0 - qd / g.T;
      const double ci = u[4];
      const double ap = A * (1.0 + ci * ci);
      const double ax = 2.0 * A * ci;
      s.cp = {ap * e2p.re, -ax * e2p.im};
      s.cx2 = {2.0 * ap * e2p.im, 2.0 * ax * e2p.re};
      s.dq = dq;
    }
  }
}

// sampling coordinates u (LDS) -> decode in sm.src, on the first two waves.
// Not inlined: the library function's and the polynomials' constants would
// otherwise be hoisted out of the band loop and held in vector registers
// across it.  Block-uniform; contains a barrier.
template <int N, bool GW>
__device__ __noinline__ void loop_decode(const Geo& g, const double* u, LoopSmem<N, GW>& sm) {
  static_assert(loop_threads<N>() >= 2 * kWave, "the decode takes two waves");
  decode_sampled(u, g, sm.src);
  __syncthreads();
}

// sampling coordinates u (LDS) -> template in sm.buf, its decode in sm.src;
// with wts, also the weights at the thread's bins of the template's window,
// and with rsrc the removed template's cached spectrum (rv) and its weights
// (wr, window start kr): all requested after the decode (a call, which waits
// for every outstanding load) and before the response and the FFT, so that
// their latency hides behind them.  F: precision of the response and the FFT
// (float: the mixed-precision sweep; the decode, the phases and every sum
// stay FP64).  Block-uniform; contains barriers.
template <int N, int BPT, bool GW, typename F>
__device__ __forceinline__ void loop_build(const Geo& g, const WaveTables<F>& tb, const double* u,
                                           LoopSmem<N, GW>& sm, const double* __restrict__ wts, double (&wh)[BPT][2],
                                           const cd* rsrc, int64_t kr, cd (&rv)[BPT][2], double (&wr)[BPT][2],
                                           int tid) {
  loop_decode<N, GW>(g, u, sm);
  if (wts) loop_weights<N, BPT>(g, wts, sm.src.q - N / 2, wh, tid);
  if (rsrc) {
    loop_load<N, BPT>(rsrc, rv, tid);
    loop_weights<N, BPT>(g, wts, kr, wr, tid);
  }
  template_transform<N, 4, F, loop_threads<N>(), true>(sm.src, g, tb, reinterpret_cast<cx<F>*>(sm.buf), tid);
}

// spectrum of the built template at the thread's bins (in FP64 whatever the
// precision of the build)
template <int N, int BPT, bool GW, typename F>
__device__ __forceinline__ void loop_bins(const Geo& g, const WaveTables<F>& tb, const LoopSmem<N, GW>& sm,
                                          cd (&h)[BPT][2], int tid) {
  constexpr int NT = loop_threads<N>();
#pragma unroll
  for (int m = 0; m < BPT; m++) {
    if constexpr (std::is_same<F, double>::value) {
      bin_spectrum<N, 2, double>(sm.src, g, tb, sm.buf, tid + NT * m, h[m]);
    } else {
      cx<F> hf[2];
      bin_spectrum<N, 2, F>(sm.src, g, tb, reinterpret_cast<const cx<F>*>(sm.buf), tid + NT * m, hf);
#pragma unroll
      for (int c = 0; c < 2; c++) h[m][c] = cd{(double)hf[c].re, (double)hf[c].im};
    }
  }
}

template <int N, bool GW>
__device__ __forceinline__ cd& win_at(LoopSmem<N, GW>& sm, cd* gw, int L, int c, int64_t i) {
  if constexpr (GW)
    return gw[c * L + i];
  else
    return sm.win[c][i];
}

// window += s h at the bins k0 + j inside it (window [k0w, k0w + L)); with
// own, the same change also goes (atomically) to that cold-chain buffer.  No
// closing barrier.
template <int N, int BPT, bool GW>
__device__ __forceinline__ void loop_add(const Geo& g, LoopSmem<N, GW>& sm, cd* gw, int L, int64_t k0w, int64_t k0,
                                         double s, const cd (&h)[BPT][2], cd* own, int tid) {
  constexpr int NT = loop_threads<N>();
#pragma unroll
  for (int m = 0; m < BPT; m++) {
    const int64_t i = k0 + tid + NT * m - k0w;
    if (i < 0 || i >= L) continue;
#pragma unroll
    for (int c = 0; c < 2; c++) {
      cd& x = win_at<N, GW>(sm, gw, L, c, i);
      x = x + cd{s * h[m][c].re, s * h[m][c].im};
      if (own) {
        const int64_t k = k0w + i - g.k_min;
        if (k >= 0 && k < g.n_bins) {
          double* dst = reinterpret_cast<double*>(own + c * g.n_bins + k);
          atomicAdd(dst, s * h[m][c].re);
          atomicAdd(dst + 1, s * h[m][c].im);
        }
      }
    }
  }
}

// dlnL = 4 df [<R|d> - 1/2 <d|d>], d = a - r, R = window, from the spectra at
// the thread's bins: a (if has_a) at ka + j with weights wa, r (if has_r) at
// kr + j with weights wr; with both, r's spectrum must also sit in sm.buf.
// Block-uniform result.
template <int N, int BPT, bool GW>
__device__ __forceinline__ double loop_dlogl(const Geo& g, LoopSmem<N, GW>& sm, cd* gw, int L, int64_t k0w,
                                             bool has_a, int64_t ka, const cd (&av)[BPT][2],
                                             const double (&wa)[BPT][2], bool has_r, int64_t kr,
                                             const cd (&rv)[BPT][2], const double (&wr)[BPT][2], int tid) {
  constexpr int NT = loop_threads<N>();
  double rd = 0.0, dd = 0.0;
  auto acc = [&](int64_t i, cd d0, cd d1, double w0, double w1) {
    if (i < 0 || i >= L) return;
    const cd R0 = win_at<N, GW>(sm, gw, L, 0, i), R1 = win_at<N, GW>(sm, gw, L, 1, i);
    rd += (R0.re * d0.re + R0.im * d0.im) * w0 + (R1.re * d1.re + R1.im * d1.im) * w1;
    dd += (d0.re * d0.re + d0.im * d0.im) * w0 + (d1.re * d1.re + d1.im * d1.im) * w1;
  };
  if (has_a) {
#pragma unroll
    for (int m = 0; m < BPT; m++) {
      const int64_t k = ka + tid + NT * m;
      cd v0 = av[m][0], v1 = av[m][1];
      const int64_t jr = k - kr;
      if (has_r && jr >= 0 && jr < N) {
        v0 = v0 - sm.buf[jr];
        v1 = v1 - sm.buf[N + jr];
      }
      acc(k - k0w, v0, v1, wa[m][0], wa[m][1]);
    }
  }
  if (has_r) {
#pragma unroll
    for (int m = 0; m < BPT; m++) {
      const int64_t k = kr + tid + NT * m;
      if (has_a && k >= ka && k < ka + N) continue;
      acc(k - k0w, cd{-rv[m][0].re, -rv[m][0].im}, cd{-rv[m][1].re, -rv[m][1].im}, wr[m][0], wr[m][1]);
    }
  }
  double sums[2] = {rd, dd};
  block_allsum<NT>(sums, sm.red);
  return g.df4 * sums[0] - 0.5 * g.df4 * sums[1];
}

template <int N, bool GW, typename F>
__global__ __launch_bounds__(loop_threads<N>(), loop_waves<N>()) void k_sweep_band(Geo g, WaveTables<F> tb,
                                                                                    SweepArgs a, int move,
                                                                                    int parity) {
  constexpr int NT = loop_threads<N>();
  constexpr int BPT = N / NT;  // window bins per thread
  __shared__ LoopSmem<N, GW> sm;
  const int nbp = (a.n_b - parity + 1) / 2;  // bands of this parity
  int bi, tw;
  band_block(nbp, a.n_t * a.n_w, bi, tw);
  const int w = tw % a.n_w;
  const int t = tw / a.n_w;
  const int b = parity + 2 * bi;
  int tid = threadIdx.x;
  const int S = a.n_slot;
  const int64_t sweep = *a.sweep_ctr;
  const int64_t k0w = win_k0<N>(a, b);
  const int L = win_len<N>(a.band_w);
  cd* const gw = GW ? wsum_entry<N>(a, t, w, b) : nullptr;  // the window in global memory
  const double beta = a.betas[(int64_t)b * a.n_t + t];
  const uint64_t unit = ((uint64_t)t * a.n_w + w) * a.n_b + b;
  cd* own = (t == 0) ? a.resid + ((int64_t)(b & 1) * a.n_w + w) * 2 * g.n_bins : nullptr;
  const double* wts = a.inv_psd + (int64_t)w * 2 * g.n_bins;
  const bool inmodel = move == kMoveInModel;

  // walker w's window from the opposite-parity buffer, the band's slots and a
  // pool entry for the slots' spectra (a bounded scan; without one the
  // spectra are recomputed)
  {
    const cd* opp = a.resid + ((int64_t)(1 - (b & 1)) * a.n_w + w) * 2 * g.n_bins;
    for (int i = tid; i < L; i += NT) {
      const int64_t k = k0w + i - g.k_min;
      const bool inb = k >= 0 && k < g.n_bins;
#pragma unroll
      for (int c = 0; c < 2; c++) win_at<N, GW>(sm, gw, L, c, i) = inb ? opp[c * g.n_bins + k] : cd{0.0, 0.0};
    }
  }
  for (int s = tid; s < S; s += NT) {
    sm.ex[s] = a.exists[uidx(a, t, w, b, s)];
    for (int k = 0; k < 8; k++) sm.su[s][k] = a.u[8 * uidx(a, t, w, b, s) + k];
  }
  if (tid == 0) sm.entry = pool_acquire(a);
  if (tid < 8) {
    const int k = tid;
    double lo = a.lo[k], hi = a.hi[k];
    if (k == 1) {
      band_f0_range<N>(g, a, b, lo, hi);
    } else if (period_of(k) > 0) {
      lo = 0.0;
      hi = period_of(k);
    }
    sm.blo[k] = lo;
    sm.bhi[k] = hi;
  }
  __syncthreads();
  cd* const spec = sm.entry >= 0 ? a.spec_pool + (int64_t)sm.entry * pool_entry(S, a.n_t, N) : nullptr;

  const double* grp = a.group + (int64_t)b * a.n_w * S * 8;
  const int G = a.group_count[b];
  const int nf = a.n_friends < G ? a.n_friends : G;
  const double lvol = (!inmodel && a.prop_u) ? log_box_volume<N>(g, a, b) : 0.0;

  // spectra and weights at the thread's bins: r (being removed), carried
  // from the plan or the previous pass, and the template just built (h, the
  // one being added when the move is a birth or an in-model move's new
  // template); each is written before it is read.  Only r lives across
  // passes: the added template is consumed in the pass that builds it.
  cd rv[BPT][2], hv[BPT][2];
  double wr[BPT][2], wh[BPT][2];
  int64_t kr = 0;
  unsigned long long n_prop = 0, n_acc = 0, n_bprop = 0, n_bacc = 0, n_dprop = 0, n_dacc = 0;

  // the reversible-jump death of slot s, r's spectrum in rv (start kr,
  // weights wr); lra = ln of the acceptance draw
  auto death = [&](int s, double lra) {
    const double dl = loop_dlogl<N, BPT, GW>(g, sm, gw, L, k0w, false, 0, rv, wr, true, kr, rv, wr, tid);
    const double lpq = a.prop_u ? a.rj_logq[uidx(a, t, w, b, s)] + lvol : 0.0;
    if (lra < beta * dl + lpq) {
      loop_add<N, BPT, GW>(g, sm, gw, L, k0w, kr, 1.0, rv, own, tid);
      if (tid == 0) sm.ex[s] = 0;
      n_dacc++;
    }
    __syncthreads();
  };

  // Block-uniform control: every thread runs the same plan on the same LDS
  // values.  phase 0 removes the band's sources (one build per occupied
  // slot), phase 1 runs the moves, phase 2 ends.  A move builds the removed
  // template first when there is no pool entry (pend then marks it built).
  enum { kSetup = 0, kOld = 1, kNew = 2 };
  int phase = 0, cur = 0, sk = 0;
  bool pend = false;
  double lr_acc = 0.0, lr = 0.0;  // ln of the acceptance draw; in-model: ln z^7
  for (;;) {
    // The thread index and the table pointers pass through an empty asm
    // statement at the top of every pass: the per-thread values derived from
    // them (addresses, twiddles, basis samples) are then recomputed in every
    // pass instead of being hoisted out of the loop, where they would stay
    // live across the whole kernel.
    WaveTables<F> tbl = tb;
    asm volatile("" : "+v"(tid), "+s"(tbl.basis), "+s"(tbl.fft_tw), "+s"(tbl.bin_F), "+s"(tbl.bin_W));
    // ---- plan: advance the moves up to the next template build
    const double* ub = nullptr;
    const cd* rsrc = nullptr;  // a cached spectrum of r to load during the build
    int kind = kSetup;
    while (phase < 2) {
      if (phase == 0) {
        while (cur < S && !sm.ex[cur]) cur++;
        if (cur < S) {
          ub = sm.su[cur];
          kind = kSetup;
          break;
        }
        if (inmodel) {
          // the occupied slots in slot order (in-model moves keep the
          // occupancy) and their friend windows, one wave per slot
          if (tid == 0) {
            int c = 0;
            for (int s = 0; s < S; s++)
              if (sm.ex[s]) sm.order[c++] = s;
            sm.n_occ = c;
          }
          __syncthreads();
          if (G > 0) {
            for (int o = tid / kWave; o < sm.n_occ; o += NT / kWave) {
              const int s = sm.order[o];
              const int st = friend_start(grp, G, nf, sm.su[s][1]);
              if ((tid & (kWave - 1)) == 0) sm.fstart[s] = st;
            }
          }
          __syncthreads();
        } else {
          // flip every slot once in a random order (Fisher-Yates from the
          // top: position j swaps with r_j <= j); the draws in parallel, the
          // swaps on one thread; every flip's uniform draws (words 64 + 16 i
          // + k: k = 0 acceptance, k = 1..8 a prior birth's coordinates)
          for (int j = tid; j < S; j += NT)
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
          // (the acceptance draw is kept as its logarithm)
          for (int q = tid; q < S * 9; q += NT) {
            const int i = q / 9, k = q - 9 * (q / 9);
            const double r = rng_uniform(a.seed, sweep, move, unit, 64 + 16 * (uint64_t)i + k);
            sm.rdraw[i][k] = k == 0 ? log_ni(r) : r;
          }
          __syncthreads();
        }
        phase = 1;
        cur = 0;
        continue;
      }
      if (inmodel) {
        if (cur >= a.n_prop) {
          phase = 2;
          break;
        }
        if (pend) {
          // every wave has read the removed template's decode and bins before
          // the next decode overwrites them (this path has no other barrier
          // since the removed template's build)
          __syncthreads();
          ub = sm.u_new;
          kind = kNew;
          break;
        }
        const int p = cur;
        if ((p & (kMaxSlots - 1)) == 0) {
          // the next kMaxSlots proposals' four draws (words 8 p + k), one per
          // thread; the acceptance draw is kept as its logarithm, and the
          // stretch draw also gives ln z^7 (column 4)
          const int pe = a.n_prop - p < kMaxSlots ? a.n_prop - p : kMaxSlots;
          __syncthreads();
          for (int q = tid; q < 4 * pe; q += NT) {
            const double r = rng_uniform(a.seed, sweep, move, unit, 8 * (uint64_t)(p + (q >> 2)) + (q & 3));
            if ((q & 3) == 2) {
              const double am = a.stretch_a;
              const double z = ((am - 1.0) * r + 1.0) * ((am - 1.0) * r + 1.0) / am;
              sm.rdraw[q >> 2][4] = 7.0 * log_ni(z);
            }
            sm.rdraw[q >> 2][q & 3] = (q & 3) == 3 ? log_ni(r) : r;
          }
          __syncthreads();
        }
        const double* rp = sm.rdraw[p & (kMaxSlots - 1)];
        const double r_pick = rp[0], r_friend = rp[1], r_z = rp[2];
        lr_acc = rp[3];
        const int gcount = sm.n_occ;
        cur++;
        if (gcount == 0) continue;
        sk = sm.order[(int)floor(r_pick * gcount)];
        const double* uk = sm.su[sk];
        n_prop++;
        if (G <= 0) continue;
        const double* X = grp + 8 * (sm.fstart[sk] + (int)floor(r_friend * nf));
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
          const double P = period_of(i);
          if (P > 0) {
            diff = wrap_p(diff + 0.5 * P, P) - 0.5 * P;
            const double zd = z * diff;
            if (!(fabs(zd) < 0.5 * P)) reversible = false;
            un[i] = wrap_p(X[i] + zd, P);
          } else {
            un[i] = X[i] + z * diff;
          }
        }
        if (!reversible || !loop_in_prior<N, GW>(sm, un)) continue;
        lr = rp[4];
        cur--;  // the move is under way
        if (tid < 8) {
          sm.u_old[tid] = uk[tid];
          sm.u_new[tid] = un[tid];
        }
        __syncthreads();
        if (spec) {
          // r's cached spectrum and weights: loaded during the build of the new template
          rsrc = spec + (int64_t)sk * 2 * N;
          kr = sm.sq[sk] - N / 2;
          ub = sm.u_new;
          kind = kNew;
        } else {
          ub = sm.u_old;
          kind = kOld;
        }
        break;
      }
      // reversible jump
      if (cur >= S) {
        phase = 2;
        break;
      }
      const int s = sm.order[cur];
      lr_acc = sm.rdraw[cur][0];
      sk = s;
      if (sm.ex[s]) {
        // death: the new template is zero; with the prior proposal (q = p)
        // only the likelihood enters, otherwise ln q - ln p as well
        n_dprop++;
        if (spec) {
          loop_load<N, BPT>(spec + (int64_t)s * 2 * N, rv, tid);
          kr = sm.sq[s] - N / 2;
          loop_weights<N, BPT>(g, wts, kr, wr, tid);
          death(s, lr_acc);
          cur++;
          continue;
        }
        if (tid < 8) sm.u_old[tid] = sm.su[s][tid];
        __syncthreads();
        ub = sm.u_old;
        kind = kOld;
        break;
      }
      n_bprop++;
      if (a.prop_u) {
        // birth from the given proposal: ln p - ln q enters
        if (tid < 8) sm.u_new[tid] = a.prop_u[8 * uidx(a, t, w, b, s) + tid];
        __syncthreads();
        if (!loop_in_prior<N, GW>(sm, sm.u_new)) {
          __syncthreads();
          cur++;
          continue;
        }
      } else {
        // birth drawn from the prior
        if (tid < 8) sm.u_new[tid] = sm.blo[tid] + (sm.bhi[tid] - sm.blo[tid]) * sm.rdraw[cur][1 + tid];
        __syncthreads();
      }
      ub = sm.u_new;
      kind = kNew;
      break;
    }
    if (phase == 2) break;

    // ---- the template build (the only one)
    loop_build<N, BPT, GW, F>(g, tbl, ub, sm, kind == kSetup ? nullptr : wts, wh, rsrc, kr, rv, wr, tid);
    loop_bins<N, BPT, GW, F>(g, tbl, sm, hv, tid);
    const int64_t kh = sm.src.q - N / 2;
    if (kind == kSetup) {
      // the band's residual: remove the slot's source, keep its spectrum
      if (spec) loop_store<N, BPT>(spec + (int64_t)cur * 2 * N, hv, tid);
      loop_add<N, BPT, GW>(g, sm, gw, L, k0w, kh, -1.0, hv, nullptr, tid);
      if (tid == 0) sm.sq[cur] = sm.src.q;
      __syncthreads();
      cur++;
      continue;
    }
    if (kind == kOld) {
#pragma unroll
      for (int m = 0; m < BPT; m++)
        for (int c = 0; c < 2; c++) {
          rv[m][c] = hv[m][c];
          wr[m][c] = wh[m][c];
        }
      kr = kh;
      if (inmodel) {
        pend = true;  // the new template next
        continue;
      }
      death(sk, lr_acc);
      cur++;
      continue;
    }
    pend = false;
    double dl;
    if (inmodel) {
      // r's spectrum into the workspace for the bins of a's window that need
      // it at another offset
      __syncthreads();
#pragma unroll
      for (int m = 0; m < BPT; m++) {
        sm.buf[tid + NT * m] = rv[m][0];
        sm.buf[N + tid + NT * m] = rv[m][1];
      }
      __syncthreads();
      dl = loop_dlogl<N, BPT, GW>(g, sm, gw, L, k0w, true, kh, hv, wh, true, kr, rv, wr, tid);
    } else {
      dl = loop_dlogl<N, BPT, GW>(g, sm, gw, L, k0w, true, kh, hv, wh, false, 0, rv, wr, tid);
    }
    double thr;
    if (inmodel)
      thr = beta * dl + lr;
    else if (a.prop_u)
      thr = beta * dl - lvol - a.rj_logq[uidx(a, t, w, b, sk)];
    else
      thr = beta * dl;
    if (lr_acc < thr) {
      if (spec) loop_store<N, BPT>(spec + (int64_t)sk * 2 * N, hv, tid);
      loop_add<N, BPT, GW>(g, sm, gw, L, k0w, kh, -1.0, hv, own, tid);
      __syncthreads();
      if (inmodel) {
        loop_add<N, BPT, GW>(g, sm, gw, L, k0w, kr, 1.0, rv, own, tid);
        // the moved slot's friend window (every wave searches, one thread writes)
        const int st = friend_start(grp, G, nf, sm.u_new[1]);
        if (tid == 0) sm.fstart[sk] = st;
        n_acc++;
      } else {
        if (tid == 0) sm.ex[sk] = 1;
        n_bacc++;
      }
      if (tid < 8) sm.su[sk][tid] = sm.u_new[tid];
      if (tid == 0) sm.sq[sk] = sm.src.q;
    }
    __syncthreads();
    cur++;
  }
  // the set's window sum for the tempering pass: H = (opposite-parity
  // window) - (final window); that buffer does not change during the pass
  // (in place when the window is the entry itself)
  if (a.wsum) {
    const cd* opp = a.resid + ((int64_t)(1 - (b & 1)) * a.n_w + w) * 2 * g.n_bins;
    cd* H = wsum_entry<N>(a, t, w, b);
    for (int i = tid; i < L; i += NT) {
      const int64_t k = k0w + i - g.k_min;
      const bool inb = k >= 0 && k < g.n_bins;
#pragma unroll
      for (int c = 0; c < 2; c++)
        H[c * L + i] = inb ? opp[c * g.n_bins + k] - win_at<N, GW>(sm, gw, L, c, i) : cd{0.0, 0.0};
    }
  }
  for (int s = tid; s < S; s += NT) {
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

// band log-likelihood -1/2 <R - H | R - H> over band b's window [k0w, k0w +
// L), R = walker w_res's opposite-parity buffer, weights 1/S of w_res
template <int N>
__device__ __forceinline__ double band_set_loglike_h(const Geo& g, const SweepArgs& a, int b, int w_res, int64_t k0w,
                                                     int L, const cd* H, double* red) {
  constexpr int NT = block_threads<N>();
  const cd* opp = a.resid + ((int64_t)(1 - (b & 1)) * a.n_w + w_res) * 2 * g.n_bins;
  const double* ip = a.inv_psd + (int64_t)w_res * 2 * g.n_bins;
  double rr = 0.0;
  for (int i = threadIdx.x; i < L; i += NT) {
    const int64_t k = k0w + i - g.k_min;
    if (k < 0 || k >= g.n_bins) continue;
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const cd r = opp[c * g.n_bins + k] - H[c * L + i];
      rr += (r.re * r.re + r.im * r.im) * ip[c * g.n_bins + k];
    }
  }
  double sums[1] = {rr};
  block_allsum<NT>(sums, red);
  rr = sums[0];
  return -0.5 * g.df4 * rr;
}

// LDS of the tempering kernel with window sums: the block reduction only
template <int N>
struct PtSumsSmem {
  double red[2 * (block_threads<N>() / kWave)];
  int entry;
};

// WS: the sweep carries window sums (every set's sum comes from the band
// passes, no template is built here, and the LDS shrinks to the reduction)
template <int N, bool WS>
__global__ __launch_bounds__(block_threads<N>()) void k_sweep_pt(Geo g, WaveTables<double> tb, SweepArgs a,
                                                                 int parity) {
  __shared__ std::conditional_t<WS, PtSumsSmem<N>, BandSmem<N>> sm;
  __shared__ int wt[256];
  __shared__ double Lc[256];
  __shared__ int hidx[256];  // window sum of the set at temperature t: entry slot hidx[t]
  const int nbp = (a.n_b - parity + 1) / 2;
  int bi, i;
  band_block(nbp, a.n_w, bi, i);
  const int b = parity + 2 * bi;
  const int tid = threadIdx.x;
  const int nt = a.n_t;
  const int64_t sweep = *a.sweep_ctr;
  const int64_t k0w = win_k0<N>(a, b);
  const int L = win_len<N>(a.band_w);  // 3N unless the window sums carry wider windows
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
  // window sums of the sets: from the band passes (wsum, entries that move
  // with the sets), else built here into a pool entry (hidx maps a
  // temperature to its set's sum), else recomputed on every evaluation
  constexpr bool ws = WS;  // (the launch picks WS by a.wsum != nullptr)
  if (tid == 0) sm.entry = ws ? -1 : pool_acquire(a);
  for (int t = tid; t < nt; t += block_threads<N>()) hidx[t] = t;
  __syncthreads();
  cd* const Hp = sm.entry >= 0 ? a.spec_pool + (int64_t)sm.entry * pool_entry(a.n_slot, nt, N) : nullptr;
  const bool Hs = ws || Hp;
  auto Hof = [&](int t) { return ws ? wsum_entry<N>(a, t, wt[t], b) : Hp + (int64_t)hidx[t] * 6 * N; };
  for (int t = 0; t < nt; t++) {
    double lnl;
    if constexpr (WS) {
      lnl = band_set_loglike_h<N>(g, a, b, wt[t], k0w, L, Hof(t), sm.red);
    } else if (Hs) {
      band_set_sum<N>(g, tb, a, t, wt[t], b, k0w, sm, Hof(t));
      lnl = band_set_loglike_h<N>(g, a, b, wt[t], k0w, L, Hof(t), sm.red);
    } else {
      if constexpr (pt_lds_window<N>())
        lnl = band_set_loglike<N>(g, tb, a, t, wt[t], b, wt[t], k0w, sm);
      else
        lnl = qnan();  // not reached: N = 1024 sweeps carry window sums
    }
    if (tid == 0) Lc[t] = lnl;
  }
  __syncthreads();
  const double* bt = a.betas + (int64_t)b * nt;
  unsigned long long n_prop = 0, n_acc = 0;
  for (int t = nt - 1; t >= 1; t--) {
    // log-likelihood of the set at temperature ts against walker w_res's residual
    auto set_ll = [&](int ts, int w_res) -> double {
      if (Hs) return band_set_loglike_h<N>(g, a, b, w_res, k0w, L, Hof(ts), sm.red);
      if constexpr (!WS && pt_lds_window<N>())
        return band_set_loglike<N>(g, tb, a, ts, wt[ts], b, w_res, k0w, sm);
      else
        return qnan();  // not reached: N = 1024 sweeps carry window sums
    };
    const double L1 = set_ll(t - 1, wt[t]);
    const double L2 = set_ll(t, wt[t - 1]);
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
        for (int i2 = tid; i2 < L; i2 += block_threads<N>()) {
          const int64_t k = k0w + i2 - g.k_min;
          if (k < 0 || k >= g.n_bins) continue;
#pragma unroll
          for (int c = 0; c < 2; c++) {
            const cd d = H0[c * L + i2] - H1[c * L + i2];
            double* dst = reinterpret_cast<double*>(own + c * g.n_bins + k);
            atomicAdd(dst, d.re);
            atomicAdd(dst + 1, d.im);
          }
        }
        __syncthreads();
      } else if (t == 1) {
        if constexpr (!WS && pt_lds_window<N>()) {
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
      }
      // exchange the source sets of (t, w_t) and (t-1, w_(t-1)), with their
      // window sums
      if (ws) {
        cd* h1 = Hof(t);
        cd* h2 = Hof(t - 1);
        for (int i2 = tid; i2 < 2 * L; i2 += block_threads<N>()) {
          const cd tmp = h1[i2];
          h1[i2] = h2[i2];
          h2[i2] = tmp;
        }
      }
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
      const double lo = (double)(a.k_band0 + (int64_t)b * a.band_w) / g.T;
      const double hi = (double)(a.k_band0 + (int64_t)(b + 1) * a.band_w) / g.T;
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
