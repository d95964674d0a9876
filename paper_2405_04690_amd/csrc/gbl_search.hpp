// gbl_search.hpp -- per-sub-band search for the loudest remaining source
// (appendix "Algorithm for fitting proposal distributions"; the search RJ
// proposal of Sec. 4): independent fixed-dimensional (one source, d = 8)
// parallel-tempered ensembles, one per sub-band, with the stretch move of
// eq. stretch, the prior confining f0 to the sub-band, and the likelihood
// gain of adding the source (eq. addsource) as target.  The likelihoods come
// from the batched fused likelihood kernels (births: old amplitude 0); these
// kernels only propose, accept, swap and keep the best point.
//
// State (caller-owned device arrays):
//   u [n_b][n_t][n_w][8] sampling coordinates, logl [n_b][n_t][n_w],
//   betas [n_t], best_u [n_b][8], best_logl [n_b], stall [n_b], stats [4];
// workspace per chain slot s (n_b n_t n_w of them): the proposal in sampling
// coordinates [8], its physical parameters [8] and the zero-amplitude copy
// [8] (a birth's old template), its likelihood, ln z^7, the prior flag, and a
// zero index.
#pragma once

#include "gbl_sampler.hpp"

namespace gbl {

enum { kMoveSearch = 6, kMoveSearchPT = 7, kMoveSearchBall = 8 };

struct Sigma8 {
  double v[8];
};

struct SearchArgs {
  int n_b, n_t, n_w, width, n_stall;
  int64_t k_band0;
  double stretch_a;
  uint64_t seed;
  double lo[8], hi[8];
  double* u;
  double* logl;
  const double* betas;
  double* best_u;
  double* best_logl;
  int32_t* stall;
  unsigned long long* stats;
  // workspace
  double* wu;    // [n_slots][8]
  double* wpn;   // [n_slots][8]
  double* wpo;   // [n_slots][8]
  double* wl;    // [n_slots]
  double* wlz;   // [n_slots]
  int32_t* wok;  // [n_slots]
  int32_t* widx; // [n_slots] zeros
};

__device__ __forceinline__ double search_period(int k) { return k == 3 ? kTwoPi : k == 5 ? kPi : k == 6 ? kTwoPi : 0.0; }

__device__ __forceinline__ void search_box(const Geo& g, const SearchArgs& a, int b, double* lo, double* hi) {
#pragma unroll
  for (int k = 0; k < 8; k++) {
    lo[k] = a.lo[k];
    hi[k] = a.hi[k];
    if (search_period(k) > 0) {
      lo[k] = 0.0;
      hi[k] = search_period(k);
    }
  }
  lo[1] = (double)(a.k_band0 + (int64_t)b * a.width) / g.T;
  hi[1] = (double)(a.k_band0 + (int64_t)(b + 1) * a.width) / g.T;
}

// sampling -> physical coordinates (amplitude, inclination, latitude mapped back)
__device__ __forceinline__ void search_physical(const double* u, double* p, bool zero_amp) {
  p[0] = zero_amp ? 0.0 : exp10(u[0]);
  p[1] = u[1];
  p[2] = u[2];
  p[3] = u[3];
  p[4] = acos(u[4]);
  p[5] = u[5];
  p[6] = u[6];
  p[7] = asin(u[7]);
}

// proposals of half h: one thread per (b, t, i), slot s = (b n_t + t) n_w/2 + i
__global__ void k_search_propose(Geo g, SearchArgs a, int64_t iter, int h) {
  const int half = a.n_w / 2;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (int64_t)a.n_b * a.n_t * half) return;
  const int i = (int)(s % half);
  const int bt = (int)(s / half);
  const int t = bt % a.n_t, b = bt / a.n_t;
  const int w = 2 * i + h;
  double P[8];
  double* out = a.wu + 8 * s;
  bool ok = false;
  double lz = 0.0;
  if (a.stall[b] < a.n_stall) {
    const uint64_t unit = ((uint64_t)b * a.n_t + t) * a.n_w + w;
    const double r_pick = rng_uniform(a.seed, iter, kMoveSearch, unit, 4 * (uint64_t)h + 0);
    const double r_z = rng_uniform(a.seed, iter, kMoveSearch, unit, 4 * (uint64_t)h + 1);
    const int j = 2 * (int)floor(r_pick * half) + (1 - h);
    const double am = a.stretch_a;
    const double z = ((am - 1.0) * r_z + 1.0) * ((am - 1.0) * r_z + 1.0) / am;
    const double* X = a.u + 8 * (((int64_t)b * a.n_t + t) * a.n_w + j);
    const double* Y = a.u + 8 * (((int64_t)b * a.n_t + t) * a.n_w + w);
    bool rev = true;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      double diff = Y[k] - X[k];
      const double Pk = search_period(k);
      if (Pk > 0) {
        diff = wrap_p(diff + 0.5 * Pk, Pk) - 0.5 * Pk;
        if (!(fabs(z * diff) < 0.5 * Pk)) rev = false;
        P[k] = wrap_p(X[k] + z * diff, Pk);
      } else {
        P[k] = X[k] + z * diff;
      }
    }
    double lo[8], hi[8];
    search_box(g, a, b, lo, hi);
    bool inside = P[1] >= lo[1] && P[1] < hi[1];
#pragma unroll
    for (int k = 0; k < 8; k++)
      if (k != 1 && search_period(k) == 0.0) inside = inside && P[k] >= lo[k] && P[k] <= hi[k];
    ok = rev && inside;
    lz = 7.0 * log(z);
  } else {
#pragma unroll
    for (int k = 0; k < 8; k++) P[k] = a.u[8 * (((int64_t)b * a.n_t + t) * a.n_w + w) + k];
  }
#pragma unroll
  for (int k = 0; k < 8; k++) out[k] = P[k];
  // a proposal outside the prior still gets finite parameters (its likelihood is unused)
  double Q[8];
#pragma unroll
  for (int k = 0; k < 8; k++) Q[k] = P[k];
  if (!ok) {
    Q[4] = fmin(fmax(Q[4], -1.0), 1.0);
    Q[7] = fmin(fmax(Q[7], -1.0), 1.0);
  }
  search_physical(Q, a.wpn + 8 * s, false);
  search_physical(Q, a.wpo + 8 * s, true);
  a.wok[s] = ok ? 1 : 0;
  a.wlz[s] = lz;
  a.widx[s] = 0;
}

// Metropolis step of half h with the likelihoods in wl
__global__ void k_search_accept(SearchArgs a, int64_t iter, int h) {
  const int half = a.n_w / 2;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (int64_t)a.n_b * a.n_t * half) return;
  const int i = (int)(s % half);
  const int bt = (int)(s / half);
  const int t = bt % a.n_t, b = bt / a.n_t;
  const int w = 2 * i + h;
  if (a.stall[b] >= a.n_stall) return;
  atomicAdd(&a.stats[0], 1ull);
  if (!a.wok[s]) return;
  const int64_t c = ((int64_t)b * a.n_t + t) * a.n_w + w;
  const uint64_t unit = ((uint64_t)b * a.n_t + t) * a.n_w + w;
  const double r_acc = rng_uniform(a.seed, iter, kMoveSearch, unit, 4 * (uint64_t)h + 2);
  if (log(r_acc) < a.betas[t] * (a.wl[s] - a.logl[c]) + a.wlz[s]) {
#pragma unroll
    for (int k = 0; k < 8; k++) a.u[8 * c + k] = a.wu[8 * s + k];
    a.logl[c] = a.wl[s];
    atomicAdd(&a.stats[1], 1ull);
  }
}

// temperature swaps per (band, walker), hottest pair first (eq. temp-orig),
// then the band's best cold-chain point (one thread per band, after a grid
// barrier between the two kernels)
__global__ void k_search_swap(SearchArgs a, int64_t iter) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)a.n_b * a.n_w) return;
  const int b = (int)(q / a.n_w), w = (int)(q % a.n_w);
  if (a.stall[b] >= a.n_stall) return;
  unsigned long long np = 0, na = 0;
  for (int t = a.n_t - 1; t >= 1; t--) {
    np++;
    const double r = rng_uniform(a.seed, iter, kMoveSearchPT, (uint64_t)b * a.n_w + w, (uint64_t)t);
    const int64_t c1 = ((int64_t)b * a.n_t + t) * a.n_w + w, c0 = ((int64_t)b * a.n_t + t - 1) * a.n_w + w;
    if (log(r) < (a.betas[t - 1] - a.betas[t]) * (a.logl[c1] - a.logl[c0])) {
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const double tmp = a.u[8 * c1 + k];
        a.u[8 * c1 + k] = a.u[8 * c0 + k];
        a.u[8 * c0 + k] = tmp;
      }
      const double tl = a.logl[c1];
      a.logl[c1] = a.logl[c0];
      a.logl[c0] = tl;
      na++;
    }
  }
  if (np) atomicAdd(&a.stats[2], np);
  if (na) atomicAdd(&a.stats[3], na);
}

__global__ void k_search_best(SearchArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_b || a.stall[b] >= a.n_stall) return;
  const double* L = a.logl + (int64_t)b * a.n_t * a.n_w;   // the cold rung's walkers
  int wb = 0;
  for (int w = 1; w < a.n_w; w++)
    if (L[w] > L[wb]) wb = w;
  if (L[wb] > a.best_logl[b]) {
    a.best_logl[b] = L[wb];
#pragma unroll
    for (int k = 0; k < 8; k++) a.best_u[8 * b + k] = a.u[8 * ((int64_t)b * a.n_t * a.n_w + wb) + k];
    a.stall[b] = 0;
  } else {
    a.stall[b] += 1;
  }
}

// every chain of every band to best_u + sigma n (Box-Muller normals from the
// uniforms of unit (b n_t + t) n_w + w, move 8, draws 2p, 2p+1), periodic
// coordinates wrapped, the others clamped into the box (f0 strictly below
// the band's top); the chains' parameters go to the workspace for the
// likelihood pass; stall cleared
__global__ void k_search_ball(Geo g, SearchArgs a, int64_t iter, Sigma8 sigma) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)a.n_b * a.n_t * a.n_w) return;
  const int w = (int)(c % a.n_w);
  const int t = (int)((c / a.n_w) % a.n_t);
  const int b = (int)(c / ((int64_t)a.n_w * a.n_t));
  double lo[8], hi[8];
  search_box(g, a, b, lo, hi);
  const uint64_t unit = ((uint64_t)b * a.n_t + t) * a.n_w + w;
  double* x = a.u + 8 * c;
  for (int p = 0; p < 4; p++) {
    const double u1 = rng_uniform(a.seed, iter, kMoveSearchBall, unit, 2 * (uint64_t)p);
    const double u2 = rng_uniform(a.seed, iter, kMoveSearchBall, unit, 2 * (uint64_t)p + 1);
    const double r = sqrt(-2.0 * log(u1));
    const double n0 = r * cos(2.0 * kPi * u2), n1 = r * sin(2.0 * kPi * u2);
    for (int q = 0; q < 2; q++) {
      const int k = 2 * p + q;
      double v = a.best_u[8 * b + k] + sigma.v[k] * (q ? n1 : n0);
      if (search_period(k) > 0) {
        v = wrap_p(v, search_period(k));
      } else {
        const double top = k == 1 ? nextafter(hi[k], lo[k]) : hi[k];
        v = v < lo[k] ? lo[k] : (v > top ? top : v);
      }
      x[k] = v;
    }
  }
  search_physical(x, a.wpn + 8 * c, false);
  search_physical(x, a.wpo + 8 * c, true);
  a.widx[c] = 0;
  if (t == 0 && w == 0) a.stall[b] = 0;
}

// chain parameters into the workspace for a full likelihood pass
__global__ void k_search_params(SearchArgs a) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)a.n_b * a.n_t * a.n_w) return;
  search_physical(a.u + 8 * c, a.wpn + 8 * c, false);
  search_physical(a.u + 8 * c, a.wpo + 8 * c, true);
  a.widx[c] = 0;
}

}  // namespace gbl
