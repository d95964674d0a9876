// gbl_flow.hpp -- the learned reversible-jump proposal: a conditional
// affine-coupling flow over the sampler's coordinates, on BF16 MFMA.
//
// The paper fits its RJ proposals with Gaussian mixtures and plans
// normalizing flows in their place (Discussion, "Single source
// search-to-parameter estimation information transfer"; appendix "Algorithm
// for fitting proposal distributions").  Form of the flow (a reading):
//   x_i = logit((u_i - lo_i) / (hi_i - lo_i)) over the prior box of sub-band b;
//   six coupling layers, layer l keeps C_l = (0,2,4,6) (l even) or (1,3,5,7)
//   and moves the other four: y_T = x_T exp(s) + t, (s_hat, t) = MLP([x_C, E[b]]),
//   s = 2 tanh(s_hat); MLP 20 -> 128 -> 128 -> 8 with SiLU;
//   ln q_x = sum ln N(z_i) + sum of s;  ln q_u = ln q_x + sum ln |dx_i/du_i|.
//
// Arithmetic: weights, embeddings and activations enter the MFMAs as BF16
// (round to nearest even), products accumulate in FP32, SiLU / tanh in FP32.
// The flow state x, the affine updates, the box map and the log-density sums
// are FP64.  Because a coupling layer feeds its conditioner the unchanged
// coordinates, the forward and inverse passes evaluate (s, t) on identical
// inputs: the sampling map is an exact bijection (to FP64 rounding) and the
// density returned with a sample equals the density evaluated at it later.
//
// MFMA orientation: v_mfma_f32_16x16x32_bf16 with features on the M axis and
// 16 samples on the N axis.  A operand: lane (r = lane % 16, g = lane / 16)
// holds row r, K slots 8g..8g+7; B operand: lane (c, g) holds column c, the
// same K slots; D: lane (c, g) holds column c, rows 4g..4g+3.  A layer's
// output tiles 2kb and 2kb+1 therefore form the next layer's K block kb when
// K slot (g, i) stands for feature 32kb + 4g + i (i < 4) or 32kb + 16 + 4g +
// (i - 4) (i >= 4); the weights are stored pre-permuted in that order, so
// hidden activations never leave registers in the forward pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbl {
namespace flow {

constexpr int kD = 8, kLayers = 6, kH = 128, kEmb = 16, kCin = 20, kOut = 8;
constexpr int oW1 = 0, oB1 = kH * kCin, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kOut * kH;
constexpr int kLayerParams = oB3 + kOut;  // 20232
// fragments (64 lanes x 16 B) per layer: forward W1 [8 mt], W2 [8 mt][4 kb], W3 [4 kb];
// backward W3^T [8 mt], W2^T [8 mt][4 kb], W1^T [2 mt][4 kb]
constexpr int fW1 = 0, fW2 = 8, fW3 = 40, fW3t = 44, fW2t = 52, fW1t = 84, kFragPerLayer = 92;
constexpr int64_t kPackedBytes = (int64_t)kLayers * kFragPerLayer * 64 * 16;
constexpr int kMaxGroups = 64;  // work-groups of the gradient kernel (partial-sum slots)
constexpr int kChunk = 64;      // samples per gradient work-group pass
constexpr int kPitch = 72;      // LDS row pitch (bf16) of the [feature][sample] tiles

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

struct FlowArgs {
  const float* params;      // FP32 master weights
  const u32x4_t* packed;    // BF16 fragments
  int32_t n_emb, width;
  int64_t k_band0;
  double T;
  double lo[8], hi[8];      // prior box (f0 and the periodic angles are set per band)
  // sample i's band when no band array is given: (i / band_div) % band_mod
  int64_t band_div;
  int32_t band_mod;
  // with a mask, sample i is processed only if mask[i] == mask_want
  int32_t mask_want;
  const int32_t* mask;
};

__device__ __forceinline__ uint32_t bf16_bits(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t pack2(float a, float b) { return bf16_bits(a) | (bf16_bits(b) << 16); }
__device__ __forceinline__ u32x4_t pack8(const float* v) {
  u32x4_t r;
  r[0] = pack2(v[0], v[1]);
  r[1] = pack2(v[2], v[3]);
  r[2] = pack2(v[4], v[5]);
  r[3] = pack2(v[6], v[7]);
  return r;
}
__device__ __forceinline__ u32x4_t pack_tiles(f32x4_t lo, f32x4_t hi) {
  u32x4_t r;
  r[0] = pack2(lo[0], lo[1]);
  r[1] = pack2(lo[2], lo[3]);
  r[2] = pack2(hi[0], hi[1]);
  r[3] = pack2(hi[2], hi[3]);
  return r;
}
__device__ __forceinline__ f32x4_t mfma(u32x4_t a, u32x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

__device__ __forceinline__ float silu(float a) { return a / (1.0f + __expf(-a)); }
__device__ __forceinline__ float silu_grad(float a) {
  const float sg = 1.0f / (1.0f + __expf(-a));
  return sg * (1.0f + a * (1.0f - sg));
}

// K slot (g, i) of block kb -> feature
__device__ __forceinline__ int perm_feature(int kb, int g, int i) {
  return 32 * kb + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}

// ---------------------------------------------------------------------------
// packing: FP32 master -> BF16 fragments (one thread per layer x fragment x lane)
// ---------------------------------------------------------------------------
__global__ void k_flow_pack(const float* __restrict__ P, u32x4_t* __restrict__ out) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= kLayers * kFragPerLayer * 64) return;
  const int lane = id & 63;
  const int f = (id >> 6) % kFragPerLayer;
  const int l = (id >> 6) / kFragPerLayer;
  const float* W = P + (int64_t)l * kLayerParams;
  const int r = lane & 15, g = lane >> 4;
  float v[8];
  for (int i = 0; i < 8; i++) {
    float x = 0.0f;
    if (f < fW2) {  // W1 [out][in]: row 16 mt + r, K slot 8g + i (natural order, in < 20)
      const int mt = f - fW1, in = 8 * g + i;
      if (in < kCin) x = W[oW1 + (16 * mt + r) * kCin + in];
    } else if (f < fW3) {
      const int mt = (f - fW2) >> 2, kb = (f - fW2) & 3;
      x = W[oW2 + (16 * mt + r) * kH + perm_feature(kb, g, i)];
    } else if (f < fW3t) {
      const int kb = f - fW3;
      if (r < kOut) x = W[oW3 + r * kH + perm_feature(kb, g, i)];
    } else if (f < fW2t) {  // W3^T: row = input feature 16 mt + r, K slot (0, i) = output i
      const int mt = f - fW3t;
      if (g == 0) x = W[oW3 + i * kH + 16 * mt + r];
    } else if (f < fW1t) {
      const int mt = (f - fW2t) >> 2, kb = (f - fW2t) & 3;
      x = W[oW2 + perm_feature(kb, g, i) * kH + 16 * mt + r];
    } else {
      const int mt = (f - fW1t) >> 2, kb = (f - fW1t) & 3, in = 16 * mt + r;
      if (in < kCin) x = W[oW1 + perm_feature(kb, g, i) * kCin + in];
    }
    v[i] = x;
  }
  out[id] = pack8(v);
}

// ---------------------------------------------------------------------------
// box map
// ---------------------------------------------------------------------------
__device__ __forceinline__ void box_of(const FlowArgs& fa, int b, double* lo, double* hi) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    lo[i] = fa.lo[i];
    hi[i] = fa.hi[i];
  }
  lo[1] = ((double)fa.k_band0 + ((double)b - 0.5) * fa.width) / fa.T;
  hi[1] = ((double)fa.k_band0 + ((double)b + 1.5) * fa.width) / fa.T;
  lo[3] = 0.0;
  hi[3] = 6.283185307179586476925286766559;
  lo[5] = 0.0;
  hi[5] = 3.1415926535897932384626433832795;
  lo[6] = 0.0;
  hi[6] = 6.283185307179586476925286766559;
}

// ---------------------------------------------------------------------------
// conditioner of one layer for the 16 samples of a wave
// ---------------------------------------------------------------------------
struct CondOut {
  f32x4_t a1[8], a2[8], o;
};

// h0 B operand of lane (c, g): features 8g..8g+7 of [x_C (4), E[b] (16), 0 ...]
__device__ __forceinline__ u32x4_t h0_operand(int g, const double* xc, const float* emb) {
  float v[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const int f = 8 * g + i;
    v[i] = f < 4 ? (float)xc[f] : (f < kCin ? emb[f - 4] : 0.0f);
  }
  return pack8(v);
}

__device__ __forceinline__ void conditioner(const float* __restrict__ W, const u32x4_t* __restrict__ pk, int lane,
                                            u32x4_t h0, CondOut& co) {
  const int g = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 8; mt++) {
    const float4 b = *reinterpret_cast<const float4*>(W + oB1 + 16 * mt + 4 * g);
    co.a1[mt] = mfma(pk[(fW1 + mt) * 64 + lane], h0, f32x4_t{b.x, b.y, b.z, b.w});
  }
  u32x4_t hb[4];
#pragma unroll
  for (int kb = 0; kb < 4; kb++) {
    f32x4_t s0, s1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      s0[j] = silu(co.a1[2 * kb][j]);
      s1[j] = silu(co.a1[2 * kb + 1][j]);
    }
    hb[kb] = pack_tiles(s0, s1);
  }
#pragma unroll
  for (int mt = 0; mt < 8; mt++) {
    const float4 b = *reinterpret_cast<const float4*>(W + oB2 + 16 * mt + 4 * g);
    f32x4_t acc{b.x, b.y, b.z, b.w};
#pragma unroll
    for (int kb = 0; kb < 4; kb++) acc = mfma(pk[(fW2 + 4 * mt + kb) * 64 + lane], hb[kb], acc);
    co.a2[mt] = acc;
  }
#pragma unroll
  for (int kb = 0; kb < 4; kb++) {
    f32x4_t s0, s1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      s0[j] = silu(co.a2[2 * kb][j]);
      s1[j] = silu(co.a2[2 * kb + 1][j]);
    }
    hb[kb] = pack_tiles(s0, s1);
  }
  f32x4_t acc{0.f, 0.f, 0.f, 0.f};
  if (g < 2) {
    const float4 b = *reinterpret_cast<const float4*>(W + oB3 + 4 * g);
    acc = f32x4_t{b.x, b.y, b.z, b.w};
  }
#pragma unroll
  for (int kb = 0; kb < 4; kb++) acc = mfma(pk[(fW3 + kb) * 64 + lane], hb[kb], acc);
  co.o = acc;
}

__device__ __forceinline__ void kept_of(const double* x, int parity, double* xc) {
#pragma unroll
  for (int j = 0; j < 4; j++) xc[j] = parity ? x[2 * j + 1] : x[2 * j];
}

// ---------------------------------------------------------------------------
// inference: ln q_u at given u (kSample = false) or samples from normals z
// (kSample = true).  One wave per 16 samples; lanes with g = 0 own the state.
// ---------------------------------------------------------------------------
// One tile of 16 samples on the calling wave (every lane takes part): lane
// (c, g) works on sample idx (the same for the four lanes of column c);
// inb = false marks a column without a sample (no output).  `in` and `u_out`
// may be the same buffer (each sample is read, then written, by the same
// lane).
template <bool kSample>
__device__ __forceinline__ void flow_tile(const FlowArgs& fa, const double* in, const int32_t* __restrict__ band,
                                          int64_t idx, bool inb, double* u_out, double* __restrict__ logq,
                                          int lane) {
  const int c = lane & 15, g = lane >> 4;
  int b = inb ? (band ? band[idx] : (int)((idx / fa.band_div) % fa.band_mod)) : 0;
  bool valid = inb && b >= 0 && b < fa.n_emb;
  if (!valid) b = 0;
  double lo[8], hi[8];
  box_of(fa, b, lo, hi);
  double x[8], lz = 0.0, logjac = 0.0, logdet = 0.0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const double v = valid ? in[idx * 8 + i] : 0.0;
    if (kSample) {
      x[i] = v;
      lz += -0.5 * v * v;
    } else {
      const double w = hi[i] - lo[i];
      const double p = (v - lo[i]) / w;
      x[i] = log(p) - log1p(-p);
      logjac += -log(w) - log(p) - log1p(-p);
      if (!(p > 0.0 && p < 1.0)) valid = false;
    }
  }
  if (!valid) {
#pragma unroll
    for (int i = 0; i < 8; i++) x[i] = 0.0;
  }
  float emb[16];
  const float* E = fa.params + (int64_t)kLayers * kLayerParams + (int64_t)b * kEmb;
#pragma unroll
  for (int i = 0; i < 16; i++) emb[i] = E[i];
  for (int step = 0; step < kLayers; step++) {
    const int l = kSample ? kLayers - 1 - step : step;
    const int par = l & 1;
    double xc[4];
    kept_of(x, par, xc);
    CondOut co;
    conditioner(fa.params + (int64_t)l * kLayerParams, fa.packed + (int64_t)l * kFragPerLayer * 64, lane,
                h0_operand(g, xc, emb), co);
    float tt[4];
#pragma unroll
    for (int j = 0; j < 4; j++) tt[j] = __shfl(co.o[j], c + 16, 64);
    if (g == 0) {
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const double s = (double)(2.0f * tanhf(co.o[j]));
        const double es = exp(s);
        const int d = 2 * j + 1 - par;
        double xd = par ? x[2 * j] : x[2 * j + 1];
        xd = kSample ? (xd - (double)tt[j]) / es : xd * es + (double)tt[j];
        if (par)
          x[2 * j] = xd;
        else
          x[2 * j + 1] = xd;
        (void)d;
        logdet += s;
      }
    }
  }
  if (g == 0 && inb) {
    if (!valid) {
      if (kSample)
        for (int i = 0; i < 8; i++) u_out[idx * 8 + i] = __builtin_nan("");
      logq[idx] = __builtin_nan("");
      return;
    }
    const double ln2pi_half = 0.91893853320467274178032973640562;
    if (kSample) {
      for (int i = 0; i < 8; i++) {
        const double p = 1.0 / (1.0 + exp(-x[i]));
        const double w = hi[i] - lo[i];
        u_out[idx * 8 + i] = lo[i] + w * p;
        logjac += -log(w) - log(p) - log1p(-p);
      }
      logq[idx] = lz - 8.0 * ln2pi_half + logdet + logjac;
    } else {
      double s2 = 0.0;
      for (int i = 0; i < 8; i++) s2 += x[i] * x[i];
      logq[idx] = -0.5 * s2 - 8.0 * ln2pi_half + logdet + logjac;
    }
  }
}

// Samples [0, B), or with a mask only those with mask[i] == mask_want.  Large
// masked passes (one kind of RJ candidate out of all slots) gather their
// samples first: each wave takes windows of up to 256 indices, collects the
// matching ones in LDS by ballot and runs full tiles of 16 over them, so a
// pass costs tiles in proportion to its samples, not to all slots; small
// ones keep one tile per 16 slots, which spreads them over more waves.  A
// sample's result does not depend on its tile-mates (each MFMA output column
// belongs to one sample).
template <bool kSample>
__global__ __launch_bounds__(256) void k_flow_apply(FlowArgs fa, const double* in, const int32_t* __restrict__ band,
                                                   int64_t B, double* u_out, double* __restrict__ logq) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  constexpr int64_t kGatherMin = 4096LL * 64;  // below: too few windows to fill the chip
  if (!fa.mask || B < kGatherMin) {
    // tiles of 16 consecutive samples (masked-out samples ride along unwritten)
    const int64_t n_tiles = (B + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < n_tiles; tile += (int64_t)gridDim.x * 4) {
      const int64_t idx = tile * 16 + (lane & 15);
      const bool inb = idx < B && (!fa.mask || fa.mask[idx] == fa.mask_want);
      flow_tile<kSample>(fa, in, band, idx, inb, u_out, logq, lane);
    }
    return;
  }
  constexpr int kMaxWin = 256;
  __shared__ int32_t found[4][kMaxWin];  // per wave: offsets of the window's matching samples
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes under this one
  // windows of 64 k indices, k = 1, 2 or 4: as wide as leaves at least 4,096
  // windows (16 per CU) to spread over the chip
  const int nk = B >= 4096LL * 256 ? 4 : (B >= 4096LL * 128 ? 2 : 1);
  const int64_t n_win = (B + 64 * nk - 1) / (64 * nk);
  for (int64_t win = (int64_t)blockIdx.x * 4 + wv; win < n_win; win += (int64_t)gridDim.x * 4) {
    const int64_t base = win * 64 * nk;
    int cnt = 0;  // uniform over the wave
    for (int k = 0; k < nk; k++) {
      const int64_t i = base + 64 * k + lane;
      const bool m = i < B && fa.mask[i] == fa.mask_want;
      const uint64_t bal = __ballot(m);
      if (m) found[wv][cnt + __popcll(bal & below)] = 64 * k + lane;
      cnt += __popcll(bal);
    }
    // (a wave's LDS accesses complete in order: the reads below see the writes above)
    for (int t0 = 0; t0 < cnt; t0 += 16) {
      const int j = t0 + (lane & 15);
      const bool inb = j < cnt;
      const int64_t idx = inb ? base + found[wv][j] : 0;
      flow_tile<kSample>(fa, in, band, idx, inb, u_out, logq, lane);
    }
  }
}

// ---------------------------------------------------------------------------
// training: gradient of the mean negative log-density.  One work-group of
// four waves per 64-sample chunk (persistent over chunks); per layer the
// conditioner is recomputed from the stored layer input, the data gradients
// run through the transposed fragments, and the weight gradients are MFMA
// contractions over the chunk's samples from [feature][sample] LDS tiles,
// summed into the work-group's own FP32 partial slot (a fixed-order reduction
// follows).  Embedding gradients go to `gradE` with FP32 atomics.
// ---------------------------------------------------------------------------
struct GradSmem {
  double xs[kLayers + 1][kChunk][8];
  uint16_t h0[32][kPitch], h1[kH][kPitch], h2[kH][kPitch];
  uint16_t d1[kH][kPitch], d2[kH][kPitch], d3[16][kPitch];
  double loss;
};

__device__ __forceinline__ void lds_put(uint16_t* row, int col, float v) { row[col] = (uint16_t)bf16_bits(v); }

__device__ __forceinline__ u32x4_t lds_frag(const uint16_t (*t)[kPitch], int row, int kb, int g) {
  return *reinterpret_cast<const u32x4_t*>(&t[row][32 * kb + 8 * g]);
}

__global__ __launch_bounds__(256) void k_flow_grad(FlowArgs fa, const double* __restrict__ u,
                                                  const int32_t* __restrict__ band, int64_t B,
                                                  float* __restrict__ partial, double* __restrict__ loss_part,
                                                  float* __restrict__ gradE) {
  __shared__ GradSmem sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int col = 16 * wave + c;  // sample column within the chunk
  float* slot = partial + (int64_t)blockIdx.x * kLayers * kLayerParams;
  for (int i = tid; i < kLayers * kLayerParams; i += 256) slot[i] = 0.0f;
  for (int i = tid; i < 16 * kPitch; i += 256) (&sm.d3[0][0])[i] = 0;
  double loss_acc = 0.0;
  const double inv_B = 1.0 / (double)B;
  const int64_t n_chunks = (B + kChunk - 1) / kChunk;
  for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
    const int64_t idx = ch * kChunk + col;
    int b = idx < B ? band[idx] : 0;
    bool valid = idx < B && b >= 0 && b < fa.n_emb;
    if (!valid) b = 0;
    double lo[8], hi[8];
    box_of(fa, b, lo, hi);
    double x[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const double v = valid ? u[idx * 8 + i] : lo[i];
      const double p = (v - lo[i]) / (hi[i] - lo[i]);
      if (!(p > 0.0 && p < 1.0)) valid = false;
      x[i] = log(p) - log1p(-p);
    }
    if (!valid)
      for (int i = 0; i < 8; i++) x[i] = 0.0;
    const double wgt = valid ? inv_B : 0.0;
    float emb[16];
    const float* E = fa.params + (int64_t)kLayers * kLayerParams + (int64_t)b * kEmb;
#pragma unroll
    for (int i = 0; i < 16; i++) emb[i] = E[i];
    if (tid == 0) sm.loss = 0.0;
    // forward, storing every layer's input
    double logdet = 0.0;
    for (int l = 0; l < kLayers; l++) {
      if (g == 0)
        for (int i = 0; i < 8; i++) sm.xs[l][col][i] = x[i];
      const int par = l & 1;
      double xc[4];
      kept_of(x, par, xc);
      CondOut co;
      conditioner(fa.params + (int64_t)l * kLayerParams, fa.packed + (int64_t)l * kFragPerLayer * 64, lane,
                  h0_operand(g, xc, emb), co);
      float tt[4];
#pragma unroll
      for (int j = 0; j < 4; j++) tt[j] = __shfl(co.o[j], c + 16, 64);
      if (g == 0) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const double s = (double)(2.0f * tanhf(co.o[j]));
          const double es = exp(s);
          if (par)
            x[2 * j] = x[2 * j] * es + (double)tt[j];
          else
            x[2 * j + 1] = x[2 * j + 1] * es + (double)tt[j];
          logdet += s;
        }
      }
    }
    __syncthreads();
    if (g == 0) {
      double s2 = 0.0;
      for (int i = 0; i < 8; i++) {
        sm.xs[kLayers][col][i] = x[i];
        s2 += x[i] * x[i];
      }
      if (valid) atomicAdd(&sm.loss, -(-0.5 * s2 - 8.0 * 0.91893853320467274178032973640562 + logdet) * wgt);
    }
    // gradient w.r.t. the current layer output (held by the g = 0 lanes)
    float gy[8];
#pragma unroll
    for (int i = 0; i < 8; i++) gy[i] = (float)(x[i] * wgt);
    for (int l = kLayers - 1; l >= 0; l--) {
      const int par = l & 1;
      const float* W = fa.params + (int64_t)l * kLayerParams;
      const u32x4_t* pk = fa.packed + (int64_t)l * kFragPerLayer * 64;
      float* gl = slot + (int64_t)l * kLayerParams;
      double xin[8];
#pragma unroll
      for (int i = 0; i < 8; i++) xin[i] = sm.xs[l][col][i];
      double xc[4];
      kept_of(xin, par, xc);
      const u32x4_t h0 = h0_operand(g, xc, emb);
      CondOut co;
      conditioner(W, pk, lane, h0, co);
      // activations into the [feature][sample] tiles
      {
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
          const int f = 8 * g + i;
          v[i] = f < 4 ? (float)xc[f] : (f < kCin ? emb[f - 4] : 0.0f);
          lds_put(sm.h0[f], col, v[i]);
        }
      }
#pragma unroll
      for (int mt = 0; mt < 8; mt++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          lds_put(sm.h1[16 * mt + 4 * g + j], col, silu(co.a1[mt][j]));
          lds_put(sm.h2[16 * mt + 4 * g + j], col, silu(co.a2[mt][j]));
        }
      // output gradient: (d s_hat, d t) on the g = 0 lanes
      float go[8];
#pragma unroll
      for (int i = 0; i < 8; i++) go[i] = 0.0f;
      if (g == 0) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const float th = tanhf(co.o[j]);
          const float s = 2.0f * th;
          const float es = __expf(s);
          const int d = par ? 2 * j : 2 * j + 1;
          const float gyd = gy[d];
          const float gs = gyd * (float)xin[d] * es - (float)wgt;
          go[j] = gs * 2.0f * (1.0f - th * th);
          go[4 + j] = gyd;
          gy[d] = gyd * es;
        }
#pragma unroll
        for (int i = 0; i < 8; i++) lds_put(sm.d3[i], col, go[i]);
      }
      // d h2 = W3^T go; d a2 = d h2 * silu'(a2)
      const u32x4_t gob = pack8(go);
      u32x4_t db[4];
      {
        f32x4_t da[8];
#pragma unroll
        for (int mt = 0; mt < 8; mt++) {
          da[mt] = mfma(pk[(fW3t + mt) * 64 + lane], gob, f32x4_t{0.f, 0.f, 0.f, 0.f});
#pragma unroll
          for (int j = 0; j < 4; j++) {
            da[mt][j] *= silu_grad(co.a2[mt][j]);
            lds_put(sm.d2[16 * mt + 4 * g + j], col, da[mt][j]);
          }
        }
#pragma unroll
        for (int kb = 0; kb < 4; kb++) db[kb] = pack_tiles(da[2 * kb], da[2 * kb + 1]);
      }
      // d h1 = W2^T d a2; d a1 = d h1 * silu'(a1)
      {
        f32x4_t da[8];
#pragma unroll
        for (int mt = 0; mt < 8; mt++) {
          f32x4_t acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kb = 0; kb < 4; kb++) acc = mfma(pk[(fW2t + 4 * mt + kb) * 64 + lane], db[kb], acc);
#pragma unroll
          for (int j = 0; j < 4; j++) {
            acc[j] *= silu_grad(co.a1[mt][j]);
            lds_put(sm.d1[16 * mt + 4 * g + j], col, acc[j]);
          }
          da[mt] = acc;
        }
#pragma unroll
        for (int kb = 0; kb < 4; kb++) db[kb] = pack_tiles(da[2 * kb], da[2 * kb + 1]);
      }
      // d h0 = W1^T d a1: kept coordinates and the embedding
#pragma unroll
      for (int mt = 0; mt < 2; mt++) {
        f32x4_t acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; kb++) acc = mfma(pk[(fW1t + 4 * mt + kb) * 64 + lane], db[kb], acc);
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int f = 16 * mt + 4 * g + j;
          if (f < 4) {
            const int d = par ? 2 * j + 1 : 2 * j;
            gy[d] += acc[j];
          } else if (f < kCin && valid) {
            atomicAdd(&gradE[(int64_t)b * kEmb + f - 4], acc[j]);
          }
        }
      }
      __syncthreads();
      // weight gradients over the chunk: 8 (W3) + 64 (W2) + 16 (W1) tiles of 16 x 16
      for (int tl = wave; tl < 88; tl += 4) {
        const uint16_t(*A)[kPitch];
        const uint16_t(*Bt)[kPitch];
        int mt, nt, in_dim, out_lim, off;
        if (tl < 8) {
          A = sm.d3, Bt = sm.h2, mt = 0, nt = tl, in_dim = kH, out_lim = kOut, off = oW3;
        } else if (tl < 72) {
          A = sm.d2, Bt = sm.h1, mt = (tl - 8) >> 3, nt = (tl - 8) & 7, in_dim = kH, out_lim = kH, off = oW2;
        } else {
          A = sm.d1, Bt = sm.h0, mt = (tl - 72) >> 1, nt = (tl - 72) & 1, in_dim = kCin, out_lim = kH, off = oW1;
        }
        f32x4_t acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; kb++)
          acc = mfma(lds_frag(A, 16 * mt + c, kb, g), lds_frag(Bt, 16 * nt + c, kb, g), acc);
        const int in = 16 * nt + c;
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int out = 16 * mt + 4 * g + j;
          if (out < out_lim && in < in_dim) gl[off + out * in_dim + in] += acc[j];
        }
      }
      // bias gradients (sum of the tiles' rows over the chunk)
      if (tid < kH) {
        float s1 = 0.f, s2 = 0.f;
        for (int s = 0; s < kChunk; s++) {
          s1 += bf16_value(sm.d1[tid][s]);
          s2 += bf16_value(sm.d2[tid][s]);
        }
        gl[oB1 + tid] += s1;
        gl[oB2 + tid] += s2;
      } else if (tid < kH + kOut) {
        float s3 = 0.f;
        for (int s = 0; s < kChunk; s++) s3 += bf16_value(sm.d3[tid - kH][s]);
        gl[oB3 + tid - kH] += s3;
      }
      __syncthreads();
    }
    if (tid == 0) loss_acc += sm.loss;
    __syncthreads();
  }
  if (tid == 0) loss_part[blockIdx.x] = loss_acc;
}

// grad[p] = sum over slots (fixed order); loss = sum of the slot losses
__global__ void k_flow_reduce(const float* __restrict__ partial, int n_slots, const double* __restrict__ loss_part,
                              float* __restrict__ grad, double* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kLayers * kLayerParams) {
    float s = 0.0f;
    for (int k = 0; k < n_slots; k++) s += partial[(int64_t)k * kLayers * kLayerParams + p];
    grad[p] = s;
  }
  if (p == 0) {
    double t = 0.0;
    for (int k = 0; k < n_slots; k++) t += loss_part[k];
    *loss = t;
  }
}

__global__ void k_flow_fill(float* __restrict__ a, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Adam with bias correction (step counts from 1)
__global__ void k_flow_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ grad, int64_t n, double bc1, double bc2, float lr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = (float)(mi / bc1);
  const float vh = (float)(vi / bc2);
  P[i] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

}  // namespace flow
}  // namespace gbl
