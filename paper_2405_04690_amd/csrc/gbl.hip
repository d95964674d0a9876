// gbl.hip -- host side of the C ABI declared in include/gbl.h.
//
// Argument checking, context set-up (tables, PSD basis, workspace) and kernel
// launches.  Every compute entry point only enqueues on the context stream.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/gbl.h"
#include "gbl_kernels.hpp"
#include "gbl_sampler.hpp"
#include "gbl_flow.hpp"
#include "gbl_search.hpp"
#include "gbl_matrix.hpp"

using gbl::cd;

// Static scratch of the allocation-free PSD likelihood: the per-chunk
// partial sums of up to 2048 parameter sets (8 MB).  Each device holds its
// own copy; host code uses the address hipGetSymbolAddress returns for the
// current device (kept per device below), never the symbol's name.
static __device__ __align__(256) double scratch[2 * gbl::kPsdChunks * 2048];

namespace {

constexpr int kNumWidths = gbl::kBucketWidths;
constexpr int kWidths[kNumWidths] = {128, 256, 512, 1024};
constexpr int64_t kMaxGrid = (int64_t)1 << 30;  // blocks per launch (grid.x limit is 2^31 - 1)
constexpr int64_t kDecodeChunk = (int64_t)1 << 17; // pairs per decode pass (workspace 2^18 decoded sources, 111 MB)
constexpr int64_t kPsdBatch = 4096;             // parameter sets per PSD-likelihood launch pair
constexpr int kBucketCap = 1 << 20;             // templates per bucketed (uneven-width) launch group
constexpr int64_t kDetCap = (int64_t)1 << 22;    // deterministic scatter: slice elements per channel and chunk
                                                 // (128 MB of slices; 2^22 / N templates per chunk)
constexpr int64_t kDetMaxChunk = kDetCap / 128;

constexpr int64_t kScratchSets = 2048;  // parameter sets the static scratch holds
constexpr int kMaxDevices = 64;
double* scratch_ptr[kMaxDevices] = {};
std::mutex scratch_mu;

// the scratch address on the current device (looked up once per device)
int scratch_for_current_device(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GBL_EHIP;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GBL_EHIP;
    scratch_ptr[dev] = (double*)p;
  }
  *out = scratch_ptr[dev];
  return GBL_OK;
}

int width_slot(int N) {
  for (int i = 0; i < kNumWidths; i++)
    if (kWidths[i] == N) return i;
  return -1;
}

}  // namespace

struct gbl_ctx {
  gbl_config cfg;
  hipStream_t stream;
  gbl::Geo geo;
  void* table_mem[kNumWidths];
  gbl::WaveTables<double> tables[kNumWidths];   // FP64 response
  gbl::WaveTables<float> tables32[kNumWidths];  // mixed precision response
  double* psd_P1;
  double* psd_P2;
  double* psd_P3;    // foreground factors (Sec. 3): 3 x^2 sin^2 x f^(-7/3)
  double* psd_LF;    // ln f
  double* psd_work;
  double* scratch;   // this device's static scratch (allocation-free PSD likelihood)
  int* counts;       // [4 widths] templates per width bucket
  int32_t* perm;     // [4 widths][kBucketCap] template indices per width
  gbl_tuning tune;        // launch-shape knobs
  int* route_counts;      // [4 widths] mixed-precision pairs queued for the FP64 pass
  int32_t* route_lists;   // [4 widths][kBucketCap]
  int* host_counts;       // pinned [8]: device-side counts read back for exact grids
  gbl::Src* src_ws;       // [2 kDecodeChunk] decoded sources of one chunk of pairs
  // deterministic scatter (GBL_DETERMINISTIC only)
  cd* det_ws;             // [2][kDetCap] A, E slices of one chunk of templates
  int64_t* det_start;     // [kDetMaxChunk]
  uint64_t* det_keys;     // [2][kDetMaxChunk] sort keys in / out
  int32_t* det_vals;      // [2][kDetMaxChunk] template slots in / out
  void* det_sort_tmp;
  size_t det_sort_bytes;
  std::string err;
};

// Device-side list lengths (width buckets, routed pairs) copied to the host
// when the caller opted in (exact_grids) and the stream is not being captured,
// at the price of one stream synchronisation, so that the launches that walk
// the lists get exact grids.  Otherwise the grids stay at their upper bound
// and the surplus blocks exit at once; for the wide templates, whose blocks
// hold 64 KB of LDS, those empty blocks cost as much as a third of the launch.
static bool host_counts(gbl_ctx* ctx, const int* dev, int n, int* out) {
  if (!ctx->tune.exact_grids) return false;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &st) != hipSuccess || st != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return false;
  }
  if (hipMemcpyAsync(ctx->host_counts, dev, sizeof(int) * n, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  for (int i = 0; i < n; i++) out[i] = ctx->host_counts[i];
  return true;
}

static int fail(gbl_ctx* ctx, int code, const char* fmt, const char* detail = "") {
  if (ctx) {
    char buf[512];
    snprintf(buf, sizeof(buf), fmt, detail);
    ctx->err = buf;
  }
  return code;
}

static int check_launch(gbl_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return GBL_EHIP;
  }
  return GBL_OK;
}

static void release(gbl_ctx* ctx) {
  for (int i = 0; i < kNumWidths; i++)
    if (ctx->table_mem[i]) (void)hipFree(ctx->table_mem[i]);
  if (ctx->psd_P1) (void)hipFree(ctx->psd_P1);
  if (ctx->psd_P2) (void)hipFree(ctx->psd_P2);
  if (ctx->psd_P3) (void)hipFree(ctx->psd_P3);
  if (ctx->psd_LF) (void)hipFree(ctx->psd_LF);
  if (ctx->psd_work) (void)hipFree(ctx->psd_work);
  if (ctx->counts) (void)hipFree(ctx->counts);
  if (ctx->perm) (void)hipFree(ctx->perm);
  if (ctx->route_counts) (void)hipFree(ctx->route_counts);
  if (ctx->route_lists) (void)hipFree(ctx->route_lists);
  if (ctx->host_counts) (void)hipHostFree(ctx->host_counts);
  if (ctx->src_ws) (void)hipFree(ctx->src_ws);
  if (ctx->det_ws) (void)hipFree(ctx->det_ws);
  if (ctx->det_start) (void)hipFree(ctx->det_start);
  if (ctx->det_keys) (void)hipFree(ctx->det_keys);
  if (ctx->det_vals) (void)hipFree(ctx->det_vals);
  if (ctx->det_sort_tmp) (void)hipFree(ctx->det_sort_tmp);
}

extern "C" int gbl_create(gbl_ctx** out, const gbl_config* cfg, void* hip_stream) {
  if (!out) return GBL_EINVAL;
  *out = nullptr;
  if (!cfg) return GBL_EINVAL;
  if (!(cfg->T > 0) || !(cfg->dt > 0) || !(cfg->L > 0) || !(cfg->f_lo > 0) || !(cfg->f_hi > cfg->f_lo) ||
      cfg->f_hi > 0.5 / cfg->dt || (cfg->flags & ~(GBL_MIXED_UNROUTED | GBL_DETERMINISTIC)) != 0 ||
      ((cfg->flags & GBL_MIXED_UNROUTED) && cfg->precision != GBL_MIXED))
    return GBL_EINVAL;
  if (cfg->precision != GBL_FP64 && cfg->precision != GBL_MIXED) return GBL_EUNSUPPORTED;

  gbl_ctx* ctx = new gbl_ctx();
  ctx->tune = gbl_tuning{4096, kBucketCap, 1, 0};
  ctx->cfg = *cfg;
  ctx->stream = (hipStream_t)hip_stream;
  int64_t k_min = (int64_t)std::ceil(cfg->f_lo * cfg->T);
  int64_t k_max = (int64_t)std::floor(cfg->f_hi * cfg->T);
  if (k_max < k_min) {
    delete ctx;
    return GBL_EINVAL;
  }
  gbl::Geo& g = ctx->geo;
  g.T = cfg->T;
  g.L = cfg->L;
  g.Lc = cfg->L / gbl::kC;
  g.inv_L = 1.0 / cfg->L;
  double e = cfg->L / (2.0 * std::sqrt(3.0) * gbl::kAU);
  g.eh = 0.5 * e * gbl::kAU;
  g.ez = std::sqrt(3.0) * e * gbl::kAU;
  g.df4 = 4.0 / cfg->T;
  g.k_min = k_min;
  g.n_bins = k_max - k_min + 1;

  for (int i = 0; i < kNumWidths; i++) {
    int N = kWidths[i];
    size_t bytes = sizeof(double) * 4 * N + sizeof(cd) * 3 * N + sizeof(gbl::cf) * 3 * N;
    if (hipMalloc(&ctx->table_mem[i], bytes) != hipSuccess) {
      release(ctx);
      delete ctx;
      return GBL_EHIP;
    }
    double* basis = (double*)ctx->table_mem[i];
    cd* tw = (cd*)(basis + 4 * N);
    cd* bF = tw + N;
    cd* bW = bF + N;
    gbl::cf* tw32 = (gbl::cf*)(bW + N);
    gbl::cf* bF32 = tw32 + N;
    gbl::cf* bW32 = bF32 + N;
    ctx->tables[i] = {basis, tw, bF, bW};
    ctx->tables32[i] = {basis, tw32, bF32, bW32};
    hipLaunchKernelGGL(gbl::k_init_wave_tables, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, N, g.T, g.Lc,
                       basis, tw, bF, bW, tw32, bF32, bW32);
  }
  size_t nbb = sizeof(double) * (size_t)g.n_bins;
  if (hipMalloc(&ctx->psd_P1, nbb) != hipSuccess || hipMalloc(&ctx->psd_P2, nbb) != hipSuccess ||
      hipMalloc(&ctx->psd_P3, nbb) != hipSuccess || hipMalloc(&ctx->psd_LF, nbb) != hipSuccess ||
      hipMalloc(&ctx->psd_work, sizeof(double) * 2 * gbl::kPsdChunks * kPsdBatch) != hipSuccess ||
      hipMalloc(&ctx->counts, sizeof(int) * kNumWidths) != hipSuccess ||
      hipMalloc(&ctx->perm, sizeof(int32_t) * (size_t)kNumWidths * kBucketCap) != hipSuccess ||
      hipMalloc(&ctx->route_counts, sizeof(int) * kNumWidths) != hipSuccess ||
      hipMalloc(&ctx->route_lists, sizeof(int32_t) * (size_t)kNumWidths * kBucketCap) != hipSuccess ||
      hipHostMalloc((void**)&ctx->host_counts, sizeof(int) * 8, hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&ctx->src_ws, sizeof(gbl::Src) * 2 * kDecodeChunk) != hipSuccess) {
    release(ctx);
    delete ctx;
    return GBL_EHIP;
  }
  if (cfg->flags & GBL_DETERMINISTIC) {
    size_t tmp = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)kDetMaxChunk, 0, 64,
                                           ctx->stream) != hipSuccess ||
        hipMalloc(&ctx->det_ws, sizeof(cd) * 2 * kDetCap) != hipSuccess ||
        hipMalloc(&ctx->det_start, sizeof(int64_t) * kDetMaxChunk) != hipSuccess ||
        hipMalloc(&ctx->det_keys, sizeof(uint64_t) * 2 * kDetMaxChunk) != hipSuccess ||
        hipMalloc(&ctx->det_vals, sizeof(int32_t) * 2 * kDetMaxChunk) != hipSuccess ||
        hipMalloc(&ctx->det_sort_tmp, tmp > 0 ? tmp : 1) != hipSuccess) {
      release(ctx);
      delete ctx;
      return GBL_EHIP;
    }
    ctx->det_sort_bytes = tmp;
  }
  if (scratch_for_current_device(&ctx->scratch) != GBL_OK) {
    (void)hipGetLastError();
    release(ctx);
    delete ctx;
    return GBL_EHIP;
  }
  hipLaunchKernelGGL(gbl::k_init_psd_basis, dim3((unsigned)((g.n_bins + 255) / 256)), dim3(256), 0, ctx->stream,
                     g.k_min, g.n_bins, g.T, g.L, ctx->psd_P1, ctx->psd_P2, ctx->psd_P3, ctx->psd_LF);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    release(ctx);
    delete ctx;
    return GBL_EHIP;
  }
  *out = ctx;
  return GBL_OK;
}

extern "C" int gbl_destroy(gbl_ctx* ctx) {
  if (!ctx) return GBL_OK;
  (void)hipStreamSynchronize(ctx->stream);
  release(ctx);
  delete ctx;
  return GBL_OK;
}

extern "C" int gbl_set_stream(gbl_ctx* ctx, void* hip_stream) {
  if (!ctx) return GBL_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return GBL_OK;
}

extern "C" const char* gbl_last_error(const gbl_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" int gbl_band(const gbl_ctx* ctx, int64_t* k_min, int64_t* n_bins) {
  if (!ctx || !k_min || !n_bins) return GBL_EINVAL;
  *k_min = ctx->geo.k_min;
  *n_bins = ctx->geo.n_bins;
  return GBL_OK;
}

// ---------------------------------------------------------------------------
// dispatch helpers over the supported widths
// ---------------------------------------------------------------------------
template <template <int> class F, typename... Args>
static void dispatch_width(int N, Args&&... args) {
  switch (N) {
    case 128: F<128>::run(args...); break;
    case 256: F<256>::run(args...); break;
    case 512: F<512>::run(args...); break;
    case 1024: F<1024>::run(args...); break;
    default: break;
  }
}

// precision dispatch: FP64 response or the mixed-precision response
template <int N, typename F>
static const gbl::WaveTables<F>& tables_for(gbl_ctx* ctx);
template <>
const gbl::WaveTables<double>& tables_for<128, double>(gbl_ctx* ctx) { return ctx->tables[0]; }
template <>
const gbl::WaveTables<double>& tables_for<256, double>(gbl_ctx* ctx) { return ctx->tables[1]; }
template <>
const gbl::WaveTables<double>& tables_for<512, double>(gbl_ctx* ctx) { return ctx->tables[2]; }
template <>
const gbl::WaveTables<double>& tables_for<1024, double>(gbl_ctx* ctx) { return ctx->tables[3]; }
template <>
const gbl::WaveTables<float>& tables_for<128, float>(gbl_ctx* ctx) { return ctx->tables32[0]; }
template <>
const gbl::WaveTables<float>& tables_for<256, float>(gbl_ctx* ctx) { return ctx->tables32[1]; }
template <>
const gbl::WaveTables<float>& tables_for<512, float>(gbl_ctx* ctx) { return ctx->tables32[2]; }
template <>
const gbl::WaveTables<float>& tables_for<1024, float>(gbl_ctx* ctx) { return ctx->tables32[3]; }

template <int N, typename F>
static void launch_waveform(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, cd* A, cd* E, cd* Tc,
                            int64_t* sb) {
  const auto& tb = tables_for<N, F>(ctx);
  if (Tc)
    hipLaunchKernelGGL((gbl::k_waveform<N, 6, F>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0,
                       ctx->stream, ctx->geo, tb, params, b0, A, E, Tc, sb);
  else
    hipLaunchKernelGGL((gbl::k_waveform<N, 4, F>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0,
                       ctx->stream, ctx->geo, tb, params, b0, A, E, Tc, sb);
}

template <int N>
struct LaunchWaveform {
  static void run(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, cd* A, cd* E, cd* Tc, int64_t* sb) {
    if (ctx->cfg.precision == GBL_MIXED)
      launch_waveform<N, float>(ctx, params, b0, nb, A, E, Tc, sb);
    else
      launch_waveform<N, double>(ctx, params, b0, nb, A, E, Tc, sb);
  }
};

static bool routed(const gbl_ctx* ctx) {
  return ctx->cfg.precision == GBL_MIXED && !(ctx->cfg.flags & GBL_MIXED_UNROUTED);
}

// mixed precision: pairs whose FP32 error estimate exceeds this are re-evaluated in FP64
constexpr double kRouteTol = 5e-4;

static gbl::DeltaArgs with_route(gbl_ctx* ctx, gbl::DeltaArgs da, int N, int64_t b0) {
  const int slot = width_slot(N);
  da.route_list = ctx->route_lists + (int64_t)slot * kBucketCap;
  da.route_count = ctx->route_counts + slot;
  da.route_tol = kRouteTol;
  da.route_b0 = b0;
  return da;
}

// FP64 re-evaluation of the routed pairs of width N; grid = the routed count
// when known on the host, else its upper bound nb
template <int N>
static void launch_route_pass(gbl_ctx* ctx, const gbl::DeltaArgs& da, int64_t b0, int64_t grid) {
  if (grid <= 0) return;
  const int slot = width_slot(N);
  hipLaunchKernelGGL((gbl::k_delta_loglike_list<N>), dim3((unsigned)grid), dim3(gbl::delta_threads<N>()), 0,
                     ctx->stream, ctx->geo, tables_for<N, double>(ctx), da, b0,
                     (const int*)(ctx->route_counts + slot),
                     (const int32_t*)(ctx->route_lists + (int64_t)slot * kBucketCap));
}

template <int N>
struct LaunchRoutePass {
  static void run(gbl_ctx* ctx, const gbl::DeltaArgs& da, int64_t b0, int64_t nb) {
    int rc[kNumWidths];
    const int slot = width_slot(N);
    launch_route_pass<N>(ctx, da, b0, host_counts(ctx, ctx->route_counts, kNumWidths, rc) ? rc[slot] : nb);
  }
};

template <int N>
struct LaunchDelta {
  static void run(gbl_ctx* ctx, const gbl::DeltaArgs& da, int64_t b0, int64_t nb) {
    if (routed(ctx)) {
      hipLaunchKernelGGL(gbl::k_bucket_reset, dim3(1), dim3(64), 0, ctx->stream, ctx->route_counts, kNumWidths);
      hipLaunchKernelGGL((gbl::k_delta_loglike<N, float>), dim3((unsigned)nb), dim3(gbl::delta_threads<N>()), 0,
                         ctx->stream, ctx->geo, tables_for<N, float>(ctx), with_route(ctx, da, N, b0), b0);
      LaunchRoutePass<N>::run(ctx, da, b0, nb);
    } else if (ctx->cfg.precision == GBL_MIXED)
      hipLaunchKernelGGL((gbl::k_delta_loglike<N, float>), dim3((unsigned)nb), dim3(gbl::delta_threads<N>()), 0,
                         ctx->stream, ctx->geo, tables_for<N, float>(ctx), da, b0);
    else
      hipLaunchKernelGGL((gbl::k_delta_loglike<N, double>), dim3((unsigned)nb), dim3(gbl::delta_threads<N>()), 0,
                         ctx->stream, ctx->geo, tables_for<N, double>(ctx), da, b0);
  }
};

// one width's bucket; grid = the bucket's size when known on the host, else
// its upper bound (the routed pairs are re-evaluated after all widths)
template <int N>
struct LaunchDeltaBucket {
  static void run(gbl_ctx* ctx, const gbl::DeltaArgs& da, int64_t b0, int64_t grid) {
    if (grid <= 0) return;
    const int slot = width_slot(N);
    const int* cnt = ctx->counts + slot;
    const int32_t* perm = ctx->perm + (int64_t)slot * kBucketCap;
    if (routed(ctx))
      hipLaunchKernelGGL((gbl::k_delta_loglike_bucket<N, float>), dim3((unsigned)grid),
                         dim3(gbl::delta_threads<N>()), 0, ctx->stream, ctx->geo, tables_for<N, float>(ctx),
                         with_route(ctx, da, N, b0), b0, cnt, perm);
    else if (ctx->cfg.precision == GBL_MIXED)
      hipLaunchKernelGGL((gbl::k_delta_loglike_bucket<N, float>), dim3((unsigned)grid),
                         dim3(gbl::delta_threads<N>()), 0, ctx->stream, ctx->geo, tables_for<N, float>(ctx), da, b0,
                         cnt, perm);
    else
      hipLaunchKernelGGL((gbl::k_delta_loglike_bucket<N, double>), dim3((unsigned)grid),
                         dim3(gbl::delta_threads<N>()), 0, ctx->stream, ctx->geo, tables_for<N, double>(ctx), da,
                         b0, cnt, perm);
  }
};

template <int N, typename F>
static void launch_waveform_bucket(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, const int64_t* off,
                                   cd* A, cd* E, cd* Tc, int64_t* sb) {
  if (nb <= 0) return;
  const int slot = width_slot(N);
  const int* cnt = ctx->counts + slot;
  const int32_t* perm = ctx->perm + (int64_t)slot * kBucketCap;
  const auto& tb = tables_for<N, F>(ctx);
  if (Tc)
    hipLaunchKernelGGL((gbl::k_waveform_bucket<N, 6, F>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0,
                       ctx->stream, ctx->geo, tb, params, b0, off, A, E, Tc, sb, cnt, perm);
  else
    hipLaunchKernelGGL((gbl::k_waveform_bucket<N, 4, F>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0,
                       ctx->stream, ctx->geo, tb, params, b0, off, A, E, Tc, sb, cnt, perm);
}

template <int N>
struct LaunchWaveformBucket {
  static void run(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, const int64_t* off, cd* A, cd* E,
                  cd* Tc, int64_t* sb) {
    if (ctx->cfg.precision == GBL_MIXED)
      launch_waveform_bucket<N, float>(ctx, params, b0, nb, off, A, E, Tc, sb);
    else
      launch_waveform_bucket<N, double>(ctx, params, b0, nb, off, A, E, Tc, sb);
  }
};

template <int N>
struct LaunchScatter {
  static void run(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, double sign, cd* residual, int n_res,
                  const int32_t* ri) {
    if (ctx->cfg.precision == GBL_MIXED)
      hipLaunchKernelGGL((gbl::k_scatter_add<N, float>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0,
                         ctx->stream, ctx->geo, tables_for<N, float>(ctx), params, b0, sign, residual, n_res, ri);
    else
      hipLaunchKernelGGL((gbl::k_scatter_add<N, double>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0,
                         ctx->stream, ctx->geo, tables_for<N, double>(ctx), params, b0, sign, residual, n_res, ri);
  }
};

// deterministic scatter: chunks of kDetCap / N templates, each built into the
// workspace, sorted by (residual, start bin) and gathered bin by bin
template <int N, typename F>
static int det_scatter(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, double sign, cd* residual,
                       int n_res, const int32_t* ri) {
  const int64_t chunk = kDetCap / N;
  uint64_t* keys_in = ctx->det_keys;
  uint64_t* keys_out = ctx->det_keys + kDetMaxChunk;
  int32_t* vals_in = ctx->det_vals;
  int32_t* vals_out = ctx->det_vals + kDetMaxChunk;
  for (int64_t c0 = 0; c0 < nb; c0 += chunk) {
    const int64_t n = nb - c0 < chunk ? nb - c0 : chunk;
    hipLaunchKernelGGL(gbl::k_det_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, ctx->geo,
                       params, b0 + c0, n, N, ri, n_res, keys_in, vals_in);
    hipLaunchKernelGGL((gbl::k_det_slices<N, F>), dim3((unsigned)n), dim3(gbl::block_threads<N>()), 0, ctx->stream,
                       ctx->geo, tables_for<N, F>(ctx), params, b0 + c0, ctx->det_ws, kDetCap, ctx->det_start);
    size_t bytes = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)keys_in, keys_out,
                                           (const int32_t*)vals_in, vals_out, (int)n, 0, 64, ctx->stream) !=
            hipSuccess ||
        bytes > ctx->det_sort_bytes)
      return fail(ctx, GBL_EHIP, "gb_scatter_add: sort workspace too small%s");
    bytes = ctx->det_sort_bytes;
    if (hipcub::DeviceRadixSort::SortPairs(ctx->det_sort_tmp, bytes, (const uint64_t*)keys_in, keys_out,
                                           (const int32_t*)vals_in, vals_out, (int)n, 0, 64, ctx->stream) !=
        hipSuccess)
      return fail(ctx, GBL_EHIP, "gb_scatter_add: sort failed%s");
    hipLaunchKernelGGL((gbl::k_det_gather<N>), dim3((unsigned)n), dim3(gbl::block_threads<N>()), 0, ctx->stream,
                       ctx->geo, (const uint64_t*)keys_out, (const int32_t*)vals_out, n, (const cd*)ctx->det_ws,
                       kDetCap, sign, residual);
  }
  return GBL_OK;
}

template <int N>
struct LaunchDetScatter {
  static void run(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, double sign, cd* residual, int n_res,
                  const int32_t* ri, int* rc) {
    if (ctx->cfg.precision == GBL_MIXED)
      *rc = det_scatter<N, float>(ctx, params, b0, nb, sign, residual, n_res, ri);
    else
      *rc = det_scatter<N, double>(ctx, params, b0, nb, sign, residual, n_res, ri);
  }
};

template <int N>
struct LaunchSnr {
  static void run(gbl_ctx* ctx, const double* params, int64_t b0, int64_t nb, const double* psd, int n_psd,
                  int psd_inv, const int32_t* psd_idx, const cd* data, int n_data, const int32_t* data_idx,
                  double* snr_opt, double* snr_obs) {
    hipLaunchKernelGGL((gbl::k_snr<N>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0, ctx->stream, ctx->geo,
                       tables_for<N, double>(ctx), params, b0, psd, n_psd, psd_inv, psd_idx, data, n_data, data_idx,
                       snr_opt, snr_obs);
  }
};

template <int N>
struct LaunchOverlap {
  static void run(gbl_ctx* ctx, const double* pa, const double* pb, int64_t b0, int64_t nb, const double* psd,
                  int n_psd, int psd_inv, const int32_t* psd_idx, double* out) {
    hipLaunchKernelGGL((gbl::k_overlap<N>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0, ctx->stream,
                       ctx->geo, tables_for<N, double>(ctx), pa, pb, b0, psd, n_psd, psd_inv, psd_idx, out);
  }
};

// device-side bucketing of templates [b0, b0 + nb) by width
static void bucket_widths(gbl_ctx* ctx, const int32_t* widths, int64_t b0, int64_t nb, double* bad_out,
                          int64_t* bad_start) {
  hipLaunchKernelGGL(gbl::k_bucket_reset, dim3(1), dim3(64), 0, ctx->stream, ctx->counts, kNumWidths);
  hipLaunchKernelGGL(gbl::k_bucket_by_width, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, ctx->stream, widths,
                     b0, nb, kBucketCap, ctx->counts, ctx->perm, bad_out, bad_start);
}

// ---------------------------------------------------------------------------
// compute entry points
// ---------------------------------------------------------------------------
extern "C" int gb_waveform(gbl_ctx* ctx, const double* params, int64_t B, int32_t N, double T, double dt, double* A,
                           double* E, double* Tch, int64_t* start_bin) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0) return fail(ctx, GBL_EINVAL, "gb_waveform: B < 0%s");
  if (width_slot(N) < 0) return fail(ctx, GBL_EUNSUPPORTED, "gb_waveform: unsupported N%s");
  if (T != ctx->cfg.T || dt != ctx->cfg.dt) return fail(ctx, GBL_EINVAL, "gb_waveform: T/dt differ from the context%s");
  if (B == 0) return GBL_OK;
  if (!params || !A || !E || !start_bin) return fail(ctx, GBL_EINVAL, "gb_waveform: null pointer%s");
  for (int64_t b0 = 0; b0 < B; b0 += kMaxGrid) {
    int64_t nb = B - b0 < kMaxGrid ? B - b0 : kMaxGrid;
    dispatch_width<LaunchWaveform>(N, ctx, params, b0, nb, (cd*)A, (cd*)E, (cd*)Tch, start_bin);
  }
  return check_launch(ctx, "gb_waveform");
}

// decode pass of pairs [b0, b0 + nb) (nb <= kDecodeChunk) into the context's
// workspace; returns the arguments that point the fused kernels at it
static gbl::DeltaArgs decode_pairs(gbl_ctx* ctx, gbl::DeltaArgs da, int64_t b0, int64_t nb) {
  hipLaunchKernelGGL(gbl::k_decode_pairs, dim3((unsigned)((2 * nb + gbl::kDecodeBlock - 1) / gbl::kDecodeBlock)),
                     dim3(gbl::kDecodeBlock), 0, ctx->stream, ctx->geo, da.p_old, da.p_new, b0, nb, ctx->src_ws);
  da.srcs = ctx->src_ws;
  da.src_b0 = b0;
  return da;
}

extern "C" int gb_delta_loglike(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* psd,
                                int32_t n_psd, int32_t psd_flags, const double* params_old, const double* params_new,
                                int32_t N, const int32_t* res_idx, const int32_t* psd_idx, int64_t B, double* dlogl) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0 || n_res < 1 || n_psd < 1) return fail(ctx, GBL_EINVAL, "gb_delta_loglike: bad sizes%s");
  if (psd_flags & ~GBL_PSD_INVERSE) return fail(ctx, GBL_EINVAL, "gb_delta_loglike: unknown psd flag%s");
  if (width_slot(N) < 0) return fail(ctx, GBL_EUNSUPPORTED, "gb_delta_loglike: unsupported N%s");
  if (B == 0) return GBL_OK;
  if (!residual || !psd || !params_old || !params_new || !res_idx || !psd_idx || !dlogl)
    return fail(ctx, GBL_EINVAL, "gb_delta_loglike: null pointer%s");
  const gbl::DeltaArgs da = {(const cd*)residual, (int)n_res, psd, (int)n_psd,
                             (psd_flags & GBL_PSD_INVERSE) ? 1 : 0, params_old, params_new, res_idx, psd_idx, dlogl,
                             nullptr, nullptr, 0.0, 0, nullptr, 0};
  const int64_t chunk = std::min<int64_t>(routed(ctx) ? (int64_t)ctx->tune.bucket_chunk : kMaxGrid, kDecodeChunk);
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    int64_t nb = B - b0 < chunk ? B - b0 : chunk;
    dispatch_width<LaunchDelta>(N, ctx, decode_pairs(ctx, da, b0, nb), b0, nb);
  }
  return check_launch(ctx, "gb_delta_loglike");
}

extern "C" int gb_delta_loglike_var(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* psd,
                                    int32_t n_psd, int32_t psd_flags, const double* params_old,
                                    const double* params_new, const int32_t* N, const int32_t* res_idx,
                                    const int32_t* psd_idx, int64_t B, double* dlogl) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0 || n_res < 1 || n_psd < 1) return fail(ctx, GBL_EINVAL, "gb_delta_loglike_var: bad sizes%s");
  if (psd_flags & ~GBL_PSD_INVERSE) return fail(ctx, GBL_EINVAL, "gb_delta_loglike_var: unknown psd flag%s");
  if (B == 0) return GBL_OK;
  if (!residual || !psd || !params_old || !params_new || !N || !res_idx || !psd_idx || !dlogl)
    return fail(ctx, GBL_EINVAL, "gb_delta_loglike_var: null pointer%s");
  const gbl::DeltaArgs da_all = {(const cd*)residual, (int)n_res, psd, (int)n_psd,
                             (psd_flags & GBL_PSD_INVERSE) ? 1 : 0, params_old, params_new, res_idx, psd_idx, dlogl,
                             nullptr, nullptr, 0.0, 0, nullptr, 0};
  const int64_t chunk = std::min<int64_t>(ctx->tune.bucket_chunk, kDecodeChunk);
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    int64_t nb = B - b0 < chunk ? B - b0 : chunk;
    const gbl::DeltaArgs dc = decode_pairs(ctx, da_all, b0, nb);
    bucket_widths(ctx, N, b0, nb, dlogl, nullptr);
    int cnt[kNumWidths];
    if (!host_counts(ctx, ctx->counts, kNumWidths, cnt))
      for (int w = 0; w < kNumWidths; w++) cnt[w] = (int)nb;
    if (routed(ctx))
      hipLaunchKernelGGL(gbl::k_bucket_reset, dim3(1), dim3(64), 0, ctx->stream, ctx->route_counts, kNumWidths);
    // widest first (default): the long blocks start early and the short ones fill in
    if (ctx->tune.widest_first) {
      LaunchDeltaBucket<1024>::run(ctx, dc, b0, cnt[3]);
      LaunchDeltaBucket<512>::run(ctx, dc, b0, cnt[2]);
      LaunchDeltaBucket<256>::run(ctx, dc, b0, cnt[1]);
      LaunchDeltaBucket<128>::run(ctx, dc, b0, cnt[0]);
    } else {
      LaunchDeltaBucket<128>::run(ctx, dc, b0, cnt[0]);
      LaunchDeltaBucket<256>::run(ctx, dc, b0, cnt[1]);
      LaunchDeltaBucket<512>::run(ctx, dc, b0, cnt[2]);
      LaunchDeltaBucket<1024>::run(ctx, dc, b0, cnt[3]);
    }
    if (routed(ctx)) {
      int rc[kNumWidths];
      const bool exact = host_counts(ctx, ctx->route_counts, kNumWidths, rc);
      launch_route_pass<1024>(ctx, dc, b0, exact ? rc[3] : cnt[3]);
      launch_route_pass<512>(ctx, dc, b0, exact ? rc[2] : cnt[2]);
      launch_route_pass<256>(ctx, dc, b0, exact ? rc[1] : cnt[1]);
      launch_route_pass<128>(ctx, dc, b0, exact ? rc[0] : cnt[0]);
    }
  }
  return check_launch(ctx, "gb_delta_loglike_var");
}

extern "C" int gb_waveform_var(gbl_ctx* ctx, const double* params, const int32_t* N, const int64_t* out_offset,
                               int64_t B, double* A, double* E, double* Tch, int64_t* start_bin) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0) return fail(ctx, GBL_EINVAL, "gb_waveform_var: B < 0%s");
  if (B == 0) return GBL_OK;
  if (!params || !N || !out_offset || !A || !E || !start_bin)
    return fail(ctx, GBL_EINVAL, "gb_waveform_var: null pointer%s");
  const int64_t chunk = ctx->tune.bucket_chunk;
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    int64_t nb = B - b0 < chunk ? B - b0 : chunk;
    bucket_widths(ctx, N, b0, nb, nullptr, start_bin);
    int cnt[kNumWidths];
    if (!host_counts(ctx, ctx->counts, kNumWidths, cnt))
      for (int w = 0; w < kNumWidths; w++) cnt[w] = (int)nb;
    LaunchWaveformBucket<1024>::run(ctx, params, b0, cnt[3], out_offset, (cd*)A, (cd*)E, (cd*)Tch, start_bin);
    LaunchWaveformBucket<512>::run(ctx, params, b0, cnt[2], out_offset, (cd*)A, (cd*)E, (cd*)Tch, start_bin);
    LaunchWaveformBucket<256>::run(ctx, params, b0, cnt[1], out_offset, (cd*)A, (cd*)E, (cd*)Tch, start_bin);
    LaunchWaveformBucket<128>::run(ctx, params, b0, cnt[0], out_offset, (cd*)A, (cd*)E, (cd*)Tch, start_bin);
  }
  return check_launch(ctx, "gb_waveform_var");
}

static gbl::PsdBasis psd_basis(const gbl_ctx* ctx) {
  return gbl::PsdBasis{ctx->psd_P1, ctx->psd_P2, ctx->psd_P3, ctx->psd_LF, ctx->geo.k_min, ctx->cfg.T};
}

static void psd_eval_launch(gbl_ctx* ctx, const double* noise, int n_par, int64_t P, int inverse, double* S) {
  if (n_par == 9)
    hipLaunchKernelGGL(gbl::k_psd_eval<9>, gbl::row_grid(ctx->geo.n_bins, 2 * P), dim3(256), 0, ctx->stream,
                       ctx->geo.n_bins, psd_basis(ctx), noise, P, inverse, S);
  else
    hipLaunchKernelGGL(gbl::k_psd_eval<4>, gbl::row_grid(ctx->geo.n_bins, 2 * P), dim3(256), 0, ctx->stream,
                       ctx->geo.n_bins, psd_basis(ctx), noise, P, inverse, S);
}

extern "C" int gb_psd_eval_n(gbl_ctx* ctx, const double* noise, int32_t n_par, int64_t P, int32_t psd_flags,
                             double* S) {
  if (!ctx) return GBL_EINVAL;
  if (P < 0) return fail(ctx, GBL_EINVAL, "gb_psd_eval: P < 0%s");
  if (n_par != 4 && n_par != 9) return fail(ctx, GBL_EINVAL, "gb_psd_eval: n_par must be 4 or 9%s");
  if (psd_flags & ~GBL_PSD_INVERSE) return fail(ctx, GBL_EINVAL, "gb_psd_eval: unknown psd flag%s");
  if (P == 0) return GBL_OK;
  if (!noise || !S) return fail(ctx, GBL_EINVAL, "gb_psd_eval: null pointer%s");
  psd_eval_launch(ctx, noise, n_par, P, (psd_flags & GBL_PSD_INVERSE) ? 1 : 0, S);
  return check_launch(ctx, "gb_psd_eval");
}

extern "C" int gb_psd_eval(gbl_ctx* ctx, const double* noise, int64_t P, int32_t psd_flags, double* S) {
  return gb_psd_eval_n(ctx, noise, 4, P, psd_flags, S);
}

// PSD likelihood of P parameter sets: partial sums in groups of kPsdSets sets (the
// remainder one set per block), then the fixed-order final sum per set.
template <int NP>
static void psd_partial_launch(gbl_ctx* ctx, const cd* residual, int n_res, const double* noise,
                               const int32_t* res_idx, int64_t p0, int64_t np, double* work, int map_nt,
                               int map_nw) {
  const int64_t ng = np / gbl::kPsdSets, rest = np - ng * gbl::kPsdSets;
  if (ng > 0)
    hipLaunchKernelGGL((gbl::k_psd_partial<gbl::kPsdSets, NP>), dim3(gbl::kPsdChunks, (unsigned)ng),
                       dim3(gbl::kPsdBlock), 0, ctx->stream, ctx->geo.n_bins, psd_basis(ctx), residual, n_res, noise,
                       res_idx, p0, p0, work, map_nt, map_nw);
  if (rest > 0)
    hipLaunchKernelGGL((gbl::k_psd_partial<1, NP>), dim3(gbl::kPsdChunks, (unsigned)rest), dim3(gbl::kPsdBlock), 0,
                       ctx->stream, ctx->geo.n_bins, psd_basis(ctx), residual, n_res, noise, res_idx, p0,
                       p0 + ng * gbl::kPsdSets, work, map_nt, map_nw);
}

// work: [kPsdBatch][kPsdChunks][2] partial sums (the context's workspace, or
// the static scratch for batches of at most kScratchSets sets)
// tn_major_nt > 0: the P sets are tn_major_nt temperatures x P / tn_major_nt
// walkers, temperature-major, each walker's sets on one residual row; the
// blocks then take them walker-major (one row read per block of sets)
static void psd_loglike_launch(gbl_ctx* ctx, const cd* residual, int n_res, const double* noise, int n_par,
                               const int32_t* res_idx, int64_t P, double* logl, double* work = nullptr,
                               int tn_major_nt = 0) {
  if (!work) work = ctx->psd_work;
  const bool mapped = tn_major_nt > 0 && P <= kPsdBatch && P % tn_major_nt == 0 &&
                      tn_major_nt % gbl::kPsdSets == 0;
  const int map_nt = mapped ? tn_major_nt : 0;
  const int map_nw = mapped ? (int)(P / tn_major_nt) : 0;
  for (int64_t p0 = 0; p0 < P; p0 += kPsdBatch) {
    const int64_t np = P - p0 < kPsdBatch ? P - p0 : kPsdBatch;
    if (n_par == 9)
      psd_partial_launch<9>(ctx, residual, n_res, noise, res_idx, p0, np, work, map_nt, map_nw);
    else
      psd_partial_launch<4>(ctx, residual, n_res, noise, res_idx, p0, np, work, map_nt, map_nw);
    hipLaunchKernelGGL(gbl::k_psd_final, dim3((unsigned)np), dim3(64), 0, ctx->stream, 1.0 / ctx->cfg.T, work, p0,
                       logl);
  }
}

extern "C" int gb_psd_loglike_n(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* noise,
                                int32_t n_par, const int32_t* res_idx, int64_t P, double* logl) {
  if (!ctx) return GBL_EINVAL;
  if (P < 0 || n_res < 1) return fail(ctx, GBL_EINVAL, "gb_psd_loglike: bad sizes%s");
  if (n_par != 4 && n_par != 9) return fail(ctx, GBL_EINVAL, "gb_psd_loglike: n_par must be 4 or 9%s");
  if (P == 0) return GBL_OK;
  if (!residual || !noise || !res_idx || !logl) return fail(ctx, GBL_EINVAL, "gb_psd_loglike: null pointer%s");
  psd_loglike_launch(ctx, (const cd*)residual, (int)n_res, noise, n_par, res_idx, P, logl);
  return check_launch(ctx, "gb_psd_loglike");
}

extern "C" int gb_psd_loglike_noalloc(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* noise,
                                      int32_t n_par, const int32_t* res_idx, int64_t P, double* logl) {
  if (!ctx) return GBL_EINVAL;
  if (P < 0 || n_res < 1) return fail(ctx, GBL_EINVAL, "gb_psd_loglike_noalloc: bad sizes%s");
  if (P > kScratchSets) return fail(ctx, GBL_EINVAL, "gb_psd_loglike_noalloc: more than 2048 parameter sets%s");
  if (n_par != 4 && n_par != 9) return fail(ctx, GBL_EINVAL, "gb_psd_loglike_noalloc: n_par must be 4 or 9%s");
  if (P == 0) return GBL_OK;
  if (!residual || !noise || !res_idx || !logl)
    return fail(ctx, GBL_EINVAL, "gb_psd_loglike_noalloc: null pointer%s");
  // every partial sum is written before it is read: nothing to clear
  psd_loglike_launch(ctx, (const cd*)residual, (int)n_res, noise, n_par, res_idx, P, logl, ctx->scratch);
  return check_launch(ctx, "gb_psd_loglike_noalloc");
}

extern "C" int gb_psd_loglike(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* noise,
                              const int32_t* res_idx, int64_t P, double* logl) {
  return gb_psd_loglike_n(ctx, residual, n_res, noise, 4, res_idx, P, logl);
}

extern "C" int gb_scatter_add(gbl_ctx* ctx, const double* params, int64_t B, int32_t N, double sign,
                              double* residual, int32_t n_res, const int32_t* res_idx) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0 || n_res < 1) return fail(ctx, GBL_EINVAL, "gb_scatter_add: bad sizes%s");
  if (width_slot(N) < 0) return fail(ctx, GBL_EUNSUPPORTED, "gb_scatter_add: unsupported N%s");
  if (B == 0) return GBL_OK;
  if (!params || !residual || !res_idx) return fail(ctx, GBL_EINVAL, "gb_scatter_add: null pointer%s");
  if (ctx->cfg.flags & GBL_DETERMINISTIC) {
    int rc = GBL_OK;
    dispatch_width<LaunchDetScatter>(N, ctx, params, (int64_t)0, B, sign, (cd*)residual, (int)n_res, res_idx, &rc);
    if (rc != GBL_OK) return rc;
    return check_launch(ctx, "gb_scatter_add");
  }
  for (int64_t b0 = 0; b0 < B; b0 += kMaxGrid) {
    int64_t nb = B - b0 < kMaxGrid ? B - b0 : kMaxGrid;
    dispatch_width<LaunchScatter>(N, ctx, params, b0, nb, sign, (cd*)residual, (int)n_res, res_idx);
  }
  return check_launch(ctx, "gb_scatter_add");
}

extern "C" int gb_inner(gbl_ctx* ctx, const double* A, const double* E, const int64_t* start_bin, int32_t N,
                        const double* residual, int32_t n_res, const double* psd, int32_t n_psd, int32_t psd_flags,
                        const int32_t* res_idx, const int32_t* psd_idx, int64_t B, double* out) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0 || N < 1 || n_res < 1 || n_psd < 1) return fail(ctx, GBL_EINVAL, "gb_inner: bad sizes%s");
  if (psd_flags & ~GBL_PSD_INVERSE) return fail(ctx, GBL_EINVAL, "gb_inner: unknown psd flag%s");
  if (B == 0) return GBL_OK;
  if (!A || !E || !start_bin || !residual || !psd || !res_idx || !psd_idx || !out)
    return fail(ctx, GBL_EINVAL, "gb_inner: null pointer%s");
  for (int64_t b0 = 0; b0 < B; b0 += kMaxGrid * gbl::kInnerWaves) {
    const int64_t nb = B - b0 < kMaxGrid * gbl::kInnerWaves ? B - b0 : kMaxGrid * gbl::kInnerWaves;
    hipLaunchKernelGGL(gbl::k_inner, dim3((unsigned)((nb + gbl::kInnerWaves - 1) / gbl::kInnerWaves)),
                       dim3(gbl::kInnerWaves * gbl::kWave), 0, ctx->stream, ctx->geo,
                       (const cd*)A + b0 * N, (const cd*)E + b0 * N, start_bin + b0, (int)N, (const cd*)residual,
                       (int)n_res, psd, (int)n_psd, (psd_flags & GBL_PSD_INVERSE) ? 1 : 0, res_idx + b0,
                       psd_idx + b0, nb, out + 2 * b0);
  }
  return check_launch(ctx, "gb_inner");
}

extern "C" int gb_overlap(gbl_ctx* ctx, const double* params_a, const double* params_b, int32_t N,
                          const double* psd, int32_t n_psd, int32_t psd_flags, const int32_t* psd_idx, int64_t B,
                          double* out) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0 || n_psd < 1) return fail(ctx, GBL_EINVAL, "gb_overlap: bad sizes%s");
  if (width_slot(N) < 0) return fail(ctx, GBL_EUNSUPPORTED, "gb_overlap: unsupported N%s");
  if (psd_flags & ~GBL_PSD_INVERSE) return fail(ctx, GBL_EINVAL, "gb_overlap: unknown psd flag%s");
  if (B == 0) return GBL_OK;
  if (!params_a || !params_b || !psd || !psd_idx || !out) return fail(ctx, GBL_EINVAL, "gb_overlap: null pointer%s");
  for (int64_t b0 = 0; b0 < B; b0 += kMaxGrid) {
    const int64_t nb = B - b0 < kMaxGrid ? B - b0 : kMaxGrid;
    dispatch_width<LaunchOverlap>(N, ctx, params_a, params_b, b0, nb, psd, (int)n_psd,
                                  (psd_flags & GBL_PSD_INVERSE) ? 1 : 0, psd_idx, out);
  }
  return check_launch(ctx, "gb_overlap");
}

extern "C" int gb_snr(gbl_ctx* ctx, const double* params, int64_t B, int32_t N, const double* psd, int32_t n_psd,
                      int32_t psd_flags, const int32_t* psd_idx, const double* data, int32_t n_data,
                      const int32_t* data_idx, double* snr_opt, double* snr_obs) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0 || n_psd < 1 || (data && n_data < 1)) return fail(ctx, GBL_EINVAL, "gb_snr: bad sizes%s");
  if (width_slot(N) < 0) return fail(ctx, GBL_EUNSUPPORTED, "gb_snr: unsupported N%s");
  if (psd_flags & ~GBL_PSD_INVERSE) return fail(ctx, GBL_EINVAL, "gb_snr: unknown psd flag%s");
  if (B == 0) return GBL_OK;
  if (!params || !psd || !psd_idx || !snr_opt || (data && (!data_idx || !snr_obs)))
    return fail(ctx, GBL_EINVAL, "gb_snr: null pointer%s");
  for (int64_t b0 = 0; b0 < B; b0 += kMaxGrid) {
    const int64_t nb = B - b0 < kMaxGrid ? B - b0 : kMaxGrid;
    dispatch_width<LaunchSnr>(N, ctx, params, b0, nb, psd, (int)n_psd, (psd_flags & GBL_PSD_INVERSE) ? 1 : 0,
                              psd_idx, (const cd*)data, (int)n_data, data_idx, snr_opt, data ? snr_obs : nullptr);
  }
  return check_launch(ctx, "gb_snr");
}

extern "C" int gb_make_noise(gbl_ctx* ctx, const double* S, const double* normals, int64_t n, double* out) {
  if (!ctx) return GBL_EINVAL;
  if (n < 0) return fail(ctx, GBL_EINVAL, "gb_make_noise: n < 0%s");
  if (n == 0) return GBL_OK;
  if (!S || !normals || !out) return fail(ctx, GBL_EINVAL, "gb_make_noise: null pointer%s");
  int64_t total = n * 2 * ctx->geo.n_bins;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(gbl::k_make_noise, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, total,
                     ctx->cfg.T / 4.0, S, (const cd*)normals, (cd*)out);
  return check_launch(ctx, "gb_make_noise");
}

// ---------------------------------------------------------------------------
// sampler sweep (Sec. 4; appendix algorithms gb1 and gb2)
// ---------------------------------------------------------------------------
static int sweep_check(gbl_ctx* ctx, const gbl_sweep_config* c, const gbl_sweep_state* st) {
  if (!c || !st) return fail(ctx, GBL_EINVAL, "sweep: null config or state%s");
  if (c->N != 128 && c->N != 256 && c->N != 512 && c->N != 1024)
    return fail(ctx, GBL_EUNSUPPORTED, "sweep: N must be 128, 256, 512 or 1024%s");
  if (c->n_temps < 1 || c->n_temps > 256 || c->n_walkers < 1 || c->n_walkers > 256 || c->n_bands < 1 ||
      c->n_slots < 1 || c->n_slots > gbl::kMaxSlots || c->n_prop < 0 || c->n_friends < 1 || !(c->stretch_a > 1.0))
    return fail(ctx, GBL_EINVAL, "sweep: configuration out of range%s");
  if (!st->u || !st->exists || !st->betas || !st->resid || !st->inv_psd || !st->group || !st->group_count ||
      !st->stats || !st->sweep_counter)
    return fail(ctx, GBL_EINVAL, "sweep: null state pointer%s");
  if ((st->prop_u == nullptr) != (st->rj_logq == nullptr))
    return fail(ctx, GBL_EINVAL, "sweep: prop_u and rj_logq must be given together%s");
  if (st->spec_pool && (!st->pool_flags || st->pool_size < 1))
    return fail(ctx, GBL_EINVAL, "sweep: spectrum pool without flags or size%s");
  if (c->adapt_ladder && (!st->swap_acc || !(c->adapt_lag > 0.0) || !(c->adapt_time > 0.0)))
    return fail(ctx, GBL_EINVAL, "sweep: ladder adaptation needs swap_acc and positive adapt_lag, adapt_time%s");
  if (c->band_width < 0 || (c->band_width & 1))
    return fail(ctx, GBL_EINVAL, "sweep: band_width must be even and non-negative%s");
  if (((c->band_width != 0 && c->band_width != c->N) || c->N == 1024) && !st->window_sums)
    return fail(ctx, GBL_EINVAL,
                "sweep: a band width other than N, or N = 1024, needs window_sums (the windows live there)%s");
  if (ctx->cfg.precision != GBL_FP64 && !(ctx->cfg.precision == GBL_MIXED && st->window_sums))
    return fail(ctx, GBL_EUNSUPPORTED,
                "sweep: FP64 contexts, or mixed-precision contexts with window_sums (tempering then builds no "
                "template)%s");
  return GBL_OK;
}

static gbl::SweepArgs sweep_args(const gbl_sweep_config* c, const gbl_sweep_state* st) {
  gbl::SweepArgs a;
  a.n_t = c->n_temps;
  a.n_w = c->n_walkers;
  a.n_b = c->n_bands;
  a.n_slot = c->n_slots;
  a.n_prop = c->n_prop;
  a.n_friends = c->n_friends;
  a.band_w = c->band_width > 0 ? c->band_width : c->N;
  a.k_band0 = c->k_band0;
  a.stretch_a = c->stretch_a;
  a.seed = c->seed;
  for (int i = 0; i < 8; i++) {
    a.lo[i] = c->prior_lo[i];
    a.hi[i] = c->prior_hi[i];
  }
  a.u = st->u;
  a.exists = st->exists;
  a.betas = st->betas;
  a.resid = (cd*)st->resid;
  a.inv_psd = st->inv_psd;
  a.group = st->group;
  a.group_count = st->group_count;
  a.stats = (unsigned long long*)st->stats;
  a.sweep_ctr = st->sweep_counter;
  a.prop_u = st->prop_u;
  a.rj_logq = st->rj_logq;
  a.cold_logl = st->cold_logl;
  a.swap_acc = st->swap_acc;
  a.spec_pool = (cd*)st->spec_pool;
  a.pool_flags = st->pool_flags;
  a.pool_size = st->pool_size;
  a.wsum = (cd*)st->window_sums;
  return a;
}

// the band loops of one parity; F: precision of their template response and
// FFT (float in mixed-precision contexts)
template <int N, typename F>
static void launch_band_loops(gbl_ctx* ctx, const gbl::SweepArgs& a, int move, int parity, int nbp) {
  const gbl::WaveTables<F>& tb = tables_for<N, F>(ctx);
  if (a.band_w != N || N == 1024 || (N == 512 && a.wsum))
    // the windows (2W + N bins) in global memory; at N = 512 also whenever the
    // window sums are there to hold them (the LDS window would leave room
    // for one block per CU, the global one for two)
    hipLaunchKernelGGL((gbl::k_sweep_band<N, true, F>), dim3((unsigned)(nbp * a.n_w * a.n_t)),
                       dim3(gbl::loop_threads<N>()), 0, ctx->stream, ctx->geo, tb, a, move, parity);
  else if constexpr (N <= 512)
    hipLaunchKernelGGL((gbl::k_sweep_band<N, false, F>), dim3((unsigned)(nbp * a.n_w * a.n_t)),
                       dim3(gbl::loop_threads<N>()), 0, ctx->stream, ctx->geo, tb, a, move, parity);
}

template <int N>
static void launch_sweep_step(gbl_ctx* ctx, const gbl::SweepArgs& a, int move, int parity) {
  const int nbp = (a.n_b - parity + 1) / 2;
  if (nbp <= 0) return;
  if (move == GBL_MOVE_PT && a.wsum)
    hipLaunchKernelGGL((gbl::k_sweep_pt<N, true>), dim3((unsigned)(nbp * a.n_w)), dim3(gbl::block_threads<N>()), 0,
                       ctx->stream, ctx->geo, tables_for<N, double>(ctx), a, parity);
  else if (move == GBL_MOVE_PT)
    hipLaunchKernelGGL((gbl::k_sweep_pt<N, false>), dim3((unsigned)(nbp * a.n_w)), dim3(gbl::block_threads<N>()),
                       0, ctx->stream, ctx->geo, tables_for<N, double>(ctx), a, parity);
  else if (ctx->cfg.precision == GBL_MIXED)
    launch_band_loops<N, float>(ctx, a, move, parity, nbp);
  else
    launch_band_loops<N, double>(ctx, a, move, parity, nbp);
}

static void sweep_adapt(gbl_ctx* ctx, const gbl_sweep_config* c, const gbl::SweepArgs& a) {
  hipLaunchKernelGGL(gbl::k_sweep_adapt, dim3((unsigned)((a.n_b + 63) / 64)), dim3(64), 0, ctx->stream, a,
                     c->adapt_lag, c->adapt_time);
}

static void sweep_shift(gbl_ctx* ctx, const gbl_sweep_config* c, const gbl::SweepArgs& a) {
  switch (c->N) {
    case 128:
      hipLaunchKernelGGL(gbl::k_sweep_shift<128>, dim3((unsigned)a.n_w), dim3(gbl::block_threads<128>()), 0,
                         ctx->stream, ctx->geo, tables_for<128, double>(ctx), a);
      break;
    case 256:
      hipLaunchKernelGGL(gbl::k_sweep_shift<256>, dim3((unsigned)a.n_w), dim3(gbl::block_threads<256>()), 0,
                         ctx->stream, ctx->geo, tables_for<256, double>(ctx), a);
      break;
    case 512:
      hipLaunchKernelGGL(gbl::k_sweep_shift<512>, dim3((unsigned)a.n_w), dim3(gbl::block_threads<512>()), 0,
                         ctx->stream, ctx->geo, tables_for<512, double>(ctx), a);
      break;
    case 1024:
      hipLaunchKernelGGL(gbl::k_sweep_shift<1024>, dim3((unsigned)a.n_w), dim3(gbl::block_threads<1024>()), 0,
                         ctx->stream, ctx->geo, tables_for<1024, double>(ctx), a);
      break;
    default: break;
  }
}

static void sweep_step(gbl_ctx* ctx, const gbl_sweep_config* c, const gbl::SweepArgs& a, int move, int parity) {
  switch (c->N) {
    case 128: launch_sweep_step<128>(ctx, a, move, parity); break;
    case 256: launch_sweep_step<256>(ctx, a, move, parity); break;
    case 512: launch_sweep_step<512>(ctx, a, move, parity); break;
    case 1024: launch_sweep_step<1024>(ctx, a, move, parity); break;
    default: break;
  }
}

extern "C" int gb_sweep_step(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st, int32_t move,
                             int32_t parity) {
  if (!ctx) return GBL_EINVAL;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  if (move < GBL_MOVE_INMODEL || move > GBL_MOVE_PT || (parity != 0 && parity != 1))
    return fail(ctx, GBL_EINVAL, "gb_sweep_step: bad move or parity%s");
  sweep_step(ctx, cfg, sweep_args(cfg, st), move, parity);
  return check_launch(ctx, "gb_sweep_step");
}

extern "C" int gb_sweep_group(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st) {
  if (!ctx) return GBL_EINVAL;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  hipLaunchKernelGGL(gbl::k_sweep_group, dim3((unsigned)cfg->n_bands), dim3(256), 0, ctx->stream,
                     sweep_args(cfg, st), 0);
  return check_launch(ctx, "gb_sweep_group");
}

extern "C" int gb_sweep_adapt_ladder(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st) {
  if (!ctx) return GBL_EINVAL;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  if (!st->swap_acc || !(cfg->adapt_lag > 0.0) || !(cfg->adapt_time > 0.0))
    return fail(ctx, GBL_EINVAL, "gb_sweep_adapt_ladder: needs swap_acc and positive adapt_lag, adapt_time%s");
  sweep_adapt(ctx, cfg, sweep_args(cfg, st));
  return check_launch(ctx, "gb_sweep_adapt_ladder");
}

extern "C" int gb_sweep_shift_ownership(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st) {
  if (!ctx) return GBL_EINVAL;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  sweep_shift(ctx, cfg, sweep_args(cfg, st));
  return check_launch(ctx, "gb_sweep_shift_ownership");
}

extern "C" int gb_sweep_advance(gbl_ctx* ctx, const gbl_sweep_state* st) {
  if (!ctx) return GBL_EINVAL;
  if (!st || !st->sweep_counter) return fail(ctx, GBL_EINVAL, "gb_sweep_advance: null state%s");
  hipLaunchKernelGGL(gbl::k_sweep_advance, dim3(1), dim3(64), 0, ctx->stream, st->sweep_counter);
  return check_launch(ctx, "gb_sweep_advance");
}

static int rj_prepare(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                      const gbl_flow_config* fcfg, const gbl_flow* fl);

static int sweep_run_impl(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                          const gbl_flow_config* fcfg, const gbl_flow* fl, int32_t n_sweeps) {
  const gbl::SweepArgs a = sweep_args(cfg, st);
  for (int i = 0; i < n_sweeps; i++) {
    if (cfg->group_every > 0)
      hipLaunchKernelGGL(gbl::k_sweep_group, dim3((unsigned)cfg->n_bands), dim3(256), 0, ctx->stream, a,
                         cfg->group_every);
    for (int move = GBL_MOVE_INMODEL; move <= GBL_MOVE_PT; move++) {
      if (move == GBL_MOVE_RJ && fl) {
        int rc = rj_prepare(ctx, cfg, st, fcfg, fl);
        if (rc) return rc;
      }
      for (int parity = 1; parity >= 0; parity--) sweep_step(ctx, cfg, a, move, parity);
    }
    if (cfg->adapt_ladder) sweep_adapt(ctx, cfg, a);
    if (cfg->shift_ownership) sweep_shift(ctx, cfg, a);
    hipLaunchKernelGGL(gbl::k_sweep_advance, dim3(1), dim3(64), 0, ctx->stream, st->sweep_counter);
  }
  return check_launch(ctx, "gb_sweep_run");
}

extern "C" int gb_sweep_run(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                            int32_t n_sweeps) {
  if (!ctx) return GBL_EINVAL;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  if (n_sweeps < 0) return fail(ctx, GBL_EINVAL, "gb_sweep_run: n_sweeps < 0%s");
  return sweep_run_impl(ctx, cfg, st, nullptr, nullptr, n_sweeps);
}

struct gbl_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipStream_t stream;
};

static int graph_create_impl(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                             const gbl_flow_config* fcfg, const gbl_flow* fl, int32_t n_sweeps, gbl_graph** out) {
  if (!ctx || !out) return GBL_EINVAL;
  *out = nullptr;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  if (n_sweeps < 1) return fail(ctx, GBL_EINVAL, "gb_sweep_graph_create: n_sweeps < 1%s");
  if (!ctx->stream) return fail(ctx, GBL_EINVAL, "gb_sweep_graph_create: capture needs a non-default stream%s");
  gbl_graph* gr = new gbl_graph();
  gr->stream = ctx->stream;
  if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete gr;
    return fail(ctx, GBL_EHIP, "gb_sweep_graph_create: begin capture failed%s");
  }
  int rr = sweep_run_impl(ctx, cfg, st, fcfg, fl, n_sweeps);
  hipError_t e = hipStreamEndCapture(ctx->stream, &gr->graph);
  if (rr != GBL_OK || e != hipSuccess) {
    if (e == hipSuccess) (void)hipGraphDestroy(gr->graph);
    delete gr;
    return fail(ctx, GBL_EHIP, "gb_sweep_graph_create: capture failed%s");
  }
  if (hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(gr->graph);
    delete gr;
    return fail(ctx, GBL_EHIP, "gb_sweep_graph_create: instantiate failed%s");
  }
  *out = gr;
  return GBL_OK;
}

extern "C" int gb_sweep_graph_create(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                                     int32_t n_sweeps, gbl_graph** out) {
  return graph_create_impl(ctx, cfg, st, nullptr, nullptr, n_sweeps, out);
}

extern "C" int gb_graph_launch(gbl_graph* gr) {
  if (!gr) return GBL_EINVAL;
  return hipGraphLaunch(gr->exec, gr->stream) == hipSuccess ? GBL_OK : GBL_EHIP;
}

extern "C" int gb_graph_destroy(gbl_graph* gr) {
  if (!gr) return GBL_OK;
  (void)hipStreamSynchronize(gr->stream);
  (void)hipGraphExecDestroy(gr->exec);
  (void)hipGraphDestroy(gr->graph);
  delete gr;
  return GBL_OK;
}

// ---------------------------------------------------------------------------
// learned RJ proposal (flow)
// ---------------------------------------------------------------------------
static int64_t flow_n_params(const gbl_flow_config* c) {
  return (int64_t)gbl::flow::kLayers * gbl::flow::kLayerParams + (int64_t)gbl::flow::kEmb * c->n_emb;
}

static int64_t flow_workspace_bytes() {
  return (int64_t)gbl::flow::kMaxGroups * gbl::flow::kLayers * gbl::flow::kLayerParams * 4 +
         (int64_t)gbl::flow::kMaxGroups * 8;
}

extern "C" int gb_flow_sizes(const gbl_flow_config* cfg, int64_t* n_params, int64_t* packed_bytes,
                             int64_t* workspace_bytes) {
  if (!cfg || cfg->n_emb < 1) return GBL_EINVAL;
  if (n_params) *n_params = flow_n_params(cfg);
  if (packed_bytes) *packed_bytes = gbl::flow::kPackedBytes;
  if (workspace_bytes) *workspace_bytes = flow_workspace_bytes();
  return GBL_OK;
}

static int flow_check(gbl_ctx* ctx, const gbl_flow_config* c, const gbl_flow* f) {
  if (!c || !f) return fail(ctx, GBL_EINVAL, "flow: null config or state%s");
  if (c->n_emb < 1 || c->width < 1) return fail(ctx, GBL_EINVAL, "flow: n_emb and width must be positive%s");
  const int dims[4] = {0, 2, 4, 7};
  for (int i : dims)
    if (!(c->prior_lo[i] < c->prior_hi[i])) return fail(ctx, GBL_EINVAL, "flow: empty prior box%s");
  if (!f->params || !f->packed) return fail(ctx, GBL_EINVAL, "flow: null params or packed buffer%s");
  return GBL_OK;
}

static gbl::flow::FlowArgs flow_args(gbl_ctx* ctx, const gbl_flow_config* c, const gbl_flow* f) {
  gbl::flow::FlowArgs a;
  a.params = f->params;
  a.packed = (const gbl::flow::u32x4_t*)f->packed;
  a.n_emb = c->n_emb;
  a.width = c->width;
  a.k_band0 = c->k_band0;
  a.T = ctx->cfg.T;
  for (int i = 0; i < 8; i++) {
    a.lo[i] = c->prior_lo[i];
    a.hi[i] = c->prior_hi[i];
  }
  a.band_div = 1;
  a.band_mod = 1;
  a.mask_want = 0;
  a.mask = nullptr;
  return a;
}

extern "C" int gb_flow_pack(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* fl) {
  if (!ctx) return GBL_EINVAL;
  int rc = flow_check(ctx, cfg, fl);
  if (rc) return rc;
  const int n = gbl::flow::kLayers * gbl::flow::kFragPerLayer * 64;
  hipLaunchKernelGGL(gbl::flow::k_flow_pack, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, fl->params,
                     (gbl::flow::u32x4_t*)fl->packed);
  return check_launch(ctx, "gb_flow_pack");
}

static unsigned flow_grid(const gbl_ctx* ctx, int64_t B) {
  const int64_t blocks = (B + 63) / 64;
  return (unsigned)(blocks < ctx->tune.flow_grid ? blocks : ctx->tune.flow_grid);
}

extern "C" int gb_flow_log_prob(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* fl, const double* u,
                                const int32_t* band, int64_t B, double* logq) {
  if (!ctx) return GBL_EINVAL;
  int rc = flow_check(ctx, cfg, fl);
  if (rc) return rc;
  if (B < 0) return fail(ctx, GBL_EINVAL, "gb_flow_log_prob: B < 0%s");
  if (B == 0) return GBL_OK;
  if (!u || !band || !logq) return fail(ctx, GBL_EINVAL, "gb_flow_log_prob: null pointer%s");
  hipLaunchKernelGGL(gbl::flow::k_flow_apply<false>, dim3(flow_grid(ctx, B)), dim3(256), 0, ctx->stream,
                     flow_args(ctx, cfg, fl), u, band, B, (double*)nullptr, logq);
  return check_launch(ctx, "gb_flow_log_prob");
}

extern "C" int gb_flow_sample(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* fl, const double* z,
                              const int32_t* band, int64_t B, double* u, double* logq) {
  if (!ctx) return GBL_EINVAL;
  int rc = flow_check(ctx, cfg, fl);
  if (rc) return rc;
  if (B < 0) return fail(ctx, GBL_EINVAL, "gb_flow_sample: B < 0%s");
  if (B == 0) return GBL_OK;
  if (!z || !band || !u || !logq) return fail(ctx, GBL_EINVAL, "gb_flow_sample: null pointer%s");
  hipLaunchKernelGGL(gbl::flow::k_flow_apply<true>, dim3(flow_grid(ctx, B)), dim3(256), 0, ctx->stream,
                     flow_args(ctx, cfg, fl), z, band, B, u, logq);
  return check_launch(ctx, "gb_flow_sample");
}

extern "C" int gb_flow_grad(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* fl, const double* u,
                            const int32_t* band, int64_t B) {
  if (!ctx) return GBL_EINVAL;
  int rc = flow_check(ctx, cfg, fl);
  if (rc) return rc;
  if (B < 1) return fail(ctx, GBL_EINVAL, "gb_flow_grad: B < 1%s");
  if (!u || !band || !fl->grad || !fl->workspace || !fl->loss)
    return fail(ctx, GBL_EINVAL, "gb_flow_grad: null pointer%s");
  using namespace gbl::flow;
  const int64_t n_layer = (int64_t)kLayers * kLayerParams;
  const int64_t n_emb = (int64_t)kEmb * cfg->n_emb;
  hipLaunchKernelGGL(k_flow_fill, dim3((unsigned)((n_emb + 255) / 256)), dim3(256), 0, ctx->stream,
                     fl->grad + n_layer, n_emb, 0.0f);
  const int64_t chunks = (B + kChunk - 1) / kChunk;
  const int groups = (int)(chunks < kMaxGroups ? chunks : kMaxGroups);
  float* partial = (float*)fl->workspace;
  double* loss_part = (double*)((char*)fl->workspace + (int64_t)kMaxGroups * n_layer * 4);
  hipLaunchKernelGGL(k_flow_grad, dim3(groups), dim3(256), 0, ctx->stream, flow_args(ctx, cfg, fl), u, band, B,
                     partial, loss_part, fl->grad + n_layer);
  hipLaunchKernelGGL(k_flow_reduce, dim3((unsigned)((n_layer + 255) / 256)), dim3(256), 0, ctx->stream,
                     (const float*)partial, groups, (const double*)loss_part, fl->grad, fl->loss);
  return check_launch(ctx, "gb_flow_grad");
}

extern "C" int gb_flow_adam(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* fl, int64_t step, float lr) {
  if (!ctx) return GBL_EINVAL;
  int rc = flow_check(ctx, cfg, fl);
  if (rc) return rc;
  if (step < 1 || !(lr >= 0.0f)) return fail(ctx, GBL_EINVAL, "gb_flow_adam: step < 1 or bad learning rate%s");
  if (!fl->adam_m || !fl->adam_v || !fl->grad) return fail(ctx, GBL_EINVAL, "gb_flow_adam: null pointer%s");
  const int64_t n = flow_n_params(cfg);
  const double bc1 = 1.0 - std::pow(0.9, (double)step);
  const double bc2 = 1.0 - std::pow(0.999, (double)step);
  hipLaunchKernelGGL(gbl::flow::k_flow_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream,
                     fl->params, fl->adam_m, fl->adam_v, (const float*)fl->grad, n, bc1, bc2, lr);
  rc = check_launch(ctx, "gb_flow_adam");
  if (rc) return rc;
  return gb_flow_pack(ctx, cfg, fl);
}

extern "C" int gb_flow_train_step(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* fl, const double* u,
                                  const int32_t* band, int64_t B, int64_t step, float lr) {
  int rc = gb_flow_grad(ctx, cfg, fl, u, band, B);
  if (rc) return rc;
  return gb_flow_adam(ctx, cfg, fl, step, lr);
}

// ---------------------------------------------------------------------------
// flow as the RJ proposal of the sweep
// ---------------------------------------------------------------------------
static int rj_prepare(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                      const gbl_flow_config* fcfg, const gbl_flow* fl) {
  int rc = flow_check(ctx, fcfg, fl);
  if (rc) return rc;
  if (!st->prop_u || !st->rj_logq) return fail(ctx, GBL_EINVAL, "gb_sweep_rj_prepare: prop_u / rj_logq not set%s");
  const int32_t band_w = cfg->band_width > 0 ? cfg->band_width : cfg->N;
  if (fcfg->n_emb != cfg->n_bands || fcfg->width != band_w || fcfg->k_band0 != cfg->k_band0)
    return fail(ctx, GBL_EINVAL, "gb_sweep_rj_prepare: flow box differs from the sweep's sub-bands%s");
  const int dims[4] = {0, 2, 4, 7};
  for (int i : dims)
    if (fcfg->prior_lo[i] != cfg->prior_lo[i] || fcfg->prior_hi[i] != cfg->prior_hi[i])
      return fail(ctx, GBL_EINVAL, "gb_sweep_rj_prepare: flow box differs from the sweep's prior%s");
  if (!st->rj_mode) return fail(ctx, GBL_EINVAL, "gb_sweep_rj_prepare: rj_mode workspace not set%s");
  const double w = fcfg->prior_weight;
  if (!(w >= 0.0 && w <= 1.0)) return fail(ctx, GBL_EINVAL, "gb_sweep_rj_prepare: prior_weight outside [0, 1]%s");
  const gbl::SweepArgs a = sweep_args(cfg, st);
  const int64_t n = (int64_t)cfg->n_temps * cfg->n_walkers * cfg->n_bands * cfg->n_slots;
  const dim3 g1((unsigned)((n + 255) / 256)), b1(256);
  switch (cfg->N) {
    case 128: hipLaunchKernelGGL(gbl::k_rj_draw<128>, g1, b1, 0, ctx->stream, ctx->geo, a, w, st->prop_u, st->rj_mode); break;
    case 256: hipLaunchKernelGGL(gbl::k_rj_draw<256>, g1, b1, 0, ctx->stream, ctx->geo, a, w, st->prop_u, st->rj_mode); break;
    default: hipLaunchKernelGGL(gbl::k_rj_draw<512>, g1, b1, 0, ctx->stream, ctx->geo, a, w, st->prop_u, st->rj_mode); break;
  }
  gbl::flow::FlowArgs fa = flow_args(ctx, fcfg, fl);
  fa.band_div = cfg->n_slots;
  fa.band_mod = cfg->n_bands;
  fa.mask = st->rj_mode;
  fa.mask_want = 1;  // flow candidates: normals -> samples, in place
  hipLaunchKernelGGL(gbl::flow::k_flow_apply<true>, dim3(flow_grid(ctx, n)), dim3(256), 0, ctx->stream, fa,
                     (const double*)st->prop_u, (const int32_t*)nullptr, n, st->prop_u, st->rj_logq);
  fa.mask_want = 0;  // occupied slots: flow density at the current source
  hipLaunchKernelGGL(gbl::flow::k_flow_apply<false>, dim3(flow_grid(ctx, n)), dim3(256), 0, ctx->stream, fa,
                     (const double*)st->u, (const int32_t*)nullptr, n, (double*)nullptr, st->rj_logq);
  fa.mask_want = 2;  // prior candidates: flow density at the candidate
  hipLaunchKernelGGL(gbl::flow::k_flow_apply<false>, dim3(flow_grid(ctx, n)), dim3(256), 0, ctx->stream, fa,
                     (const double*)st->prop_u, (const int32_t*)nullptr, n, (double*)nullptr, st->rj_logq);
  switch (cfg->N) {
    case 128: hipLaunchKernelGGL(gbl::k_rj_mix<128>, g1, b1, 0, ctx->stream, ctx->geo, a, w, st->rj_logq); break;
    case 256: hipLaunchKernelGGL(gbl::k_rj_mix<256>, g1, b1, 0, ctx->stream, ctx->geo, a, w, st->rj_logq); break;
    default: hipLaunchKernelGGL(gbl::k_rj_mix<512>, g1, b1, 0, ctx->stream, ctx->geo, a, w, st->rj_logq); break;
  }
  return check_launch(ctx, "gb_sweep_rj_prepare");
}

extern "C" int gb_sweep_rj_prepare(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                                   const gbl_flow_config* fcfg, const gbl_flow* fl) {
  if (!ctx) return GBL_EINVAL;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  return rj_prepare(ctx, cfg, st, fcfg, fl);
}

extern "C" int gb_sweep_run_flow(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                                 const gbl_flow_config* fcfg, const gbl_flow* fl, int32_t n_sweeps) {
  if (!ctx) return GBL_EINVAL;
  int rc = sweep_check(ctx, cfg, st);
  if (rc) return rc;
  if (n_sweeps < 0) return fail(ctx, GBL_EINVAL, "gb_sweep_run_flow: n_sweeps < 0%s");
  rc = flow_check(ctx, fcfg, fl);
  if (rc) return rc;
  return sweep_run_impl(ctx, cfg, st, fcfg, fl, n_sweeps);
}

extern "C" int gb_sweep_graph_create_flow(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                                          const gbl_flow_config* fcfg, const gbl_flow* fl, int32_t n_sweeps,
                                          gbl_graph** out) {
  if (!ctx || !out) return GBL_EINVAL;
  int rc = flow_check(ctx, fcfg, fl);
  if (rc) return rc;
  return graph_create_impl(ctx, cfg, st, fcfg, fl, n_sweeps, out);
}

// ---------------------------------------------------------------------------
// launch-shape knobs
// ---------------------------------------------------------------------------
extern "C" int gbl_get_tuning(const gbl_ctx* ctx, gbl_tuning* out) {
  if (!ctx || !out) return GBL_EINVAL;
  *out = ctx->tune;
  return GBL_OK;
}

extern "C" int gbl_set_tuning(gbl_ctx* ctx, const gbl_tuning* t) {
  if (!ctx) return GBL_EINVAL;
  if (!t) return fail(ctx, GBL_EINVAL, "gbl_set_tuning: null tuning%s");
  const bool pow2 = t->bucket_chunk > 0 && (t->bucket_chunk & (t->bucket_chunk - 1)) == 0;
  if (t->flow_grid < 64 || t->flow_grid > 65536 || !pow2 ||
      t->bucket_chunk < 4096 || t->bucket_chunk > kBucketCap || (t->widest_first != 0 && t->widest_first != 1) ||
      (t->exact_grids != 0 && t->exact_grids != 1))
    return fail(ctx, GBL_EINVAL, "gbl_set_tuning: knob out of range%s");
  ctx->tune = *t;
  return GBL_OK;
}

// ---------------------------------------------------------------------------
// noise-PSD step
// ---------------------------------------------------------------------------
extern "C" int gb_psd_sweep_step(gbl_ctx* ctx, const gbl_psd_sweep_config* c, const gbl_psd_sweep_state* st) {
  if (!ctx) return GBL_EINVAL;
  if (!c || !st) return fail(ctx, GBL_EINVAL, "gb_psd_sweep_step: null config or state%s");
  if (c->n_tn < 1 || c->n_walkers < 2 || c->n_walkers % 2 || !(c->stretch_a > 1.0) ||
      (c->n_par != 4 && c->n_par != 9))
    return fail(ctx, GBL_EINVAL, "gb_psd_sweep_step: configuration out of range%s");
  for (int k = 0; k < c->n_par; k++)
    if (!(c->prior_lo[k] < c->prior_hi[k])) return fail(ctx, GBL_EINVAL, "gb_psd_sweep_step: empty prior box%s");
  if (!st->theta || !st->logl || !st->betas || !st->data || !st->resid || !st->full_resid || !st->inv_psd ||
      !st->work || !st->res_idx || !st->stats || !st->sweep_counter)
    return fail(ctx, GBL_EINVAL, "gb_psd_sweep_step: null state pointer%s");
  const int nt = c->n_tn, nw = c->n_walkers, half = nw / 2;
  const int64_t nb = ctx->geo.n_bins;
  gbl::PsdArgs p;
  p.nt = nt;
  p.nw = nw;
  p.np = c->n_par;
  p.a = c->stretch_a;
  p.seed = c->seed;
  for (int k = 0; k < c->n_par; k++) {
    p.lo[k] = c->prior_lo[k];
    p.hi[k] = c->prior_hi[k];
  }
  p.theta = st->theta;
  p.logl = st->logl;
  p.betas = st->betas;
  p.sweep_ctr = st->sweep_counter;
  p.stats = (unsigned long long*)st->stats;
  cd* full = (cd*)st->full_resid;
  // 1. full residuals, 2. current log-likelihoods
  hipLaunchKernelGGL(gbl::k_psd_full_resid, gbl::row_grid(nb, 2 * (int64_t)nw), dim3(256), 0, ctx->stream, nb, nw,
                     (const cd*)st->resid, (const cd*)st->data, full);
  const int n_all = nt * nw, n_half = nt * half;
  hipLaunchKernelGGL(gbl::k_psd_res_idx, dim3((n_all + 255) / 256), dim3(256), 0, ctx->stream, nt, nw, -1,
                     st->res_idx);
  psd_loglike_launch(ctx, full, nw, st->theta, p.np, st->res_idx, n_all, st->logl, nullptr, nt);
  // 3. stretch moves, half by half
  double* prop = st->work;
  double* lprop = prop + (int64_t)p.np * n_half;
  double* lz = lprop + n_half;
  double* ok = lz + n_half;
  for (int h = 0; h < 2; h++) {
    hipLaunchKernelGGL(gbl::k_psd_propose, dim3((n_half + 255) / 256), dim3(256), 0, ctx->stream, p, h, prop, lz, ok);
    hipLaunchKernelGGL(gbl::k_psd_res_idx, dim3((n_half + 255) / 256), dim3(256), 0, ctx->stream, nt, nw, h,
                       st->res_idx);
    psd_loglike_launch(ctx, full, nw, prop, p.np, st->res_idx, n_half, lprop, nullptr, nt);
    hipLaunchKernelGGL(gbl::k_psd_accept, dim3((n_half + 255) / 256), dim3(256), 0, ctx->stream, p, h,
                       (const double*)prop, (const double*)lprop, (const double*)lz, (const double*)ok);
  }
  // 4. vertical swaps, 5. the cold chain's 1/S
  hipLaunchKernelGGL(gbl::k_psd_swap, dim3((nw + 63) / 64), dim3(64), 0, ctx->stream, p);
  psd_eval_launch(ctx, st->theta, p.np, (int64_t)nw, 1, st->inv_psd);
  return check_launch(ctx, "gb_psd_sweep_step");
}

// ---------------------------------------------------------------------------
// general capture of the context's stream
// ---------------------------------------------------------------------------
extern "C" int gb_graph_begin(gbl_ctx* ctx) {
  if (!ctx) return GBL_EINVAL;
  if (!ctx->stream) return fail(ctx, GBL_EINVAL, "gb_graph_begin: capture needs a non-default stream%s");
  if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(ctx, GBL_EHIP, "gb_graph_begin: begin capture failed%s");
  return GBL_OK;
}

extern "C" int gb_graph_end(gbl_ctx* ctx, gbl_graph** out) {
  if (!ctx || !out) return GBL_EINVAL;
  *out = nullptr;
  gbl_graph* gr = new gbl_graph();
  gr->stream = ctx->stream;
  if (hipStreamEndCapture(ctx->stream, &gr->graph) != hipSuccess) {
    delete gr;
    return fail(ctx, GBL_EHIP, "gb_graph_end: end capture failed%s");
  }
  if (hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(gr->graph);
    delete gr;
    return fail(ctx, GBL_EHIP, "gb_graph_end: instantiate failed%s");
  }
  *out = gr;
  return GBL_OK;
}

// ---------------------------------------------------------------------------
// per-sub-band source search (appendix on fitting proposal distributions)
// ---------------------------------------------------------------------------
static int64_t search_chains(const gbl_search_config* c) {
  return (int64_t)c->n_bands * c->n_temps * c->n_walkers;
}

extern "C" int gb_search_workspace(const gbl_search_config* c, int64_t* bytes) {
  if (!c || !bytes) return GBL_EINVAL;
  *bytes = search_chains(c) * (26 * (int64_t)sizeof(double) + 2 * (int64_t)sizeof(int32_t));
  return GBL_OK;
}

static int search_check(gbl_ctx* ctx, const gbl_search_config* c, const gbl_search_state* st, const double* residual,
                        const double* psd) {
  if (!c || !st) return fail(ctx, GBL_EINVAL, "search: null config or state%s");
  if (c->n_bands < 1 || c->n_temps < 1 || c->n_walkers < 2 || c->n_walkers % 2 || c->width < 1 ||
      c->n_stall < 1 || !(c->stretch_a > 1.0))
    return fail(ctx, GBL_EINVAL, "search: configuration out of range%s");
  if (width_slot(c->N) < 0) return fail(ctx, GBL_EUNSUPPORTED, "search: unsupported N%s");
  if (!st->u || !st->logl || !st->betas || !st->best_u || !st->best_logl || !st->stall || !st->stats ||
      !st->workspace || !residual || !psd)
    return fail(ctx, GBL_EINVAL, "search: null pointer%s");
  if (ctx->cfg.precision != GBL_FP64) return fail(ctx, GBL_EUNSUPPORTED, "search: FP64 contexts only%s");
  return GBL_OK;
}

static gbl::SearchArgs search_args(const gbl_search_config* c, const gbl_search_state* st) {
  gbl::SearchArgs a;
  a.n_b = c->n_bands;
  a.n_t = c->n_temps;
  a.n_w = c->n_walkers;
  a.width = c->width;
  a.n_stall = c->n_stall;
  a.k_band0 = c->k_band0;
  a.stretch_a = c->stretch_a;
  a.seed = c->seed;
  for (int k = 0; k < 8; k++) {
    a.lo[k] = c->prior_lo[k];
    a.hi[k] = c->prior_hi[k];
  }
  a.u = st->u;
  a.logl = st->logl;
  a.betas = st->betas;
  a.best_u = st->best_u;
  a.best_logl = st->best_logl;
  a.stall = st->stall;
  a.stats = (unsigned long long*)st->stats;
  const int64_t n = search_chains(c);
  double* w = (double*)st->workspace;
  a.wu = w;
  a.wpn = w + 8 * n;
  a.wpo = w + 16 * n;
  a.wl = w + 24 * n;
  a.wlz = w + 25 * n;
  a.wok = (int32_t*)(w + 26 * n);
  a.widx = a.wok + n;
  return a;
}

static unsigned grid_of(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

extern "C" int gb_search_eval(gbl_ctx* ctx, const gbl_search_config* cfg, const gbl_search_state* st,
                              const double* residual, const double* psd) {
  if (!ctx) return GBL_EINVAL;
  int rc = search_check(ctx, cfg, st, residual, psd);
  if (rc) return rc;
  const gbl::SearchArgs a = search_args(cfg, st);
  const int64_t n = search_chains(cfg);
  hipLaunchKernelGGL(gbl::k_search_params, dim3(grid_of(n, 256)), dim3(256), 0, ctx->stream, a);
  rc = gb_delta_loglike(ctx, residual, 1, psd, 1, 0, a.wpo, a.wpn, cfg->N, a.widx, a.widx, n, st->logl);
  if (rc) return rc;
  return check_launch(ctx, "gb_search_eval");
}

extern "C" int gb_search_step(gbl_ctx* ctx, const gbl_search_config* cfg, const gbl_search_state* st, int64_t iter,
                              const double* residual, const double* psd) {
  if (!ctx) return GBL_EINVAL;
  int rc = search_check(ctx, cfg, st, residual, psd);
  if (rc) return rc;
  const gbl::SearchArgs a = search_args(cfg, st);
  const int64_t n_half = (int64_t)cfg->n_bands * cfg->n_temps * (cfg->n_walkers / 2);
  for (int h = 0; h < 2; h++) {
    hipLaunchKernelGGL(gbl::k_search_propose, dim3(grid_of(n_half, 256)), dim3(256), 0, ctx->stream, ctx->geo, a,
                       iter, h);
    rc = gb_delta_loglike(ctx, residual, 1, psd, 1, 0, a.wpo, a.wpn, cfg->N, a.widx, a.widx, n_half, a.wl);
    if (rc) return rc;
    hipLaunchKernelGGL(gbl::k_search_accept, dim3(grid_of(n_half, 256)), dim3(256), 0, ctx->stream, a, iter, h);
  }
  hipLaunchKernelGGL(gbl::k_search_swap, dim3(grid_of((int64_t)cfg->n_bands * cfg->n_walkers, 256)), dim3(256), 0,
                     ctx->stream, a, iter);
  hipLaunchKernelGGL(gbl::k_search_best, dim3(grid_of(cfg->n_bands, 64)), dim3(64), 0, ctx->stream, a);
  return check_launch(ctx, "gb_search_step");
}

extern "C" int gb_search_ball(gbl_ctx* ctx, const gbl_search_config* cfg, const gbl_search_state* st, int64_t iter,
                              const double* sigma, const double* residual, const double* psd) {
  if (!ctx) return GBL_EINVAL;
  int rc = search_check(ctx, cfg, st, residual, psd);
  if (rc) return rc;
  if (!sigma) return fail(ctx, GBL_EINVAL, "gb_search_ball: null sigma%s");
  gbl::Sigma8 sg;
  for (int k = 0; k < 8; k++) sg.v[k] = sigma[k];
  const gbl::SearchArgs a = search_args(cfg, st);
  const int64_t n = search_chains(cfg);
  hipLaunchKernelGGL(gbl::k_search_ball, dim3(grid_of(n, 256)), dim3(256), 0, ctx->stream, ctx->geo, a, iter, sg);
  rc = gb_delta_loglike(ctx, residual, 1, psd, 1, 0, a.wpo, a.wpn, cfg->N, a.widx, a.widx, n, st->logl);
  if (rc) return rc;
  return check_launch(ctx, "gb_search_ball");
}

// ---------------------------------------------------------------------------
// correlated A/E channels (Sec. 2): noise matrix and matrix-weighted likelihoods
// ---------------------------------------------------------------------------
extern "C" int gb_noise_matrix(gbl_ctx* ctx, const double* levels, int64_t P, double* out) {
  if (!ctx) return GBL_EINVAL;
  if (P < 0) return fail(ctx, GBL_EINVAL, "gb_noise_matrix: P < 0%s");
  if (P == 0) return GBL_OK;
  if (!levels || !out) return fail(ctx, GBL_EINVAL, "gb_noise_matrix: null pointer%s");
  hipLaunchKernelGGL(gbl::k_noise_matrix, gbl::row_grid(ctx->geo.n_bins, P), dim3(256), 0, ctx->stream,
                     ctx->geo.n_bins, ctx->geo.k_min, ctx->cfg.T, ctx->cfg.L, (const gbl::NoiseLevels*)levels, P,
                     out);
  return check_launch(ctx, "gb_noise_matrix");
}

template <int N>
struct LaunchDeltaMat {
  static void run(gbl_ctx* ctx, const cd* residual, int n_res, const double* K, int n_K, const double* po,
                  const double* pn, const int32_t* ri, const int32_t* ki, int64_t b0, int64_t nb, double* out) {
    hipLaunchKernelGGL((gbl::k_delta_loglike_mat<N>), dim3((unsigned)nb), dim3(gbl::block_threads<N>()), 0,
                       ctx->stream, ctx->geo, tables_for<N, double>(ctx), residual, n_res, K, n_K, po, pn, ri, ki,
                       b0, out);
  }
};

extern "C" int gb_delta_loglike_matrix(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* K,
                                       int32_t n_K, const double* params_old, const double* params_new, int32_t N,
                                       const int32_t* res_idx, const int32_t* k_idx, int64_t B, double* dlogl) {
  if (!ctx) return GBL_EINVAL;
  if (B < 0 || n_res < 1 || n_K < 1) return fail(ctx, GBL_EINVAL, "gb_delta_loglike_matrix: bad sizes%s");
  if (width_slot(N) < 0) return fail(ctx, GBL_EUNSUPPORTED, "gb_delta_loglike_matrix: unsupported N%s");
  if (B == 0) return GBL_OK;
  if (!residual || !K || !params_old || !params_new || !res_idx || !k_idx || !dlogl)
    return fail(ctx, GBL_EINVAL, "gb_delta_loglike_matrix: null pointer%s");
  for (int64_t b0 = 0; b0 < B; b0 += kMaxGrid) {
    const int64_t nb = B - b0 < kMaxGrid ? B - b0 : kMaxGrid;
    dispatch_width<LaunchDeltaMat>(N, ctx, (const cd*)residual, (int)n_res, K, (int)n_K, params_old, params_new,
                                   res_idx, k_idx, b0, nb, dlogl);
  }
  return check_launch(ctx, "gb_delta_loglike_matrix");
}

extern "C" int gb_loglike_matrix(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* K, int32_t n_K,
                                 const int32_t* res_idx, const int32_t* k_idx, int64_t P, double* logl) {
  if (!ctx) return GBL_EINVAL;
  if (P < 0 || n_res < 1 || n_K < 1) return fail(ctx, GBL_EINVAL, "gb_loglike_matrix: bad sizes%s");
  if (P == 0) return GBL_OK;
  if (!residual || !K || !res_idx || !k_idx || !logl) return fail(ctx, GBL_EINVAL, "gb_loglike_matrix: null pointer%s");
  for (int64_t p0 = 0; p0 < P; p0 += kPsdBatch) {
    const int64_t np = P - p0 < kPsdBatch ? P - p0 : kPsdBatch;
    hipLaunchKernelGGL(gbl::k_loglike_mat_partial, dim3(gbl::kPsdChunks, (unsigned)np), dim3(gbl::kPsdBlock), 0,
                       ctx->stream, ctx->geo.n_bins, (const cd*)residual, (int)n_res, K, (int)n_K, res_idx, k_idx, p0,
                       ctx->psd_work);
    hipLaunchKernelGGL(gbl::k_psd_final, dim3((unsigned)np), dim3(64), 0, ctx->stream, 1.0 / ctx->cfg.T,
                       ctx->psd_work, p0, logl);
  }
  return check_launch(ctx, "gb_loglike_matrix");
}
