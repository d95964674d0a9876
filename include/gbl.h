/*
 * gbl.h -- C ABI of the MI355X (gfx950) Galactic-Binary likelihood library.
 *
 * The library computes, on one GPU, the data-parallel hot path of the LISA
 * global-fit GB sampler of arXiv:2405.04690:
 *   - heterodyned, frequency-domain GB templates (A/E/T band slices) for a
 *     rigid equal-arm constellation with first-generation Michelson TDI
 *     (Sec. 2, "Input Template Models" and appendix "GB Waveform Generation";
 *     the TDI channels A, E, T of Sec. 2);
 *   - noise-weighted likelihood changes for swapping, adding or removing one
 *     source (Sec. 2, eqs. addsource and swapsource, with the inner product of
 *     eq. inner summed over channels A and E);
 *   - the log-likelihood of the instrument-noise parameters (Sec. 2 eq. like
 *     with Sec. 3 eq. psd).
 *
 * Conventions shared by every call
 *   Pointers   All array arguments are DEVICE pointers owned by the caller
 *              (e.g. PyTorch allocations on the same GPU).  The library
 *              allocates device memory only inside gbl_create (constant tables,
 *              PSD basis, reduction workspace, and a 111 MB workspace for the
 *              decoded sources of up to 2^17 likelihood pairs, through which
 *              longer batches pass in chunks) and frees it in gbl_destroy.
 *   Streams    Compute calls only enqueue work on the context's stream and
 *              return; outputs are valid once the caller synchronises that
 *              stream.  Compute calls never allocate, synchronise or print
 *              (so they can be captured into graphs), unless the caller opts
 *              into the exact_grids knob (gbl_tuning): then the
 *              width-bucketed calls and the FP64 re-evaluation pass of
 *              GBL_MIXED read device-side list lengths back to size their
 *              launches, outside stream capture only.
 *   Errors     Calls return GBL_OK (0) or a negative status.  Argument errors
 *              are detected on the host before anything is launched;
 *              gbl_last_error() returns a message for the last failure.
 *   Values     Non-finite template parameters give NaN outputs (not an error).
 *              Template bins outside the analysis band [k_min, k_min+n_bins)
 *              are clipped: they contribute zero to every sum.
 *   Threading  A context is not thread-safe; use one context per host thread.
 *   Complex    Complex values are interleaved (re, im) doubles.
 *
 * Units and parameters
 *   params[b][8] = (A, f0 [Hz], fdot [Hz/s], phi0, iota, psi, lambda, beta):
 *   strain amplitude, initial frequency and its derivative, initial phase,
 *   inclination, polarisation angle, ecliptic longitude and latitude.
 *   Frequency bin k is f_k = k / T; the analysis band is
 *   k in [ceil(f_lo T), floor(f_hi T)].
 *   A template of width N has carrier bin q = floor(f0 T); its bin j
 *   (0 <= j < N) is global bin start_bin + j with start_bin = q - N/2.
 *   Supported widths: N in {128, 256, 512, 1024}.
 *
 * Array layouts (row-major)
 *   residual  [n_res][2][n_bins] complex  channel 0 = A, 1 = E; index k - k_min
 *   psd       [n_psd][2][n_bins] double   S_n (or 1/S_n with GBL_PSD_INVERSE)
 *   noise     [P][4] double  (sqrt S_oms^A, sqrt S_acc^A, sqrt S_oms^E, sqrt S_acc^E)
 *             in m/sqrt(Hz) and m s^-2/sqrt(Hz); with the Galactic foreground
 *             (the *_n calls with n_par = 9) [P][9]: those four followed by
 *             (A_fg, alpha, f_k [Hz], s1, s2) of Sec. 3 "Galactic foreground
 *             noise parameterization"
 */
#ifndef GBL_H
#define GBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GBL_OK 0
#define GBL_EINVAL (-1)       /* null pointer, negative size, index out of range, bad flag */
#define GBL_EUNSUPPORTED (-2) /* template width or configuration not supported */
#define GBL_EHIP (-3)         /* HIP runtime or launch error */

/* precision modes */
#define GBL_FP64 0  /* everything in double precision */
#define GBL_MIXED 1 /* orbital and carrier phases, their reduction and all
                       likelihood sums in double; link amplitudes, the TDI
                       response, the FFT and the per-bin factor in float */

/* config flags.  In a GBL_MIXED context gb_delta_loglike(_var) estimates the
 * FP32 error of every pair (20 * 2^-24 times the largest of <a|a>, <r|r>,
 * |<R|a>|, |<R|r>|) and re-evaluates the pairs whose estimate exceeds 5e-4 in
 * FP64 in a second pass, so every result stays within 1e-3 of the FP64 path;
 * GBL_MIXED_UNROUTED skips that pass (pure FP32 response). */
#define GBL_MIXED_UNROUTED 1
/* GBL_DETERMINISTIC: gb_scatter_add sums overlapping templates in a fixed
 * order (sorted by residual, start bin, then template index; no atomics), so
 * its result does not depend on scheduling.  Costs a 128 MB workspace
 * allocated by gbl_create and a sort per chunk of 2^22 / N templates. */
#define GBL_DETERMINISTIC 2

/* psd flags */
#define GBL_PSD_INVERSE 1 /* the psd array holds 1/S_n instead of S_n */

typedef struct gbl_ctx gbl_ctx;

typedef struct {
  double T;          /* observation time [s] */
  double dt;         /* sampling cadence [s]; sets the Nyquist limit 1/(2 dt) */
  double L;          /* arm length [m] */
  double f_lo;       /* analysis band [Hz] */
  double f_hi;
  int32_t precision; /* GBL_FP64 or GBL_MIXED */
  int32_t flags;     /* 0 or GBL_DETERMINISTIC, plus GBL_MIXED_UNROUTED with GBL_MIXED */
} gbl_config;

/* Create a context for one configuration on the current HIP device.
 * hip_stream: a hipStream_t (NULL = the default stream).  Builds the orbit,
 * twiddle and per-bin tables for every supported N, the PSD basis over the
 * band and the reduction workspace.  Errors: GBL_EINVAL for a null ctx/cfg,
 * non-positive T/dt/L, f_lo <= 0, f_hi <= f_lo or f_hi above Nyquist;
 * GBL_EUNSUPPORTED for an unknown precision; GBL_EHIP on allocation failure.
 * On failure *ctx is NULL. */
int gbl_create(gbl_ctx** ctx, const gbl_config* cfg, void* hip_stream);

/* Release everything gbl_create allocated.  Synchronises the context's stream
 * first.  A NULL ctx is a no-op. */
int gbl_destroy(gbl_ctx* ctx);

/* Change the stream later calls enqueue on. */
int gbl_set_stream(gbl_ctx* ctx, void* hip_stream);

/* Message for the last failed call on this context ("" if none). */
const char* gbl_last_error(const gbl_ctx* ctx);

/* First bin and number of bins of the analysis band. */
int gbl_band(const gbl_ctx* ctx, int64_t* k_min, int64_t* n_bins);

/* Launch-shape knobs of a context (set by the autotuner, paper_2405_04690_amd/autotune.py):
 *   flow_grid     maximum work-groups of a flow inference launch, in [64, 65536]
 *                 (default 4096);
 *   bucket_chunk  templates per bucketed launch group (uneven widths; the FP64
 *                 re-evaluation of mixed-precision pairs), a
 *                 power of two in [4096, 1048576] (default 1048576); likelihood
 *                 calls use at most 2^17 pairs per group (the decode workspace);
 *   widest_first  uneven widths: launch the widest bucket first (1) or last (0);
 *   exact_grids   0 (default): never synchronise; the bucketed launches and
 *                 the FP64 re-evaluation pass of GBL_MIXED use the upper bound
 *                 (the batch size) as grid and the surplus work-groups exit;
 *                 1: when the context's stream is not being captured,
 *                 gb_waveform_var, gb_delta_loglike_var and that pass copy the
 *                 device-side bucket sizes (and routed-pair counts) to pinned
 *                 host memory, one stream synchronisation each, and launch
 *                 exactly that many work-groups.  Under capture the upper
 *                 bound is always used.
 * Results do not depend on them (bitwise for the FP64 paths). */
typedef struct {
  int32_t flow_grid;
  int32_t bucket_chunk;
  int32_t widest_first;
  int32_t exact_grids;
} gbl_tuning;

int gbl_get_tuning(const gbl_ctx* ctx, gbl_tuning* out);
int gbl_set_tuning(gbl_ctx* ctx, const gbl_tuning* tuning);  /* GBL_EINVAL if a knob is out of range */

/* Heterodyned GB templates (Sec. 2 and appendix "GB Waveform Generation";
 * the response is the rigid equal-arm, first-generation-TDI reading described
 * in the library's design notes).  For every template b writes
 *   A[b][N], E[b][N], Tch[b][N]  complex band slices of the TDI channels,
 *   start_bin[b]                 global bin of slice element 0.
 * T and dt must equal the context's (they are part of the problem statement
 * and checked).  Tch may be NULL (the T channel is then not computed).
 * Errors: GBL_EINVAL (null pointers, B < 0, T/dt mismatch),
 * GBL_EUNSUPPORTED (N not supported). */
int gb_waveform(gbl_ctx* ctx, const double* params, int64_t B, int32_t N, double T, double dt, double* A,
                double* E, double* Tch, int64_t* start_bin);

/* Likelihood change for swapping one source (Sec. 2 eq. swapsource):
 *   dlogl[b] = -1/2 [<a|a> + <r|r> - 2<a|r> - 2<R|a> + 2<R|r>]
 *            = <R|a - r> - 1/2 <a - r|a - r>         (the form evaluated)
 * with a = template(params_new[b]), r = template(params_old[b]),
 * R = residual[res_idx[b]] (= d - H, H containing r) and the inner product of
 * eq. inner over channels A, E weighted by psd[psd_idx[b]], restricted to the
 * union of the two template windows clipped to the band.  A birth
 * (eq. addsource) has params_old amplitude 0, a death params_new amplitude 0.
 * psd_flags: 0 or GBL_PSD_INVERSE.  All templates have width N.
 * Errors: GBL_EINVAL (null pointers, B < 0, n_res/n_psd < 1, bad flags),
 * GBL_EUNSUPPORTED (N).  Indices res_idx/psd_idx must lie in [0, n_res) and
 * [0, n_psd); they are not checked on the host (they live on the device), and
 * an out-of-range index gives a NaN output for that template, never an
 * out-of-bounds access. */
int gb_delta_loglike(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* psd, int32_t n_psd,
                     int32_t psd_flags, const double* params_old, const double* params_new, int32_t N,
                     const int32_t* res_idx, const int32_t* psd_idx, int64_t B, double* dlogl);

/* Uneven template widths in one call (the paper's sub-band widths depend on
 * frequency, Sec. 4): as gb_waveform, but template b has width N[b] (device
 * array) and its slices start at element out_offset[b] (device array, in
 * complex elements) of A, E and Tch.  Templates are bucketed by width on the
 * device (atomic position counters) and each width runs as one launch over
 * its bucket, sized as the exact_grids knob says.  A template whose N[b] is not
 * supported is skipped and gets start_bin[b] = INT64_MIN.  The caller owns the
 * layout: slices of different templates must not overlap.
 * Errors: GBL_EINVAL (null pointers, B < 0). */
int gb_waveform_var(gbl_ctx* ctx, const double* params, const int32_t* N, const int64_t* out_offset, int64_t B,
                    double* A, double* E, double* Tch, int64_t* start_bin);

/* Uneven template widths in one call: as gb_delta_loglike with the width of
 * pair b given by N[b] (device array; both templates of a pair share it).
 * Bucketed on the device and run as one launch per width.  An unsupported
 * N[b] gives dlogl[b] = NaN.
 * Errors: GBL_EINVAL (null pointers, bad sizes or flags). */
int gb_delta_loglike_var(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* psd, int32_t n_psd,
                         int32_t psd_flags, const double* params_old, const double* params_new, const int32_t* N,
                         const int32_t* res_idx, const int32_t* psd_idx, int64_t B, double* dlogl);

/* Instrument PSD of eq. psd over the band for P noise-parameter sets:
 *   S[p][c][k - k_min] = S_n(f_k; sqrt S_oms^c, sqrt S_acc^c), c = A, E
 * (or 1/S_n with GBL_PSD_INVERSE).  Errors: GBL_EINVAL. */
int gb_psd_eval(gbl_ctx* ctx, const double* noise, int64_t P, int32_t psd_flags, double* S);

/* As gb_psd_eval for noise sets of n_par = 4 or 9 parameters.  With 9, the
 * Galactic foreground of Sec. 3 is added to both channels:
 *   S_fg(f) = 6 x^2 sin^2 x h_fg(f),  x = 2 pi f L / c,
 *   h_fg(f) = 1/2 A_fg f^(-7/3) exp(-s1 f^alpha) [1 + tanh(-s2 (f - f_k))],
 * one foreground (noise[p][4..8]) shared by A and E.  A_fg = 0 gives S_n
 * exactly.  Errors: GBL_EINVAL (n_par not 4 or 9, P < 0, null pointers,
 * unknown flags). */
int gb_psd_eval_n(gbl_ctx* ctx, const double* noise, int32_t n_par, int64_t P, int32_t psd_flags, double* S);

/* Noise-parameter log-likelihood (Sec. 2 eq. like with Sec. 3 eq. psd):
 *   logl[p] = sum_{c in A,E} [ -2 df sum_k |R_c,k|^2 / S_c,k - sum_k ln S_c,k ]
 * with R = residual[res_idx[p]] and S from noise[p].  The sum over bins is a
 * fixed-order two-pass reduction, so results are bitwise reproducible, and a
 * set's result does not depend on P or on the other sets of the call.
 * Errors: GBL_EINVAL.  Out-of-range res_idx gives NaN for that set. */
int gb_psd_loglike(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* noise,
                   const int32_t* res_idx, int64_t P, double* logl);

/* As gb_psd_loglike with noise sets of n_par = 4 or 9 parameters (9: the
 * PSD includes the Galactic foreground as in gb_psd_eval_n; Sec. 4 "Noise
 * and stochastic foreground signal PSD fitting").  Errors: GBL_EINVAL. */
int gb_psd_loglike_n(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* noise, int32_t n_par,
                     const int32_t* res_idx, int64_t P, double* logl);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gb_psd_loglike_n with its partial
 * sums in a static device array of the library instead of the context's
 * workspace.  P <= 2048 parameter sets (the array holds 2048 x 256 x 2
 * doubles, 8 MB per device, kept until the process ends); larger P is
 * rejected with GBL_EINVAL.  Allocates nothing.  Every call on one device
 * shares that device's array: calls that overlap on one device (several
 * streams or contexts) race and must be serialised by the caller.  Results
 * equal gb_psd_loglike_n's (same kernels, same summation order). */
int gb_psd_loglike_noalloc(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* noise,
                           int32_t n_par, const int32_t* res_idx, int64_t P, double* logl);

/* residual[res_idx[b]] += sign * (A, E) of template b, clipped to the band
 * (the residual updates of the sampling algorithm's write-back step).  By
 * default FP64 atomic adds, so overlapping templates are summed in an
 * unspecified order; in a GBL_DETERMINISTIC context every bin is written by
 * one thread that adds the templates covering it in (residual, start bin,
 * template index) order, so repeated calls give bitwise equal residuals.
 * Zero-amplitude and undefined templates and out-of-range res_idx add
 * nothing.  Errors: GBL_EINVAL, GBL_EUNSUPPORTED (N). */
int gb_scatter_add(gbl_ctx* ctx, const double* params, int64_t B, int32_t N, double sign, double* residual,
                   int32_t n_res, const int32_t* res_idx);

/* Noise-weighted inner products of stored band slices (Sec. 2 eq. inner,
 * summed over channels A and E):
 *   out[b][0] = <h_b|h_b>,  out[b][1] = <R|h_b>,  R = residual[res_idx[b]],
 * weighted by psd[psd_idx[b]] (S_n, or 1/S_n with GBL_PSD_INVERSE), where
 * h_b = (A[b][j], E[b][j]) sits at global bin start_bin[b] + j, 0 <= j < N
 * (the layout gb_waveform writes), and bins outside the band contribute 0.
 * Any N >= 1.  This is the likelihood stage alone over slices already in
 * memory (bound by HBM bandwidth): 4 dlnL-style terms of eq. swapsource
 * follow from two calls.  Sums in FP64, fixed order (bitwise reproducible).
 * An out-of-range res_idx/psd_idx gives NaN for that template.
 * Errors: GBL_EINVAL (null pointers, B < 0, N < 1, n_res/n_psd < 1, flags). */
int gb_inner(gbl_ctx* ctx, const double* A, const double* E, const int64_t* start_bin, int32_t N,
             const double* residual, int32_t n_res, const double* psd, int32_t n_psd, int32_t psd_flags,
             const int32_t* res_idx, const int32_t* psd_idx, int64_t B, double* out);

/* Overlaps of template pairs (Sec. 4 "Cataloging Operation": sources are
 * grouped by overlap above 0.9):
 *   out[b] = (<a|a>, <b|b>, <a|b>, <a|b> / sqrt(<a|a> <b|b>)),
 * a = width-N template of params_a[b], b of params_b[b], the inner product of
 * eq. inner over A and E weighted by psd[psd_idx[b]] (S_n, or 1/S_n with
 * GBL_PSD_INVERSE), bins outside the band dropped; FP64 response whatever the
 * context's precision.  Undefined parameters or an out-of-range psd_idx give
 * NaN; a zero-amplitude template gives a NaN overlap (0/0).
 * Errors: GBL_EINVAL, GBL_EUNSUPPORTED (N). */
int gb_overlap(gbl_ctx* ctx, const double* params_a, const double* params_b, int32_t N, const double* psd,
               int32_t n_psd, int32_t psd_flags, const int32_t* psd_idx, int64_t B, double* out);

/* Optimal SNR rho_opt = sqrt(<h|h>) and observed SNR <d|h> / sqrt(<h|h>) of
 * width-N templates built from params (Sec. 2: the inner product of eq. inner
 * over A and E, the optimal SNR defined with the likelihood), FP64 response
 * whatever the context's precision.  data (may be NULL: snr_obs is then not
 * written) holds n_data series [n_data][2][n_bins] complex, template b uses
 * data[data_idx[b]] and psd[psd_idx[b]].  A zero-amplitude template gives
 * snr_opt 0 and snr_obs NaN (0/0); undefined parameters or out-of-range
 * indices give NaN.  Errors: GBL_EINVAL (null pointers, sizes, flags),
 * GBL_EUNSUPPORTED (N). */
int gb_snr(gbl_ctx* ctx, const double* params, int64_t B, int32_t N, const double* psd, int32_t n_psd,
           int32_t psd_flags, const int32_t* psd_idx, const double* data, int32_t n_data, const int32_t* data_idx,
           double* snr_opt, double* snr_obs);

/* Stationary Gaussian noise with PSD S (Sec. 3): for n series,
 *   out[i][c][k] = sqrt(S[i][c][k] / (4 df)) * normals[i][c][k]
 * with normals complex standard normal draws supplied by the caller, so that
 * E[<n|n>] = 2 per bin and channel.  Errors: GBL_EINVAL. */
int gb_make_noise(gbl_ctx* ctx, const double* S, const double* normals, int64_t n, double* out);

/* ------------------------------------------------------------------------
 * Sampler sweep (Sec. 4 "Galactic binary search and parameter estimation";
 * appendix algorithms gb1 "Galaxy sampling" and gb2 "Galaxy tempering";
 * eqs. rj-acceptance, stretch, temp-final).
 *
 * Sub-band b covers bins [k_band0 + b N, k_band0 + (b+1) N) (N = template
 * width, 128/256/512); its analysis window is sub-bands b-1..b+1.  A sweep is:
 * stationary-group refresh (every group_every sweeps), in-model group-stretch
 * band loops (odd bands, then even), the reversible-jump pass that flips every
 * slot (odd, even), residual-aware parallel tempering (odd, even), when
 * configured the ladder adaptation and the ownership shift, and
 * sweep_counter += 1.  Bands of one parity run in parallel: they read the
 * opposite-parity cold-chain buffer and write only their own.
 * Sampling coordinates u = (log10 A, f0 [Hz], fdot [Hz/s], phi0, cos iota,
 * psi, lambda, sin beta) with a uniform prior on a box: prior_lo/hi give the
 * bounds of log10 A, fdot, cos iota and sin beta; f0 ranges over the band
 * widened by N/2 per side; phi0, psi, lambda are periodic (2 pi, pi, 2 pi).
 * Random numbers: Philox4x64-10 keyed by seed with counter
 * (sweep, move << 40 | unit, draw / 4, 0).
 * ------------------------------------------------------------------------ */
#define GBL_MOVE_INMODEL 0
#define GBL_MOVE_RJ 1
#define GBL_MOVE_PT 2

typedef struct {
  int32_t n_temps, n_walkers, n_bands, n_slots; /* n_slots <= 64, n_temps and n_walkers <= 256 */
  int32_t N;                                   /* template width: 128, 256, 512 or 1024 */
  int32_t n_prop;                              /* in-model proposals per band per sweep */
  int32_t n_friends;                           /* group-stretch friends */
  int32_t group_every;                         /* stationary-group refresh period (sweeps); 0 = never */
  int64_t k_band0;                             /* first bin of sub-band 0 */
  double stretch_a;                            /* stretch scale a > 1 */
  uint64_t seed;
  double prior_lo[8], prior_hi[8];
  /* After the tempering step of every sweep (0 = off):                      */
  int32_t adapt_ladder;    /* 1: adapt each band's ladder (gb_sweep_adapt_ladder) */
  int32_t shift_ownership; /* 1: move strayed cold-chain sources (gb_sweep_shift_ownership) */
  double adapt_lag;        /* t0 of the adaptation's decay t0 / (t + t0), > 0 when adapting */
  double adapt_time;       /* nu, the adaptation's time scale, > 0 when adapting */
  /* Sub-band width W in bins (even; 0: W = N).  Sub-band b covers bins
   * [k_band0 + bW, k_band0 + (b+1)W); its sources' f0 range over the band
   * widened by W/2 on each side, and its window, [k_band0 + bW - W/2 - N/2,
   * k_band0 + (b+1)W + W/2 + N/2) (2W + N bins), holds every bin one of its
   * templates reaches.  W != N, and N = 1024, need window_sums in the
   * state: the band loops keep their windows there (in LDS otherwise). */
  int32_t band_width;
} gbl_sweep_config;

/* Sampler state: caller-owned device arrays (checkpointable as they are). */
typedef struct {
  double* u;              /* [n_temps][n_walkers][n_bands][n_slots][8] sampling coordinates */
  int32_t* exists;        /* [n_temps][n_walkers][n_bands][n_slots] 0/1 */
  double* betas;          /* [n_bands][n_temps] inverse temperatures, betas[b][0] = 1 */
  double* resid;          /* [2][n_walkers][2][n_bins] complex: parity-p buffer = data minus the
                             cold-chain sources of the bands with b % 2 == p */
  const double* inv_psd;  /* [n_walkers][2][n_bins] 1/S per walker */
  double* group;          /* [n_bands][n_walkers * n_slots][8] stationary groups (sorted by f0) */
  int32_t* group_count;   /* [n_bands] */
  int64_t* stats;         /* [10] in-model proposed/accepted, births, deaths, swaps (proposed/accepted),
                             ownership shifts (moved, no free slot) */
  int64_t* sweep_counter; /* [1] current sweep index */
  /* Optional (NULL = prior RJ proposal, no log-likelihood trace): */
  double* prop_u;         /* [n_t][n_w][n_b][n_slot][8] birth candidates (read for empty slots) */
  double* rj_logq;        /* [n_t][n_w][n_b][n_slot] ln q of the RJ proposal at the candidate
                             (empty slot) or at the current source (occupied slot) */
  double* cold_logl;      /* [n_w][n_b] cold chain's band log-likelihood, written by tempering */
  int32_t* rj_mode;       /* [n_t][n_w][n_b][n_slot] workspace of gb_sweep_rj_prepare */
  /* Optional cache (NULL: everything is recomputed): pool_size entries of
   * max(n_slot x 2N, n_temps x 6N) complex doubles -- the band loops keep the
   * spectra of their slots, the tempering kernel the window sums of its
   * source sets -- and pool_size flags that must be zero before the first
   * call.  A block takes a free entry for its lifetime (bounded scan; without
   * one it recomputes); pool_size >= 1024 covers the blocks one launch keeps
   * resident.  Results do not depend on it beyond FP64 rounding order. */
  double* spec_pool;
  int32_t* pool_flags;
  int32_t pool_size;
  /* Needed with adapt_ladder (else may be NULL): [n_bands][n_temps] accepted
   * swaps of rungs (t-1, t) since the last adaptation (tempering adds to it,
   * the adaptation clears it); must start at zero. */
  int32_t* swap_acc;
  /* Optional (NULL: the tempering pass rebuilds every set's templates;
   * required when band_width != N):
   * [n_temps][n_walkers][n_bands][2][2W + N] complex doubles, the sum of each
   * source set's templates over its band's window (A then E; zero outside the
   * analysis band).  Every band
   * pass (moves 0 and 1) writes the entries of its parity; the tempering pass
   * of that parity reads them instead of rebuilding the templates and moves
   * them with the source sets it swaps, so they stay valid until the sets
   * change.  Write it with a band pass of each parity before the first
   * tempering pass.  Results do not depend on it beyond FP64 rounding order. */
  double* window_sums;
} gbl_sweep_state;

typedef struct gbl_graph gbl_graph;

/* One move type over the bands of one parity, using *sweep_counter for the
 * random streams.  In a GBL_MIXED context the band passes (moves 0 and 1)
 * build their templates with the FP32 response and FFT (source decode,
 * phases, the spectra at the bins, the windows and every likelihood sum stay
 * FP64), so a decision can differ from the FP64 one where the FP32 template
 * error moves the log acceptance ratio across the draw; such a context needs
 * window_sums (the tempering pass then builds no template).  Errors:
 * GBL_EINVAL (null pointers, out-of-range config), GBL_EUNSUPPORTED (a
 * mixed-precision context without window_sums). */
int gb_sweep_step(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st, int32_t move,
                  int32_t parity);

/* Rebuild the stationary groups from the cold chain (t = 0) of every walker. */
int gb_sweep_group(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st);

/* Temperature-ladder adaptation of every band (appendix "Parallel tempering
 * in a residual-based analysis": independent ladders that adapt, after
 * Vousden, Farr & Mandel 2016).  With T = 1/beta and A_j = swap_acc[b][j+1] /
 * n_walkers the accepted fraction of swaps of rungs (j, j+1):
 *   T_(j+1) - T_j <- (T_(j+1) - T_j) exp(kappa (A_j - A_(j+1))),
 *   kappa = adapt_lag / (adapt_time (*sweep_counter + adapt_lag)),
 * for j = 0..n_temps-3; rung 0 (beta = 1) and the hottest rung stay, the
 * others are rung 0's temperature plus the running sum of the gaps.  Clears
 * swap_acc.  Errors: GBL_EINVAL (no swap_acc, adapt_lag or adapt_time <= 0). */
int gb_sweep_adapt_ladder(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st);

/* Sub-band ownership (Sec. 4: samples may move half a band into the
 * neighbours; afterwards a cold-chain sample that lies in a neighbouring band
 * is handed to it): every cold-chain (t = 0) source whose f0 left its band's
 * nominal range [k_band0 + b N, k_band0 + (b+1) N) / T moves to the lowest
 * free cold-chain slot of the neighbouring band it lies in (it stays when
 * there is none, or at the ends of the band range), and the two cold-chain
 * buffers are updated (added back to the old parity's buffer, removed from the
 * new one's).  Per walker, bands and then slots in increasing order.  Counts
 * in stats[8] (moved) and stats[9] (no free slot). */
int gb_sweep_shift_ownership(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st);

/* *sweep_counter += 1 on the device. */
int gb_sweep_advance(gbl_ctx* ctx, const gbl_sweep_state* st);

/* n_sweeps full sweeps (see above), enqueued without any host synchronisation. */
int gb_sweep_run(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st, int32_t n_sweeps);

/* Capture n_sweeps full sweeps into a HIP graph on the context's stream (which
 * must not be the default stream); gb_graph_launch replays it (each replay
 * advances the sweep counter, so replays draw fresh random numbers).
 * The captured launches keep the state pointers given here. */
int gb_sweep_graph_create(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st, int32_t n_sweeps,
                          gbl_graph** graph);
int gb_graph_launch(gbl_graph* graph);
int gb_graph_destroy(gbl_graph* graph);

/* General capture: every library call enqueued on the context's stream
 * (non-default) between gb_graph_begin and gb_graph_end is recorded into one
 * graph, e.g. a sweep with the flow proposal followed by the noise-PSD step.
 * No call in between may synchronise the stream. */
int gb_graph_begin(gbl_ctx* ctx);
int gb_graph_end(gbl_ctx* ctx, gbl_graph** graph);

/* ---------------------------------------------------------------------------
 * Noise-PSD step of the sweep (Sec. 3 eq. psd with Sec. 2 eq. like; Sec. 4:
 * the PSD parameters are sampled with ensemble stretch moves, eq. stretch,
 * and vertical tempering -- chain (t, w) always uses walker w's residual, so a
 * temperature swap is eq. temp-orig).  One call:
 *   1. full residual of walker w = cold-chain buffer 0 + buffer 1 - data;
 *   2. logl of every chain refreshed against it;
 *   3. for half h = 0, 1: every chain (t, w) with w % 2 == h proposes
 *      theta' = theta_j + z (theta - theta_j), j a walker of the other half at
 *      the same temperature, z = ((a-1) u + 1)^2 / a; accepted with
 *      ln alpha = beta_t (L' - L) + (n_par - 1) ln z inside the uniform prior
 *      box (z^(d-1) for the d = n_par dimensional stretch);
 *   4. per walker, swaps from the hottest pair down;
 *   5. inv_psd[w] = 1/S at the cold chain's parameters (foreground included
 *      when n_par = 9).
 * Random numbers: the Philox stream of the sweep (seed, *sweep_counter):
 * stretch unit t n_w + w, move 4, draws 4 h + (0 partner, 1 z, 2 accept);
 * swaps unit w, move 5, draw t.  n_walkers must be even.
 * --------------------------------------------------------------------------- */
typedef struct {
  int32_t n_tn;          /* PSD temperatures */
  int32_t n_walkers;     /* the sweep's walkers */
  int32_t n_par;         /* 4 (instrument noise) or 9 (with the Galactic foreground, Sec. 3) */
  double stretch_a;
  uint64_t seed;
  double prior_lo[9];    /* box of (sqrt S_oms^A, sqrt S_acc^A, sqrt S_oms^E, sqrt S_acc^E[, A_fg, alpha,
                            f_k, s1, s2]); entries past n_par are ignored */
  double prior_hi[9];
} gbl_psd_sweep_config;

typedef struct {
  double* theta;             /* [n_tn][n_w][n_par] */
  double* logl;              /* [n_tn][n_w] */
  const double* betas;       /* [n_tn] */
  const double* data;        /* [2][n_bins] complex: the data d (A, E) */
  const double* resid;       /* the sweep's cold-chain buffers [2][n_w][2][n_bins] complex */
  double* full_resid;        /* workspace [n_w][2][n_bins] complex */
  double* inv_psd;           /* [n_w][2][n_bins], written (the sweep's 1/S) */
  double* work;              /* workspace, 7 n_tn n_w doubles */
  int32_t* res_idx;          /* workspace, n_tn n_w */
  int64_t* stats;            /* [4]: stretch proposed, accepted; swaps proposed, accepted */
  const int64_t* sweep_counter;
} gbl_psd_sweep_state;

int gb_psd_sweep_step(gbl_ctx* ctx, const gbl_psd_sweep_config* cfg, const gbl_psd_sweep_state* st);

/* ---------------------------------------------------------------------------
 * Learned reversible-jump proposal: a conditional affine-coupling flow.
 *
 * The paper fits its RJ proposal distributions with Gaussian mixtures and
 * plans normalizing flows instead (Discussion, "Single source
 * search-to-parameter estimation information transfer"; appendix "Algorithm
 * for fitting proposal distributions"; Sec. 4 "Online updating of RJ sampling
 * distributions" for the online refit).  The flow's form is a reading:
 *   u = (log10 A, f0, fdot, phi0, cos iota, psi, lambda, sin beta) inside the
 *   prior box of sub-band b (f0 in [k_band0 + (b - 1/2) width,
 *   k_band0 + (b + 3/2) width) / T; phi0, lambda in [0, 2 pi); psi in [0, pi);
 *   the other four from prior_lo / prior_hi) maps to x_i = logit of its
 *   position in the box; six affine coupling layers (layer l keeps the
 *   coordinates (0,2,4,6) for even l, (1,3,5,7) for odd l, and moves the rest:
 *   y = x exp(s) + t, s = 2 tanh(s_hat), (s_hat, t) = MLP([x_kept, E[b]]) with
 *   MLP 20 -> 128 -> 128 -> 8 and SiLU, E a learned 16-wide embedding of b);
 *   ln q_u(u) = sum ln N(z_i; 0, 1) + sum of s + sum ln |dx_i/du_i|.
 * Arithmetic: BF16 MFMA inputs (weights, embeddings, activations; round to
 * nearest even), FP32 accumulation, FP64 flow state and log-density sums.
 *
 * Parameter vector (FP32, caller-owned, n_params = 6 * GBL_FLOW_LAYER_PARAMS
 * + 16 * n_emb): for each layer W1 [128][20], b1 [128], W2 [128][128],
 * b2 [128], W3 [8][128], b3 [8] (row-major, output-major), then E [n_emb][16].
 * `packed` holds the BF16 copy in MFMA fragment order (write it with
 * gb_flow_pack after changing params; gb_flow_adam repacks by itself).
 * --------------------------------------------------------------------------- */
#define GBL_FLOW_LAYER_PARAMS 20232

typedef struct {
  int32_t n_emb;       /* number of sub-bands (conditioning values b = 0..n_emb-1) */
  int32_t width;       /* sub-band width in bins */
  int64_t k_band0;     /* first bin of sub-band 0 */
  double prior_lo[8];  /* box bounds of log10 A, fdot, cos iota, sin beta (entries 0, 2, 4, 7) */
  double prior_hi[8];
  double prior_weight; /* RJ proposal = (1 - prior_weight) flow + prior_weight prior, in [0, 1] */
} gbl_flow_config;

typedef struct {
  float* params;     /* [n_params] FP32 master weights */
  float* adam_m;     /* [n_params] Adam first moment */
  float* adam_v;     /* [n_params] Adam second moment */
  float* grad;       /* [n_params] gradient of the last gb_flow_grad */
  void* packed;      /* packed_bytes: BF16 fragments */
  void* workspace;   /* workspace_bytes: partial sums of gb_flow_grad */
  double* loss;      /* [1] mean negative log-density of the last gb_flow_grad */
} gbl_flow;

/* Sizes of the caller-owned flow buffers (host call; no device work). */
int gb_flow_sizes(const gbl_flow_config* cfg, int64_t* n_params, int64_t* packed_bytes, int64_t* workspace_bytes);

/* packed <- BF16(params). */
int gb_flow_pack(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* flow);

/* logq[i] = ln q_u(u[i] | band[i]); u [B][8], band [B] int32.  A point not
 * strictly inside its box or an out-of-range band gives NaN. */
int gb_flow_log_prob(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* flow, const double* u,
                     const int32_t* band, int64_t B, double* logq);

/* Push standard normals z [B][8] through the inverse flow: u [B][8] inside the
 * box of band[i] and logq[i] = ln q_u(u[i] | band[i]) (equal to what
 * gb_flow_log_prob returns at u[i], up to FP64 rounding). */
int gb_flow_sample(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* flow, const double* z,
                   const int32_t* band, int64_t B, double* u, double* logq);

/* Training gradient: flow->grad = d/dparams of -(1/B) sum_i ln q_x(x(u[i]) | band[i])
 * and flow->loss = that mean (B >= 1; points outside their box contribute 0). */
int gb_flow_grad(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* flow, const double* u,
                 const int32_t* band, int64_t B);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias correction with
 * `step` counted from 1) from flow->grad, then repack. */
int gb_flow_adam(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* flow, int64_t step, float lr);

/* gb_flow_grad followed by gb_flow_adam. */
int gb_flow_train_step(gbl_ctx* ctx, const gbl_flow_config* cfg, const gbl_flow* flow, const double* u,
                       const int32_t* band, int64_t B, int64_t step, float lr);

/* RJ with a proposal density q instead of the prior (appendix on the RJ
 * proposal basis: the in-sampler flags and proposal density values are the
 * RJ pass's inputs).  With st->prop_u and st->rj_logq set, a birth in an
 * empty slot proposes prop_u and is accepted with
 *   ln alpha = beta dlnL + ln p(theta) - ln q(theta),
 * a death of an occupied slot with ln alpha = beta dlnL - ln p(theta) +
 * ln q(theta) (p = the uniform prior density of the band's box; a candidate
 * outside the prior, or a NaN ln q, is rejected).
 *
 * gb_sweep_rj_prepare fills prop_u and rj_logq for every slot with the
 * mixture proposal q = (1 - w) q_flow + w p, w = fcfg->prior_weight (as the
 * paper mixes its fitted RJ proposals with prior draws, Sec. 4 "Transition
 * from search to parameter estimation"): from the sweep's Philox stream
 * (unit (t, w, b), move RJ, draws 2048 + 16 s + k) an empty slot takes a
 * prior draw (probability w, uniforms k = 0..7) or 8 Box-Muller normals pushed
 * through the flow of sub-band b; rj_logq is ln q at the candidate (empty
 * slot) or at the current source (occupied slot).  st->rj_mode is its
 * workspace.  fcfg must describe the sweep's own box (n_emb = n_bands,
 * width = N, same k_band0 and prior bounds). */
int gb_sweep_rj_prepare(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                        const gbl_flow_config* fcfg, const gbl_flow* flow);

/* gb_sweep_run / gb_sweep_graph_create with the flow as RJ proposal: every
 * sweep runs gb_sweep_rj_prepare between the in-model and the RJ moves. */
int gb_sweep_run_flow(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                      const gbl_flow_config* fcfg, const gbl_flow* flow, int32_t n_sweeps);
int gb_sweep_graph_create_flow(gbl_ctx* ctx, const gbl_sweep_config* cfg, const gbl_sweep_state* st,
                               const gbl_flow_config* fcfg, const gbl_flow* flow, int32_t n_sweeps,
                               gbl_graph** graph);

/* ---------------------------------------------------------------------------
 * Search for the loudest remaining source in every sub-band (appendix
 * "Algorithm for fitting proposal distributions"; the search RJ proposal of
 * Sec. 4 "Online updating of RJ sampling distributions").  Independent,
 * fixed-dimensional (one source, d = 8), parallel-tempered ensembles, one per
 * sub-band b = [k_band0 + b width, k_band0 + (b+1) width) (f0 confined to it),
 * with the stretch move of eq. stretch and the target
 *   l(u) = <R|h(u)> - 1/2 <h(u)|h(u)>   (eq. addsource; births of the batched
 * likelihood kernels), tempered as beta_t l.  One gb_search_step:
 *   for half h = 0, 1: every chain (b, t, w), w % 2 == h, of a band still
 *     running proposes Y = X_j + z (X_w - X_j), j = 2 floor(U0 n_w/2) + 1 - h
 *     of the same (b, t), z = ((a-1) U1 + 1)^2 / a (periodic phi0, psi,
 *     lambda on their circles; a stretched periodic difference of half a
 *     period or more is rejected), accepted iff ln U2 < beta_t (l' - l) +
 *     7 ln z inside the band's prior box;
 *   swaps per (b, w) from the hottest pair down (eq. temp-orig);
 *   the best cold-chain point: best_logl[b], best_u[b] take the first maximum
 *     over the cold walkers when it improves, else stall[b] += 1; a band whose
 *     stall reaches n_stall has converged and no longer moves.
 * Random numbers: stretch unit (b n_t + t) n_w + w, move 6, draws 4 h + k;
 * swaps unit b n_w + w, move 7, draw t; the restart ball move 8.  The
 * iteration index `iter` is the Philox stream's first counter word.
 * --------------------------------------------------------------------------- */
typedef struct {
  int32_t n_bands, n_temps, n_walkers; /* n_walkers even */
  int32_t N;                           /* template width */
  int32_t width;                       /* sub-band width in bins */
  int32_t n_stall;                     /* converged after this many iterations without improvement */
  int64_t k_band0;                     /* first bin of sub-band 0 */
  double stretch_a;
  uint64_t seed;
  double prior_lo[8], prior_hi[8];     /* box of log10 A, fdot, cos iota, sin beta (entries 0, 2, 4, 7) */
} gbl_search_config;

typedef struct {
  double* u;            /* [n_b][n_t][n_w][8] sampling coordinates */
  double* logl;         /* [n_b][n_t][n_w] */
  const double* betas;  /* [n_t], betas[0] = 1 */
  double* best_u;       /* [n_b][8] */
  double* best_logl;    /* [n_b], start at -inf */
  int32_t* stall;       /* [n_b], start at 0 */
  int64_t* stats;       /* [4]: proposed, accepted, swaps proposed, accepted */
  void* workspace;      /* gb_search_workspace bytes */
} gbl_search_state;

/* Bytes of the search workspace (host call). */
int gb_search_workspace(const gbl_search_config* cfg, int64_t* bytes);

/* logl of every chain at its current point.  residual [2][n_bins] complex
 * (one series), psd [2][n_bins] S_n. */
int gb_search_eval(gbl_ctx* ctx, const gbl_search_config* cfg, const gbl_search_state* st, const double* residual,
                   const double* psd);

/* One iteration (see above).  Errors: GBL_EINVAL, GBL_EUNSUPPORTED (N, or a
 * mixed-precision context). */
int gb_search_step(gbl_ctx* ctx, const gbl_search_config* cfg, const gbl_search_state* st, int64_t iter,
                   const double* residual, const double* psd);

/* Restart ball: every chain of band b moves to best_u[b] + sigma n (n
 * standard normals by Box-Muller from the uniforms of unit (b n_t + t) n_w +
 * w, move 8, draws 2p and 2p+1 for coordinates 2p, 2p+1), periodic
 * coordinates wrapped, the others clamped into the box (f0 strictly below the
 * band's top); logl re-evaluated, stall cleared, the best points kept.
 * sigma: HOST array [8]. */
int gb_search_ball(gbl_ctx* ctx, const gbl_search_config* cfg, const gbl_search_state* st, int64_t iter,
                   const double* sigma, const double* residual, const double* psd);

/* ---------------------------------------------------------------------------
 * Correlated A/E channels (Sec. 2: the A, E, T variables are uncorrelated only
 * under idealised assumptions; with unequal noise a likelihood matrix across
 * channels is needed).  Noise model: twelve independent noises -- the
 * metrology noise of each link and the Doppler noise of each test mass --
 * with the spectral shapes of eq. psd; a link y_{s->r} carries o_{sr} +
 * delta_{rs} + D delta_{sr}, D = exp(-2 pi i f L / c); the first-generation
 * Michelson combinations and A = (Z - X)/sqrt 2, E = (X - 2Y + Z)/sqrt 6 give
 * the 2 x 2 noise matrix C per bin.  Equal levels reproduce eq. psd with no
 * cross term.  The inner product becomes <a|b>_K = 4 df Re sum_k a_k^H K_k
 * b_k with K = C^-1.
 * levels [P][12]: sqrt S_oms of the links 0->1, 0->2, 1->0, 1->2, 2->0, 2->1,
 * then sqrt S_acc of the test masses (0,1), (0,2), (1,0), (1,2), (2,0), (2,1)
 * (mass (a, b): on craft a, facing craft b).
 * Matrix arrays K [n_K][5][n_bins]: K_AA, K_EE, Re K_AE, Im K_AE, ln det C.
 * --------------------------------------------------------------------------- */
int gb_noise_matrix(gbl_ctx* ctx, const double* levels, int64_t P, double* out);

/* eq. swapsource with the channel matrix:
 *   dlogl[b] = <R|a - r>_K - 1/2 <a - r|a - r>_K,  R = residual[res_idx[b]],
 * K = K[k_idx[b]], a/r the width-N templates of params_new/params_old (FP64),
 * the sum over the union of their windows clipped to the band.  Undefined
 * parameters or out-of-range indices give NaN.
 * Errors: GBL_EINVAL, GBL_EUNSUPPORTED (N). */
int gb_delta_loglike_matrix(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* K, int32_t n_K,
                            const double* params_old, const double* params_new, int32_t N, const int32_t* res_idx,
                            const int32_t* k_idx, int64_t B, double* dlogl);

/* eq. like with the channel matrix: logl[p] = -1/2 <R|R>_K - sum_k ln det C_k,
 * R = residual[res_idx[p]], K = K[k_idx[p]]; fixed-order reduction.  An
 * out-of-range index gives NaN.  Errors: GBL_EINVAL. */
int gb_loglike_matrix(gbl_ctx* ctx, const double* residual, int32_t n_res, const double* K, int32_t n_K,
                      const int32_t* res_idx, const int32_t* k_idx, int64_t P, double* logl);

#ifdef __cplusplus
}
#endif

#endif /* GBL_H */
