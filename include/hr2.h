/*
 * hr2.h — C ABI of libhr2, the MI355X (gfx950) emission-spectrum forward model
 * of Helios-r2 (Kitzmann et al. 2020, arXiv:1910.01070).
 *
 * The forward model maps one atmospheric column (one parameter set of the
 * nested sampler) to the theoretical observation D_m(M, Theta) at the data
 * bins (Sect. 3.1, the quantity entering Eq. 19).  It runs in three stages,
 * each a HIP kernel on the device (Sect. 2.8 lists them as the GPU part):
 *
 *   1. opacity      chi_l(nu) = sum_s n_s,l sigma_s(nu; T_l, p_l)  + CIA
 *                   (Sect. 2.3: cross-sections tabulated in (T, p, nu),
 *                   interpolated to each level; H2-H2 and H2-He CIA)
 *   2. emission RT  short characteristics with a linear source, alpha = 0
 *                   (Eq. 4-7), source S = B_nu(T) (Eq. 2), outgoing flux by
 *                   Gauss quadrature over mu in (0, 1] (Eq. 8)
 *   3. observation  scaling F = F+ f (R/d)^2 (Eq. 9), Gaussian instrument
 *                   profile truncated at 5 sigma (Eq. 17), binning to the
 *                   observational bins (Sect. 2.8)
 *
 * Readings of points the paper leaves open (all fixed here and in the
 * oracle alike):
 *   - levels are indexed bottom (0, highest p) to top (L-1); layer l joins
 *     levels l and l+1; the recurrence runs upward, the deeper level is the
 *     upwind point, Delta = dtau_l / mu >= 0 (Eq. 4, 7);
 *   - Eq. 4's attenuation is exp(-Delta) (dtau over mu);
 *   - gamma = (1 - exp(-Delta))/Delta - exp(-Delta) (the linear-source
 *     upwind coefficient; the printed sign of Eq. 6 makes beta + gamma exceed
 *     1 - exp(-Delta));
 *   - lower boundary I+(bottom, mu) = B_nu(T_0) (semi-infinite atmosphere);
 *   - n_mu-point Gauss-Legendre nodes on mu in [0, 1] (Eq. 8);
 *   - dtau_l = (chi_l + chi_{l+1})/2 * dz_l with hydrostatic, ideal-gas
 *     dz_l = k_B Tbar_l / (mubar m_u g) * ln(p_l / p_{l+1}),
 *     Tbar_l = (T_l + T_{l+1})/2;
 *   - cross-sections: bilinear in (T, log10 p) on log sigma, clamped to the
 *     table, lower node i = largest index with axis[i] <= value (capped at
 *     N-2), weight w = (value - axis[i]) / (axis[i+1] - axis[i]);
 *   - CIA: n_a n_b k(T, nu), linear in T on log k, same T axis, clamped;
 *   - H2 and He fill the rest of the gas, x_He = r x_H2 (r = he_h2_ratio);
 *   - Planck in wavenumber form, 2 h c^2 nu^3 / expm1(h c nu / (k_B T)),
 *     with the unclamped level temperature;
 *   - instrument profile: Gaussian of FWHM nu/R evaluated at the output
 *     point, points with |k| * dnu_eff <= 5 sigma kept, weights renormalised
 *     over the points of the window;
 *   - bins: trapezoid mean of the convolved spectrum between edges snapped
 *     to the nearest window point (ties away from the start), adjacent bins
 *     share the edge point.
 *
 * Units: cgs, wavenumber in cm^-1, pressure in bar, temperature in K.
 * chi in cm^-1; F+ in erg s^-1 cm^-2 (cm^-1)^-1; bins = f (R/d)^2 times the
 * bin mean of the convolved F+.
 *
 * Precision: device arrays of stage and batch calls hold `hr2_real`
 * elements: double when the tables were created with HR2_TABLE_F64, float
 * otherwise.  With F32/F16/BF16 storage the arithmetic is FP32; with F64 it
 * is FP64.
 *
 * Ownership: the caller owns every array it passes.  *_create copies what it
 * needs; host arrays may be freed on return.  The library owns handles,
 * resident tables, observation layouts and its scratch.  Stage and batch
 * calls are asynchronous on `stream` (a hipStream_t passed as void*, NULL =
 * the null stream); device buffers must stay alive until the stream has
 * completed them.  Host arrays passed to them may be reused on return.
 *
 * Errors: every call returns hr2_status; nothing is thrown across the ABI.
 * Host-side validation happens before anything is enqueued, so an
 * HR2_E_INVALID_ARG / HR2_E_OUT_OF_RANGE return leaves every output
 * untouched.  A failed HIP call returns HR2_E_DEVICE.  hr2_last_error()
 * gives a thread-local text of the last failure on the calling thread.
 *
 * Threading: a context (and the tables / observation layouts made from it)
 * is used by one thread at a time; hr2_serve_submit and hr2_serve_poll are
 * thread-safe.
 */
#ifndef HR2_H
#define HR2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HR2_OK = 0,
  HR2_NOT_READY = 1,        /* hr2_serve_poll only: request still pending or running */
  HR2_E_INVALID_ARG = -1,   /* NULL pointer, NaN/Inf, non-monotone axis, bad count     */
  HR2_E_OUT_OF_RANGE = -2,  /* window outside the table, n_mu outside [1, 8], too big */
  HR2_E_NO_MEMORY = -3,     /* device or host allocation failed; request > budget     */
  HR2_E_DEVICE = -4,        /* a HIP call failed                                       */
  HR2_E_NOT_FOUND = -5,     /* unknown or already consumed ticket                      */
  HR2_E_UNSUPPORTED = -6,   /* valid request the library does not implement          */
  HR2_E_CANCELLED = -7      /* request cancelled by hr2_serve_destroy                  */
} hr2_status;

typedef enum {
  HR2_OFFSET_ROW = 0,      /* one log2 offset per table row (default) */
  HR2_OFFSET_SPECIES = 1   /* one log2 offset per species */
} hr2_offset_mode;

typedef enum {
  HR2_TABLE_F32 = 0,   /* log2-sigma rows minus a per-row offset, float    */
  HR2_TABLE_F16 = 1,   /* same, IEEE binary16 (one RNE rounding from FP64) */
  HR2_TABLE_BF16 = 2,  /* same, bfloat16 (RNE to float, then RNE to bf16)  */
  HR2_TABLE_F64 = 3    /* log2-sigma, no offset, double; FP64 arithmetic   */
} hr2_table_dtype;

enum {
  HR2_MAX_SPECIES = 12,
  HR2_MAX_CIA = 2,
  HR2_MAX_LEVELS = 1024,
  HR2_MAX_MU = 8,
  HR2_MAX_ORDER = 8,          /* finite-element order q */
  HR2_MAX_TNODES = 128,       /* temperature nodes K_e q + 1 */
  HR2_NOALLOC_SCRATCH_BYTES = 32 << 20   /* fixed device array of hr2_forward_batch_dev_noalloc */
};

typedef struct hr2_ctx hr2_ctx;
typedef struct hr2_tables hr2_tables;
typedef struct hr2_obs hr2_obs;
typedef struct hr2_server hr2_server;
typedef struct hr2_params hr2_params;

/* Create a context on HIP device `hip_device`.  Allocates the angular
 * quadrature constants and grow-only scratch.  Errors: HR2_E_INVALID_ARG
 * (out == NULL), HR2_E_DEVICE (no such device). */
hr2_status hr2_ctx_create(int hip_device, hr2_ctx **out);
/* Waits for the context's work, frees its scratch.  NULL is a no-op. */
void hr2_ctx_destroy(hr2_ctx *ctx);
/* Thread-local text of the last failure on this thread ("" if none). */
const char *hr2_last_error(void);

/* Context options.  CHUNKS, NU_PER_LANE and TIMING shape launches only
 * (results do not depend on them beyond FP32 rounding of the chunk
 * combination).  SOURCE selects the source-function interpolant of the
 * short characteristics (Eq. 4-7): 1 = linear (default, the paper's
 * choice), 2 = parabolic (the quadratic through the upwind, local and
 * downwind levels, Olson & Kunasz 1987 coefficients; the top step, which
 * has no downwind level, and a step whose downwind layer has zero optical
 * depth stay linear).  The parabolic coefficients grow like 1/dd when the
 * downwind layer is much thinner than the upwind one, so FP32 results lose
 * accuracy at sharp optical-depth contrasts (an opaque cloud top). */
typedef enum {
  HR2_OPT_CHUNKS = 0,      /* layer chunks per wavenumber tile: 0 = auto, 1 .. 8 */
  HR2_OPT_NU_PER_LANE = 1, /* wavenumbers per lane of the one-launch-per-set path
                              (one-species tables, windows of at most 4096 points,
                              batches that fill the device): 0 = auto (2 up to
                              three angles, 1 above), 1 or 2;
                              the column kernel keeps 1 (2 costs it half its
                              resident waves)                                        */
  HR2_OPT_TIMING = 2,      /* n > 0: time the kernels of every n-th forward-batch
                              call through HIP events attached to their launches
                              (0 = off)                                            */
  HR2_OPT_SOURCE = 3,      /* 1 = linear source (default), 2 = parabolic; servers
                              take the value their context has at creation          */
  HR2_OPT_ROW_POLICY = 4,  /* table-row loads of one-set calls: 0 = auto (non-temporal
                              when the call's rows would overflow the last-level
                              cache), 1 = always non-temporal, 2 = always cached.
                              Batches always load cached.  Results do not change. */
  HR2_OPT_TILE_PAIRS = 5,  /* one-set calls whose tiles spill past one round of
                              resident workgroups: 0 = auto (the first round's
                              workgroups take two tiles each, the tiles left
                              over twice the layer chunks), 1 = off.  The
                              leftover tiles' F+ changes by the rounding of a
                              different chunk split (below 1e-6 relative).      */
  HR2_OPT_TIMING_KERNELS = 6 /* which kernels a timed call times, a bit mask: 1 the
                              level kernel, 2 the column kernel (or the whole-
                              forward-model kernel), 4 the convolution; 1..7,
                              default 7.  Each timed launch costs a few
                              microseconds of GPU time.                          */
} hr2_option;
hr2_status hr2_ctx_set_option(hr2_ctx *ctx, hr2_option opt, int value);

/* Kernel timing of the forward-batch calls made while HR2_OPT_TIMING was on
 * (each kernel's own start and end, from HIP events attached to its launch on
 * the caller's stream, so the gaps between kernels are not counted): waits
 * for those calls, writes the summed milliseconds of the level kernel, the
 * opacity+RT column kernel and the convolve/bin kernel to ms[0..2] and the
 * number of calls to *n_calls, then resets.  A call that runs the whole
 * forward model in one launch (small windows in large batches) counts that
 * launch as its column kernel and nothing for the other two.  At most 65536
 * calls are recorded between collections (later ones are not timed). */
hr2_status hr2_ctx_collect_timing(hr2_ctx *ctx, double ms[3], int64_t *n_calls);

/* Cross-section and CIA tables (Sect. 2.3).  All arrays are host FP64.
 *   T_K[n_T]            strictly increasing, > 0 (non-uniform allowed), n_T >= 2
 *   log10_p_bar[n_p]    strictly increasing, n_p >= 2
 *   nu_k = nu0_cm + k * dnu_cm, k < n_nu (cm^-1), dnu_cm > 0, nu0_cm > 0
 *   log10_sigma         [n_species][n_T][n_p][n_nu], sigma in cm^2/molecule
 *   molar_mass[n_species]   g/mol (enters the mean molecular weight)
 *   n_cia               0 or 2 (pair 0 = H2-H2, pair 1 = H2-He)
 *   log10_k_cia         [n_cia][n_T][n_nu], k in cm^5/molecule^2, same T axis
 *   he_h2_ratio         x_He / x_H2 of the filler gas, > 0
 *   dtype               storage in HBM.  For F32/F16/BF16 each row
 *                       (species, T, p) (and each CIA row) is stored as
 *                       y = log10_sigma * log2(10) - off_row in the dtype,
 *                       off_row = (min + max)/2 of that row's
 *                       log10_sigma * log2(10) values (FP64); F64 keeps
 *                       log10_sigma * log2(10) with no offset.  CIA rows are
 *                       float (double for F64) in every case.
 *   offset_mode         HR2_OFFSET_ROW (0, the default above) or
 *                       HR2_OFFSET_SPECIES (1): every row of a species uses
 *                       the midpoint of the whole species' log2 range (a
 *                       coarser rule kept for comparison: the stored values
 *                       are larger, so FP16/BF16 rounding errors grow).
 *                       CIA rows keep per-row offsets; ignored for F64.
 * Copies everything to the device; host arrays may be freed on return.  One
 * species block (n_T * n_p rows of n_nu rounded up to 64 entries, in the
 * storage type) must stay below 4 GiB, and so must the CIA blocks of both
 * pairs together (n_cia * n_T rows); the whole table may be larger.  These
 * sizes are checked before anything is read or allocated.
 * Errors: HR2_E_INVALID_ARG (NULL, NaN/Inf, non-monotone axis, counts out of
 * [1, HR2_MAX_SPECIES], n_cia not 0/2, offset_mode not 0/1), HR2_E_OUT_OF_RANGE (a species block,
 * or the CIA blocks together, of 4 GiB or more), HR2_E_NO_MEMORY,
 * HR2_E_DEVICE. */
typedef struct {
  int n_species, n_T, n_p;
  const double *T_K;
  const double *log10_p_bar;
  double nu0_cm, dnu_cm;
  int64_t n_nu;
  const double *log10_sigma;
  const double *molar_mass;
  int n_cia;
  const double *log10_k_cia;
  double he_h2_ratio;
  hr2_table_dtype dtype;
  int offset_mode;   /* hr2_offset_mode; zero-initialise for the default */
} hr2_tables_desc;

hr2_status hr2_tables_create(hr2_ctx *ctx, const hr2_tables_desc *desc, hr2_tables **out);
void hr2_tables_destroy(hr2_tables *tables);

/* One atmospheric column = one parameter set (Table 1 parameters after the
 * temperature profile (Sect. 2.5) and free chemistry (Sect. 5.2) have been
 * evaluated).
 *   n_levels   2 <= L <= HR2_MAX_LEVELS; layers = L - 1
 *   p_bar[L]   strictly decreasing, > 0 (level 0 = bottom)
 *   T_K[L]     > 0; table lookups clamp to the T axis, Planck uses T as given
 *   x[n_species]  isoprofile mixing ratios, >= 0, sum < 1 (Sect. 5.2)
 *   log_g_cgs  log10 of surface gravity in cm s^-2
 *   scale      f (R/d)^2 (Eq. 9), finite
 *   tau_cloud, p_cloud_top_bar, cloud_bottom_frac
 *              optional gray cloud layer (App. B): total optical depth
 *              tau_cloud >= 0 (0 = clear sky, the other two ignored),
 *              independent of wavenumber, between p_cloud_top_bar > 0 and
 *              p_cloud_top_bar * cloud_bottom_frac (cloud_bottom_frac > 1).
 *              Reading (the appendix is silent): the optical depth is spread
 *              uniformly in ln p over that range and each layer adds its
 *              share to its optical depth.  Zero-initialise for clear sky. */
typedef struct {
  int n_levels;
  const double *p_bar;
  const double *T_K;
  const double *x;
  double log_g_cgs;
  double scale;
  double tau_cloud;
  double p_cloud_top_bar;
  double cloud_bottom_frac;
} hr2_column;

/* Wavenumber window: table points nu_begin + j * nu_stride, j < nu_count.
 * Requires nu_begin >= 0, nu_count >= 1, nu_stride >= 1 and
 * nu_begin + (nu_count - 1) * nu_stride < n_nu (else HR2_E_OUT_OF_RANGE). */
typedef struct {
  int64_t nu_begin, nu_count, nu_stride;
} hr2_window;

/* Stage 1 alone (Sect. 2.3 / 2.8): absorption coefficient at every level.
 * chi_dev: device hr2_real[L][nu_count], cm^-1.  Enqueued on stream. */
hr2_status hr2_opacity(hr2_ctx *ctx, const hr2_tables *tables, const hr2_column *col,
                       hr2_window window, void *chi_dev, void *stream);

/* Stage 2 alone (Eq. 2, 4-8): outgoing top-of-atmosphere flux F+ from a
 * given absorption coefficient.  chi_dev: device hr2_real[L][nu_count]
 * (e.g. from hr2_opacity); fplus_dev: device hr2_real[nu_count];
 * 1 <= n_mu <= HR2_MAX_MU.  The column supplies T (Planck), p, x, log g
 * (layer thicknesses).  Enqueued on stream. */
hr2_status hr2_rt_emission(hr2_ctx *ctx, const hr2_tables *tables, const hr2_column *col,
                           hr2_window window, const void *chi_dev, int n_mu,
                           void *fplus_dev, void *stream);

/* Observation layout (Eq. 17 and the binning of Sect. 2.8): resolving power
 * R > 0 (sigma(nu) = nu / (R 2 sqrt(2 ln 2))), n_bins >= 1 bins with
 * increasing edges bin_edges_cm[n_bins + 1], each snapped to the nearest
 * window point; snapped edges must be strictly increasing.  The convolution
 * and binning are linear, so the layout is held as one banded weight row per
 * bin (the composite of trapezoid weights and renormalised Gaussians), built
 * on the device; with FP64 tables the Gaussians' normalisations are summed
 * tap by tap, otherwise they come from a closed form (Euler-Maclaurin) that
 * equals those sums within 1e-9 relative.  Blocks until built.  Errors: HR2_E_INVALID_ARG,
 * HR2_E_OUT_OF_RANGE (window, or a snapped edge outside it), HR2_E_NO_MEMORY. */
hr2_status hr2_obs_create(hr2_ctx *ctx, const hr2_tables *tables, hr2_window window,
                          double resolving_power, int n_bins, const double *bin_edges_cm,
                          hr2_obs **out);
void hr2_obs_destroy(hr2_obs *obs);
/* Number of bins of a layout (0 for NULL). */
int hr2_obs_n_bins(const hr2_obs *obs);

/* Stage 3 alone (Eq. 9, 17, binning): bins_dev[n_bins] = scale * binned,
 * convolved fplus_dev[nu_count].  Device hr2_real arrays; enqueued. */
hr2_status hr2_convolve_bin(hr2_ctx *ctx, const hr2_obs *obs, const void *fplus_dev,
                            double scale, void *bins_dev, void *stream);

/* The whole forward model for n_sets columns that share n_levels (host
 * columns, validated on the host, staged to the device).  bins_dev: device
 * hr2_real[n_sets][n_bins].  fplus_dev: NULL, or device
 * hr2_real[n_sets][nu_count] that receives the unscaled F+ of each set.
 * Each set's result does not depend on the other sets of the call.  A call
 * of one set whose table rows would overflow the 256 MB last-level cache
 * (estimated at one new row per level and species) loads them non-temporal,
 * which leaves the other kernels' small working set cached; the results are
 * the same either way.  The same holds for the _dev, ln L and parameter-
 * vector entry points below. */
hr2_status hr2_forward_batch(hr2_ctx *ctx, const hr2_tables *tables, const hr2_obs *obs,
                             int n_sets, const hr2_column *cols, int n_mu,
                             void *bins_dev, void *fplus_dev, void *stream);

/* Same, with the columns already resident in device memory (FP64):
 *   p_dev[n_sets][n_levels], T_dev[n_sets][n_levels],
 *   x_dev[n_sets][n_species], log_g_dev[n_sets], scale_dev[n_sets],
 *   cloud_dev: NULL (clear sky) or [n_sets][3] = (tau_cloud,
 *   p_cloud_top_bar, cloud_bottom_frac) as in hr2_column.
 * Nothing is validated on the host (that would need a device read); the
 * level kernel checks every set and writes its status to set_status_dev
 * (device int[n_sets], may be NULL): 0 = valid, HR2_E_INVALID_ARG otherwise.
 * An invalid set's bins and F+ are NaN; other sets are unaffected.
 * This call may be captured into a HIP graph once it has been made with the
 * same sizes outside capture (so no staging copy or scratch growth is
 * needed; otherwise it returns HR2_E_UNSUPPORTED under capture).  A captured
 * graph writes the context's scratch (level records, F+ when fplus_dev is
 * NULL): order its replays against other calls on the same context (same
 * stream, or events), since neither waits for the other.  Once a call has
 * been captured on a context, scratch that a later, larger call replaces is
 * kept until hr2_ctx_destroy, so an older graph never writes freed memory. */
hr2_status hr2_forward_batch_dev(hr2_ctx *ctx, const hr2_tables *tables, const hr2_obs *obs,
                                 int n_sets, int n_levels, const double *p_dev,
                                 const double *T_dev, const double *x_dev,
                                 const double *log_g_dev, const double *scale_dev,
                                 const double *cloud_dev, int n_mu, void *bins_dev,
                                 void *fplus_dev, int *set_status_dev, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * as hr2_forward_batch_dev (same arguments, kernels and results, bit for
 * bit), except that its scratch lives in one fixed device array of
 * HR2_NOALLOC_SCRATCH_BYTES (32 MiB) per GPU instead of the context's
 * grow-only buffers: the level records (128 bytes per set and level, 256
 * with F64 tables, rounded up to 256 bytes in all) and, when fplus_dev is
 * NULL, the unscaled F+ (4 bytes per set and window point, 8 with F64
 * tables).  Every GPU the library runs on holds its array from the first
 * context made on it until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine, no timing events)
 * and needs no staging copy, so it may be captured into a HIP graph at any
 * time.  The kernels write every byte of the array they read, so nothing
 * in it has to start at zero; it keeps the last call's contents.
 * All calls on one GPU share its array: calls that overlap on one GPU
 * (other streams, other contexts of the device) race on it, so the caller
 * must order them (one stream, or events).  The other entry points do not
 * use it.  Errors: as hr2_forward_batch_dev, plus HR2_E_OUT_OF_RANGE
 * (before anything is enqueued) when the call's scratch exceeds the array
 * (e.g. more than 55 sets of a 150,000-point window without an F+ buffer),
 * and HR2_E_DEVICE when the array's address could not be looked up. */
hr2_status hr2_forward_batch_dev_noalloc(hr2_ctx *ctx, const hr2_tables *tables,
                                         const hr2_obs *obs, int n_sets, int n_levels,
                                         const double *p_dev, const double *T_dev,
                                         const double *x_dev, const double *log_g_dev,
                                         const double *scale_dev, const double *cloud_dev,
                                         int n_mu, void *bins_dev, void *fplus_dev,
                                         int *set_status_dev, void *stream);

/* ---- likelihood: the forward model fused with ln L (Sect. 3.1, Eq. 19;
 * error inflation of Sect. 3.3, Eq. 22-23) ----
 * ln L = sum_j [ -(D_j - m_j)^2 / (2 s_j^2) - 1/2 ln(2 pi s_j^2) ], where m_j
 * is the model's bin j (exactly what hr2_forward_batch returns, in
 * hr2_real) and s_j^2 = sigma_j^2, or sigma_j^2 + 10^eps with inflation.
 * Reading of Eq. 23: its normalisation term belongs inside the sum, as in
 * Eq. 19.  The per-bin terms are formed in FP64 and summed per set in a
 * fixed order, so repeated calls give identical results.
 *
 * hr2_obs_set_data attaches observed data to a layout: D[n_bins] (finite)
 * and sigma[n_bins] (finite, > 0), host FP64, copied (the caller keeps its
 * arrays).  It may be called again to replace the data; it first waits for
 * the calls already enqueued through the context that created the layout
 * (not for the rest of the device, and not for replays of captured graphs,
 * which the caller orders).  Errors: HR2_E_INVALID_ARG (NULL, non-finite,
 * sigma <= 0), HR2_E_NO_MEMORY. */
hr2_status hr2_obs_set_data(hr2_obs *obs, const double *D, const double *sigma);

/* ln L of n_sets host columns (as hr2_forward_batch): lnl_dev is device
 * double[n_sets].  log10_eps: NULL (Eq. 19) or host double[n_sets], the
 * exponent of Eq. 22 per set.  bins_dev: NULL, or device
 * hr2_real[n_sets][n_bins] that also receives the model bins.  Enqueued on
 * stream; only n_sets doubles need to come back to the host.  Errors: as
 * hr2_forward_batch, plus HR2_E_INVALID_ARG when the layout has no data or
 * a log10_eps is not finite. */
hr2_status hr2_loglike_batch(hr2_ctx *ctx, const hr2_tables *tables, const hr2_obs *obs,
                             int n_sets, const hr2_column *cols, int n_mu,
                             const double *log10_eps, double *lnl_dev, void *bins_dev,
                             void *stream);

/* Same with device-resident FP64 columns and optional clouds (as
 * hr2_forward_batch_dev); log10_eps_dev: NULL or device double[n_sets].  An invalid set's ln L is
 * NaN and its set_status_dev entry HR2_E_INVALID_ARG.  Capturable into a HIP
 * graph under the same condition as hr2_forward_batch_dev. */
hr2_status hr2_loglike_batch_dev(hr2_ctx *ctx, const hr2_tables *tables, const hr2_obs *obs,
                                 int n_sets, int n_levels, const double *p_dev,
                                 const double *T_dev, const double *x_dev,
                                 const double *log_g_dev, const double *scale_dev,
                                 const double *cloud_dev, const double *log10_eps_dev, int n_mu,
                                 double *lnl_dev, void *bins_dev, int *set_status_dev,
                                 void *stream);

/* ---- parameter vectors: Theta -> column on the device ----
 * Temperature (Sect. 2.5.1, Eq. 12-16): n_elements elements of order q
 * split [log10_p_top, log10_p_bottom] into equal parts; on each the
 * temperature is the Lagrange interpolant (Eq. 13) through q + 1 nodes at
 * the Gauss-Lobatto points of the reference element [0, 1]; elements share
 * boundary nodes, so there are N_T = n_elements q + 1 node temperatures
 * (Eq. 16).  The bottom node's temperature T1 is a parameter; node n (from
 * the bottom) is b_n times node n - 1.  Readings: element 1 and local
 * coordinate 0 are at the bottom; a level on an element boundary takes the
 * element above (the same value, the profile being continuous).
 * Levels: n_levels, equidistant in log p, level 0 at log10_p_bottom.
 * Free chemistry (Sect. 5.2): height-independent mixing ratios; table
 * species s gets species_factor[s] * xfree[species_src[s]], or 0 when
 * species_src[s] < 0 (sodium from potassium with the solar ratio, say).
 * Scale (Eq. 9): f (radius_cm / (d_pc * 3.0856775814913673e18 cm))^2.
 *
 * One parameter vector (FP64, row of theta_dev[n_sets][n_theta]):
 *   log g (cgs), f, d (parsec), T1 (K), b_1 .. b_{N_T - 1},
 *   xfree[0 .. n_free - 1], then tau_cloud, p_cloud_top_bar,
 *   cloud_bottom_frac (as in hr2_column) when with_cloud, then log10 eps
 *   (Eq. 22) when with_eps.
 * An invalid vector (T1, b, f or d not > 0, x < 0, a cloud outside the
 * hr2_column ranges, anything not finite) yields NaN temperatures, which the forward model reports as an invalid
 * set (status HR2_E_INVALID_ARG, NaN bins and ln L). */
typedef struct {
  int n_elements;                 /* K_e >= 1 */
  int order;                      /* q in [1, HR2_MAX_ORDER]; K_e q + 1 <= HR2_MAX_TNODES */
  int n_levels;                   /* [2, HR2_MAX_LEVELS] */
  double log10_p_bottom;          /* bar */
  double log10_p_top;             /* bar, < log10_p_bottom */
  double radius_cm;               /* R_* of Eq. 9, > 0 */
  int n_free;                     /* free mixing ratios in theta, [0, HR2_MAX_SPECIES] */
  int with_cloud;                 /* 0 or 1: theta carries a gray cloud (App. B) */
  int with_eps;                   /* 0 or 1 */
  const int *species_src;         /* [n_species of the tables], each in [-1, n_free) */
  const double *species_factor;   /* [n_species], finite, >= 0 */
} hr2_param_layout;

/* Validate and keep a layout for these tables (copied; host arrays may be
 * freed afterwards).  Errors: HR2_E_INVALID_ARG (NULL, out-of-range field). */
hr2_status hr2_params_create(hr2_ctx *ctx, const hr2_tables *tables,
                             const hr2_param_layout *layout, hr2_params **out);
void hr2_params_destroy(hr2_params *params);
/* Parameters per set: 3 + N_T + n_free + 3 with_cloud + with_eps (0 for NULL). */
int hr2_params_n_theta(const hr2_params *params);

/* Unpack n_sets device parameter vectors into device FP64 columns in the
 * layout hr2_forward_batch_dev reads: p_dev, T_dev [n_sets][n_levels],
 * x_dev [n_sets][n_species], log_g_dev, scale_dev [n_sets]; cloud_dev
 * [n_sets][3] or NULL (zeros without with_cloud); log10_eps_dev [n_sets] or
 * NULL (0 without with_eps).  Enqueued on stream. */
hr2_status hr2_params_unpack_dev(hr2_ctx *ctx, const hr2_params *params, int n_sets,
                                 const double *theta_dev, double *p_dev, double *T_dev,
                                 double *x_dev, double *log_g_dev, double *scale_dev,
                                 double *cloud_dev, double *log10_eps_dev, void *stream);

/* Parameter vectors straight to spectra and/or ln L: the level stage forms
 * each set's column from its vector (the same arithmetic as the unpack
 * above, so results equal unpack-then-forward exactly), then the forward
 * model, then (lnl_dev non-NULL) the
 * likelihood of Eq. 19, or Eq. 22-23 with the vector's own eps when the
 * layout has with_eps.  bins_dev: NULL or device hr2_real[n_sets][n_bins];
 * lnl_dev: NULL or device double[n_sets]; at least one of the two.
 * set_status_dev as in hr2_forward_batch_dev.  Capturable into a HIP graph
 * after one eager call with the same sizes.  Errors: as
 * hr2_loglike_batch_dev; HR2_E_INVALID_ARG when the layout's tables differ. */
hr2_status hr2_forward_params_dev(hr2_ctx *ctx, const hr2_tables *tables, const hr2_obs *obs,
                                  const hr2_params *params, int n_sets,
                                  const double *theta_dev, int n_mu, void *bins_dev,
                                  double *lnl_dev, int *set_status_dev, void *stream);

/* ---- serving: continuous batching of uneven forward-model requests ----
 * A scheduler thread owns two streams.  Requests (each n_sets columns
 * sharing n_levels, its own window, resolving power and bins) are admitted
 * while their device footprint fits the budget and a slot is free; every
 * step takes all admitted, not yet launched requests and runs them with one
 * upload of their columns and bin plans, one level-record launch, one pair
 * of observation-layout launches, one opacity+RT launch per kernel variant
 * (chunking and angle tier), one convolution/binning launch and one copy of
 * all their bins to pinned host memory.  Requests arriving meanwhile join
 * the next step; up to two steps are in flight.  Per-set arithmetic does not
 * depend on the other requests in a step, so a result is bit-identical
 * alone and in the mix. */
typedef struct {
  hr2_window window;
  double resolving_power;
  int n_bins;
  const double *bin_edges_cm;   /* [n_bins + 1] */
  int n_sets;
  const hr2_column *cols;       /* [n_sets], all with the same n_levels */
  int n_mu;
} hr2_request;

typedef enum {
  HR2_REQ_PENDING = 0, HR2_REQ_RUNNING = 1, HR2_REQ_DONE = 2,
  HR2_REQ_ERROR = 3, HR2_REQ_CANCELLED = 4
} hr2_request_state;

typedef struct {
  int state;                 /* hr2_request_state */
  double t_submit, t_admit, t_done;   /* seconds, CLOCK_MONOTONIC */
  hr2_status error;          /* why a request ended in ERROR / CANCELLED */
  int n_bins, n_sets;
} hr2_request_info;

/* hbm_budget_bytes: cap on the device bytes held by admitted requests
 * (level records, F+, layouts and their build scratch); max_slots: cap on
 * admitted requests.  Each of the two step streams also keeps a grow-only
 * stage outside the budget for the inputs and bins of the step it runs
 * (per request 8 (2 L + S + 5) n_sets + 28 n_bins bytes of inputs and
 * 4 n_sets n_bins bytes of bins, 8 with F64 tables, each rounded up to 256).
 * Errors: HR2_E_INVALID_ARG, HR2_E_DEVICE. */
hr2_status hr2_serve_create(hr2_ctx *ctx, const hr2_tables *tables, size_t hbm_budget_bytes,
                            int max_slots, hr2_server **out);
/* Non-blocking.  Validates and deep-copies the request, returns a ticket.
 * Errors: HR2_E_INVALID_ARG / HR2_E_OUT_OF_RANGE (validation),
 * HR2_E_NO_MEMORY (the request alone exceeds the budget). */
hr2_status hr2_serve_submit(hr2_server *srv, const hr2_request *req, uint64_t *ticket);
/* Same as hr2_serve_submit with the request's columns packed host arrays
 * (FP64): p_bar[n_sets][n_levels], T_K[n_sets][n_levels],
 * x[n_sets][n_species], log_g[n_sets], scale[n_sets].  Deep-copied. */
hr2_status hr2_serve_submit_packed(hr2_server *srv, hr2_window window, double resolving_power,
                                   int n_bins, const double *bin_edges_cm, int n_sets,
                                   int n_levels, const double *p_bar, const double *T_K,
                                   const double *x, const double *log_g, const double *scale,
                                   int n_mu, uint64_t *ticket);
/* HR2_NOT_READY while pending/running.  When done, copies n_sets * n_bins
 * results (float; double for F64 tables) to bins_host if capacity allows
 * (else HR2_E_INVALID_ARG, ticket kept), releases the ticket and returns
 * HR2_OK.  A request that failed returns its error and is released.
 * info may be NULL.  Unknown / released ticket: HR2_E_NOT_FOUND. */
hr2_status hr2_serve_poll(hr2_server *srv, uint64_t ticket, void *bins_host,
                          size_t capacity_elems, hr2_request_info *info);
/* Blocks until ticket completes (or timeout_s elapses: HR2_NOT_READY), then
 * behaves as hr2_serve_poll. */
hr2_status hr2_serve_wait(hr2_server *srv, uint64_t ticket, double timeout_s, void *bins_host,
                          size_t capacity_elems, hr2_request_info *info);
/* Cancels pending requests (state CANCELLED), waits for launched ones,
 * joins the scheduler and frees everything. */
void hr2_serve_destroy(hr2_server *srv);

/* Test hook: the next scheduler step is treated as a failed launch, which
 * marks exactly that step's requests ERROR (HR2_E_DEVICE); later steps run
 * normally.  Nothing is enqueued for the failed step. */
hr2_status hr2_serve_debug_fail_next_step(hr2_server *srv);

/* Test hook: while hold != 0 the scheduler admits requests but launches no
 * step; hold = 0 releases it (the held requests then share steps). */
hr2_status hr2_serve_debug_hold(hr2_server *srv, int hold);

/* Counters of a server: steps launched, requests done / failed, most
 * requests admitted at once, most requests in one step, peak admitted bytes. */
typedef struct {
  uint64_t steps, requests_done, requests_failed, max_inflight, max_step_requests;
  size_t peak_bytes;
} hr2_serve_stats;
hr2_status hr2_serve_get_stats(hr2_server *srv, hr2_serve_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* HR2_H */
