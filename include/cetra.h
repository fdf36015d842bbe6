/*
 * cetra.h -- C ABI of the MI355X (gfx950) transit-search library.
 *
 * The library implements the two-stage transit search of Smith et al. 2025
 * ("CETRA", arXiv:2503.20875): a linear search that correlates a transit
 * template with a regularly resampled light curve over a grid of reference
 * times and durations (Sec. 2.2), followed by a periodic search that
 * phase-folds the single-event results over a grid of periods with a common
 * transit depth and keeps the maximum-likelihood candidate per period
 * (Sec. 2.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units      Times are days (FP64).  Fluxes are offsets from baseline (FP32):
 *            0 is the baseline and 1 means the star is fully blocked, so a
 *            transit is a positive offset (Sec. 2, units).  Reference times
 *            t0 are transit mid-points measured from the resampled grid's
 *            origin (grid.t_origin).
 * Memory     "device" pointers are HIP device memory on the current device;
 *            "host" pointers are ordinary host memory.  The caller allocates
 *            and owns every buffer, including workspaces; the library never
 *            allocates device memory and keeps no pointer after a call
 *            returns.  The one exception is the fixed scratch array of
 *            cetra_periodic_search_noalloc, a static device array of the
 *            library's own code object.
 * Streams    `stream` is a hipStream_t passed as void* (NULL = the default
 *            stream).  Device work is only enqueued: no entry point
 *            synchronises, so results are ready when the stream is.  No entry
 *            point allocates, frees or synchronises on the device, so the
 *            calls may be captured into a HIP graph.
 * Errors     Every entry point returns a status (CETRA_OK = 0, negative on
 *            failure).  Arguments are validated on the host before anything
 *            is enqueued; on failure nothing is enqueued.  A launch failure is
 *            reported as CETRA_ERR_HIP.  cetra_last_error() gives the
 *            calling thread's last message.  No exception crosses the ABI.
 * Layouts    A resampled light curve is flux[N], ivar[N] (ivar = 1/sigma^2;
 *            0 marks a null point, i.e. infinite uncertainty).  Linear-search
 *            arrays are duration-major [J][I].  The fold-ready array is
 *            float pairs [J][I][2] = (S_fm, S_mm) per element, where
 *            S_fm = sum w f m and S_mm = sum w m^2 over the window.
 * Nulls      A linear element with no usable data (Sec. 2.2, null outputs)
 *            has fold pair (0, 0), depth NaN, variance +inf, LR 0.  A period
 *            with no usable candidate has LR 0, epoch = duration = -1,
 *            depth NaN, variance +inf.
 */
#ifndef CETRA_H
#define CETRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CETRA_VERSION 100
#define CETRA_MAX_DURATIONS 64
#define CETRA_MAX_MODEL 4096

enum cetra_status {
    CETRA_OK = 0,
    CETRA_ERR_INVALID = -1,   /* bad argument (null pointer, bad size, unsorted grid ...) */
    CETRA_ERR_RANGE = -2,     /* a size exceeds what the library supports          */
    CETRA_ERR_WORKSPACE = -3, /* workspace smaller than the size query returned    */
    CETRA_ERR_HIP = -4,       /* a HIP runtime call or kernel launch failed        */
    CETRA_ERR_DEVICE = -5     /* no usable gfx950 device                           */
};

/* Geometry of one search, produced by cetra_grid_plan (host only). */
typedef struct cetra_grid {
    double t_first;   /* time of the first observation (days)                   */
    double cadence;   /* resampled cadence c (days)                             */
    double t_origin;  /* time of resampled point 0 = t_first - n_pad * c        */
    double t0_step;   /* reference-time step dt (days)                          */
    int64_t n_pad;    /* null points padded before the data (and after it)      */
    int64_t n_data;   /* grid points from the first to the last observation     */
    int64_t n;        /* N = n_data + 2 n_pad                                   */
    int64_t n_t0;     /* I: reference times t_i = i * dt, i in [0, I)            */
    int32_t n_dur;    /* J: trial durations                                     */
    int32_t n_model;  /* M: template samples                                    */
    double durations[CETRA_MAX_DURATIONS];    /* ascending, days                */
    uint64_t dur_step_fx[CETRA_MAX_DURATIONS]; /* template samples per grid point, 32.32 fixed point */
} cetra_grid;

/* Best period of a periodogram (written to device memory by cetra_best). */
typedef struct cetra_best_record {
    int64_t k;          /* index of the best period, -1 if every period is null */
    int32_t epoch;      /* reference-time index i* of the best candidate          */
    int32_t dur;        /* duration index j*                                      */
    double period;      /* days                                                   */
    double duration;    /* days                                                   */
    double t0;          /* mid-transit time of the epoch, relative to t_origin     */
    double t0_abs;      /* the same in the input's time system                    */
    double lr;          /* log-likelihood ratio against the constant model        */
    double depth;       /* maximum-likelihood common depth Z                       */
    double depth_var;   /* its variance                                           */
    double snr;         /* depth / sqrt(depth_var)                                */
} cetra_best_record;

/* Most single events one cetra_single_events call returns. */
#define CETRA_MAX_EVENTS 64

/* One single-transit candidate (written to device memory by
 * cetra_single_events). */
typedef struct cetra_event {
    int32_t epoch;      /* reference-time index i, -1 if no candidate remained  */
    int32_t dur;        /* duration index j                                       */
    double t0;          /* mid-transit time relative to t_origin (days)           */
    double t0_abs;      /* the same in the input's time system                    */
    double duration;    /* days                                                   */
    double lr;          /* log-likelihood ratio (Eq. 2 at the best depth)          */
    double depth;       /* maximum-likelihood depth                               */
    double depth_var;   /* its variance                                           */
    double snr;         /* depth / sqrt(depth_var)                                */
} cetra_event;

/* Launch tuning of the periodic search, process-wide for this library
 * instance (an autotuner sets it; the defaults are 8, 8, 4, 2, 4).  Results do
 * not depend on it. */
typedef struct cetra_tuning {
    int32_t fold_period_block;  /* trial periods accumulated per lane: 4, 8 or 16     */
    int32_t fold_wgs_per_cu;    /* resident workgroups per compute unit, 1..32       */
    int32_t fold_units_per_wg;  /* target work units per workgroup, 1..64            */
    int32_t fold_variant;       /* 0: register fold, lane epochs 64 apart;
                                   2: register fold, adjacent lane epochs and
                                      16-byte loads (1, 3 and 4 are retired:
                                      LDS-staged forms that measured slower)   */
    int32_t linear_windows;     /* linear-search windows per lane: 1, 2 or 4 (a
                                   workgroup computes 256 x this many reference
                                   times; results do not depend on it)         */
    int32_t reserved[3];
} cetra_tuning;

/* ---------------------------------------------------------------- service */

/* Library version (CETRA_VERSION). */
int cetra_version(void);

/* Last error message of the calling thread ("" if none).  The pointer stays
 * valid until the thread's next failing call. */
const char *cetra_last_error(void);

/* Static description of a status code. */
const char *cetra_status_string(int status);

/* Current launch tuning (host memory). */
int cetra_get_tuning(cetra_tuning *out);

/* Set the launch tuning (host memory; NULL restores the defaults).  Invalid
 * values are rejected with CETRA_ERR_INVALID and change nothing.  Affects
 * calls enqueued afterwards from any thread. */
int cetra_set_tuning(const cetra_tuning *in);

/* ------------------------------------------------------------------ setup */

/* Grid plan (host only; Sec. 2.1.1 padding and index rule, Sec. 2.1.3 grids).
 * t_first, t_last: first and last observation times (days, t_last >= t_first).
 * cadence: resampled cadence c > 0 (days; the paper's default is the median
 *   input cadence, which the caller computes).
 * durations[n_dur]: trial durations, strictly ascending, 1 <= n_dur <= 64.
 * t0_step: reference-time step; <= 0 selects the paper's default of 1% of the
 *   shortest duration.
 * n_model: template samples M, 1 <= M <= CETRA_MAX_MODEL.
 * The grid has n_pad = ceil(max(D)/2 / c) null points before and after the
 * n_data = floor((t_last - t_first)/c + 1/2) + 1 data points, and
 * I = floor((N-1) c / dt) + 1 reference times.  Fails with CETRA_ERR_RANGE if
 * J * I does not fit 32 bits.  `out` is host memory. */
int cetra_grid_plan(double t_first, double t_last, double cadence, const double *durations,
                    int32_t n_dur, double t0_step, int32_t n_model, cetra_grid *out);

/* Period grid of the default search (Sec. 2.1.3, which adopts the optimally
 * sampled grid of Ofir 2014 as used by TLS).  Frequencies are spaced evenly
 * in f^(1/3): a step moves the last transit of a span of `span` days by
 * 1/oversample of the duty cycle q(f) = (3 pi / (G rho))^(1/3) f^(2/3) / pi
 * of a central transit across a star of mean density `rho` (g cm^-3), i.e.
 * d(f^(1/3)) = (3 pi / (G rho))^(1/3) / (3 pi span oversample).  The grid
 * starts at 1/p_max and covers [p_min, p_max] days.  *n_out (host) receives
 * the number of periods; if `periods` (host) is not NULL it receives them in
 * ascending order and must hold `cap` >= *n_out values (else
 * CETRA_ERR_INVALID).  Invalid ranges fail with CETRA_ERR_INVALID. */
int cetra_period_grid(double span, double p_min, double p_max, double rho, double oversample, double *periods,
                      int64_t cap, int64_t *n_out);

/* Keplerian duration limits for one period (days), the range Sec. 2.1.3
 * keeps per period: circular orbits around stars of mean density
 * [rho_min, rho_max] (g cm^-3), with first-to-last-contact duration
 * T = (P/pi) asin(sqrt((1+k)^2 - b^2) / (a/R sin i)), (a/R)^3 = G rho P^2/(3 pi),
 * cos i = b/(a/R).  *d_max is T at rho_min, radius ratio k_max and b = 0;
 * *d_min is T at rho_max, k = 0 and b = b_max (0 <= k_max, b_max < 1).  An
 * orbit inside the star gives P/2, a non-transiting one 0.  Host only. */
int cetra_duration_limits(double period, double rho_min, double rho_max, double k_max, double b_max,
                          double *d_min, double *d_max);

/* Per-period duration-index ranges for cetra_periodic_search's `jrange`
 * (host arrays): jrange[k] = {first j with durations[j] >= d_min(P_k), last j
 * with durations[j] <= d_max(P_k)} for the limits of cetra_duration_limits
 * (an empty range, lo > hi, when no duration qualifies).  durations[n_dur]
 * ascending, days; periods[n_periods] days.  Host only. */
int cetra_keplerian_jrange(const double *periods, int64_t n_periods, const double *durations, int32_t n_dur,
                           double rho_min, double rho_max, double k_max, double b_max, int32_t *jrange);

/* Template resampling (Sec. 2.1.2): the dense template dense[n_dense]
 * (device, FP64, contact-normalised time from first to last contact, max
 * offset 1) is resampled by linear interpolation to model[n_model] (device,
 * FP32) at the cell centres tau_k = (k + 1/2)/M.  n_dense >= 2. */
int cetra_template_resample(void *stream, const double *dense, int64_t n_dense, int32_t n_model,
                            float *model);

/* Resampling onto the regular grid (Sec. 2.1.1).  t[n_obs] (device, FP64,
 * non-decreasing), f[n_obs] (device, FP32 flux offsets) and sigma[n_obs]
 * (device, FP32) are binned to the nearest grid point,
 * q = n_pad + floor((t - t_first)/c + 1/2); co-located points are combined by
 * their inverse-variance weighted mean.  Outputs flux[N], ivar[N] (device,
 * FP32; ivar = sum of sigma^-2, 0 for a null point).  Observations with a
 * non-finite f or sigma, or sigma <= 0, count as missing.  If `status`
 * (device int32, may be NULL) is given it is set to 0, or to 1 if t is not
 * non-decreasing or not finite (the output is then undefined). */
int cetra_resample(void *stream, const cetra_grid *grid, const double *t, const float *f,
                   const float *sigma, int64_t n_obs, float *flux, float *ivar, int32_t *status);

/* ----------------------------------------------------------- linear search */

/* Linear search (Sec. 2.2).  For every reference time i and duration j the
 * window [t_i - D_j/2, t_i + D_j/2] covers grid points ceil(t_s/c) ..
 * floor(t_e/c); each point is compared with the nearest template sample
 * (32.32 fixed-point index, clamped to M-1).  The maximum-likelihood depth is
 * the inverse-variance weighted mean of f/m, its variance the reciprocal of
 * the summed weights, and the likelihood ratio against the constant model
 * (Eq. 2) equals S_fm^2 / (2 S_mm).  A window that leaves [0, (N-1) c] or
 * holds no data is null.
 * flux, ivar[N], model[M] (device) in; fold[J][I][2] (device, required) out;
 * depth, var, lr [J][I] (device) are optional (NULL to skip). */
int cetra_linear_search(void *stream, const cetra_grid *grid, const float *flux, const float *ivar,
                        const float *model, float *fold, float *depth, float *var, float *lr);

/* Log-likelihood of the constant (zero-offset) model over the non-null grid
 * points (Eq. 1 at zero depth; Sec. 2.2 and Sec. 2.3 note that adding it to a
 * likelihood ratio gives the full log-likelihood).  out: one double (device). */
int cetra_loglike0(void *stream, const cetra_grid *grid, const float *flux, const float *ivar,
                   double *out);

/* --------------------------------------------------------- periodic search */

/* Workspace bytes for cetra_periodic_search over n_eval periods (host only). */
int cetra_periodic_workspace(const cetra_grid *grid, int64_t n_eval, size_t *bytes);

/* Periodic search (Sec. 2.3).  For each evaluated period P_k every epoch
 * i in [0, ceil(P_k/dt)) and allowed duration j (D_j < P_k, and j inside
 * jrange[k] if given) combines the single-transit elements at
 * i + round(m P_k/dt), m = 0, 1, ... (nearest reference time) with a common
 * inverse-variance depth Z; its likelihood ratio, the sum of Eq. 4 over the
 * transits, equals (sum S_fm)^2 / (2 sum S_mm).  The maximum over (j, i) is
 * kept, ties going to the smallest j, then the smallest i; candidates are
 * ranked on FP32 sums (two whose LR agree to within a few 1e-6 relative may
 * be taken in either order) and the winner's record is recomputed in FP64.
 * fold[J][I][2] (device) from cetra_linear_search.
 * periods[n_periods] (device, FP64, days; ascending order gives the best
 *   performance but is not required).  A period shorter than the
 *   reference-time step, or not finite, gets the null record.
 * jrange: NULL, or device int32 [n_periods][2] inclusive duration-index range.
 * subset: NULL to evaluate every period, else device int64 [n_subset] period
 *   indices to evaluate (the others get the null record).
 * work/work_bytes: device workspace of at least
 *   cetra_periodic_workspace(grid, n_subset or n_periods) bytes.
 * Outputs (device, [n_periods]): lr (FP32), epoch (int32 i*), dur (int32 j*),
 *   depth (FP32 Z), depth_var (FP32 1/sum S_mm). */
int cetra_periodic_search(void *stream, const cetra_grid *grid, const float *fold,
                          const double *periods, int64_t n_periods, const int32_t *jrange,
                          const int64_t *subset, int64_t n_subset, void *work, size_t work_bytes,
                          float *lr, int32_t *epoch, int32_t *dur, float *depth, float *depth_var);

/* Periodic search without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, outputs, kernels and
 * results as cetra_periodic_search, except that the fold workspace is a
 * fixed 16 MiB device array inside the library (one per device, kept until
 * the process ends; its address is resolved once per device at the first
 * call).  Nothing is allocated or freed.  Every evaluated period's argmax key
 * and table entry is rewritten by each call, so nothing carries over from
 * the previous call; but all calls on one device share the array, so calls
 * that overlap on one device (concurrent streams or host threads) race and
 * must be serialised by the caller.  More evaluated periods than
 * cetra_periodic_search_noalloc_limit reports returns CETRA_ERR_RANGE with
 * nothing enqueued. */
int cetra_periodic_search_noalloc(void *stream, const cetra_grid *grid, const float *fold,
                                  const double *periods, int64_t n_periods, const int32_t *jrange,
                                  const int64_t *subset, int64_t n_subset, float *lr, int32_t *epoch,
                                  int32_t *dur, float *depth, float *depth_var);

/* Largest number of evaluated periods cetra_periodic_search_noalloc accepts
 * (host only; *max_eval out). */
int cetra_periodic_search_noalloc_limit(const cetra_grid *grid, int64_t *max_eval);

/* Fold epoch strides for a reference-time step that grows with the duration,
 * the TLS grid that Sec. 2.1.3 mentions adopting (the paper itself keeps one
 * step): on the fixed grid of step dt, stride[j] = max(1, floor(fraction *
 * D_j / dt + 1e-9)), the largest whole number of steps not above `fraction`
 * of D_j (the 1e-9 keeps whole multiples from landing one short).
 * stride[n_dur] (host) out.  fraction must be finite and > 0, else
 * CETRA_ERR_INVALID.  Host only. */
int cetra_epoch_strides(const cetra_grid *grid, double fraction, int32_t *stride);

/* cetra_periodic_search on a coarser epoch grid per duration: duration j
 * evaluates only the epochs i that are multiples of stride[j] (host int32
 * [n_dur], each >= 1, else CETRA_ERR_INVALID; NULL evaluates every epoch,
 * as cetra_periodic_search does).  Transits stay at i + round(m P_k/dt) on the
 * fixed grid, so every record is the plain search's value at the (i*, j*) it
 * reports, and the fold visits about 1/stride[j] of duration j's elements.
 * Other arguments, outputs and workspace as cetra_periodic_search. */
int cetra_periodic_search_strided(void *stream, const cetra_grid *grid, const float *fold,
                                  const double *periods, int64_t n_periods, const int32_t *jrange,
                                  const int64_t *subset, int64_t n_subset, const int32_t *stride,
                                  void *work, size_t work_bytes, float *lr, int32_t *epoch, int32_t *dur,
                                  float *depth, float *depth_var);

/* Best period of a periodogram (Sec. 2.3 outputs): the maximum LR over the
 * n_periods records (ties to the smallest index), with SNR = Z / sqrt(var_Z)
 * and the epoch converted to time.  Inputs are the device outputs of
 * cetra_periodic_search; `out` is one cetra_best_record in device memory. */
int cetra_best(void *stream, const cetra_grid *grid, const double *periods, int64_t n_periods,
               const float *lr, const int32_t *epoch, const int32_t *dur, const float *depth,
               const float *depth_var, cetra_best_record *out);

/* Single-event (monotransit) search on the linear search's results (the
 * search for single transits in the linear output that Sec. 1 and Sec. 5
 * describe).  Event e is the element (j, i) of fold[J][I][2] (device, from
 * cetra_linear_search) with the largest likelihood ratio
 * LR = S_fm^2 / (2 S_mm) among the non-null elements whose transit window
 * overlaps none of events 0..e-1 (|t_i - t_e| < (D_j + D_e) / 2 excludes
 * it); candidates are ranked on FP32 and the winner's record is computed
 * in FP64 from its pair, ties going to the smallest j, then i.  out[n_events]
 * (device) receives the events in order; once no candidate remains the rest
 * have epoch -1.  1 <= n_events <= CETRA_MAX_EVENTS.  work/work_bytes: device
 * workspace of cetra_single_events_workspace(n_events) bytes. */
int cetra_single_events_workspace(int32_t n_events, size_t *bytes);
int cetra_single_events(void *stream, const cetra_grid *grid, const float *fold, int32_t n_events, void *work,
                        size_t work_bytes, cetra_event *out);

/* Per-period merge of n_sets period searches stacked set after set (device
 * arrays [n_sets][n_periods], as cetra_periodic_search writes them), e.g.
 * one per template when searching across a sequence of impact parameters
 * (Sec. 2.1.2): each output period takes the record of the set with the
 * largest LR (ties: the smaller set index); null records (epoch -1) never
 * win over a valid one, and a period null in every set stays null.
 * out_set[k] (device int32) is the winning set, -1 if none. */
int cetra_periodic_merge(void *stream, int32_t n_sets, int64_t n_periods, const float *lr, const int32_t *epoch,
                         const int32_t *dur, const float *depth, const float *depth_var, float *out_lr,
                         int32_t *out_epoch, int32_t *out_dur, float *out_depth, float *out_depth_var,
                         int32_t *out_set);

/* Nulls a found signal for the next search (the iterative search of Sec. 5,
 * which nullifies the flux in and around the strongest signal before
 * searching again): every resampled point q (time q c after t_origin) with
 * |q c - t0 - n P| <= width * duration / 2 for the nearest integer n gets
 * flux = ivar = 0 (device arrays [N] from cetra_resample).  A period that is
 * not a finite positive number nulls the single event at t0 only.  t0 is
 * relative to t_origin (as in cetra_best_record and cetra_event). */
int cetra_mask_transits(void *stream, const cetra_grid *grid, double period, double t0, double duration,
                        double width, float *flux, float *ivar);

/* ------------------------------------------------------------- autotuner */

/* Shape class of a search, the key of the autotuner's cache. */
typedef struct cetra_shape_class {
    char arch[32];          /* GPU architecture ("gfx950"); empty = the current device's */
    int32_t log2_t0;        /* ceil(log2(I))                                           */
    int32_t n_dur;          /* J                                                        */
    int32_t log2_periods;   /* ceil(log2(K))                                           */
    int32_t reserved;
} cetra_shape_class;

/* Shape class of a grid and a period count (host only; arch left empty). */
int cetra_shape_class_of(const cetra_grid *grid, int64_t n_periods, cetra_shape_class *out);

/* Device workspace bytes cetra_autotune needs for this grid and period count
 * (host only). */
int cetra_autotune_workspace(const cetra_grid *grid, int64_t n_periods, size_t *bytes);

/* Launch autotuner.  If cache_path (nullable) names a JSON cache holding an
 * entry for shape's architecture and class, that tuning is applied
 * (cetra_set_tuning) and returned with *from_cache = 1: no device work, no
 * synchronisation.  Otherwise the candidates are timed with HIP events on
 * `stream` on the caller's data: the linear search under 1, 2 and 4 windows
 * per lane (flux, ivar, model as for cetra_linear_search; fold[J][I][2] is
 * overwritten with the same values each time), then the periodic search
 * under period blocks 4/8/16 x workgroups per CU 2/4/8 x units per workgroup
 * 2/4/8 x fold variants 0/2 over a contiguous slice of periods[n_periods]
 * (device) from the middle of the grid, sized to about 5e11 algorithmic
 * bytes.  The fastest of each is applied and returned (*from_cache = 0,
 * times in ms through fold_ms / linear_ms, nullable), and written to the
 * cache (entries of other classes are kept; the file is replaced
 * atomically).  work: device workspace of cetra_autotune_workspace bytes.
 * This call synchronises the stream (a set-up step, not capturable).
 * Results of the search do not depend on the tuning. */
int cetra_autotune(void *stream, const cetra_shape_class *shape, const cetra_grid *grid,
                   const float *flux, const float *ivar, const float *model, float *fold,
                   const double *periods, int64_t n_periods, void *work, size_t work_bytes,
                   const char *cache_path, cetra_tuning *out, double *fold_ms, double *linear_ms,
                   int32_t *from_cache);

/* ---------------------------------------------------------- batched search */

/* A batch of light curves searched by one persistent launch that drains a
 * work queue (the per-curve method is Sec. 2.1-2.3 unchanged; batching is
 * this library's addition).  Curves share the durations and template size;
 * each has its own grid plan, observations and period grid, concatenated
 * (CSR) in device arrays. */
typedef struct cetra_batch_desc {
    int32_t n_curves;              /* >= 1                                           */
    int32_t fold_period_block;     /* periods per fold lane block: 4 or 8, 0 = the
                                      library tuning's (if that is 16, 8)              */
    const cetra_grid *grids;       /* host [n_curves]: cetra_grid_plan of each curve;
                                      all with the same n_dur, durations and n_model    */
    const int64_t *obs_offsets;    /* host [n_curves + 1], starting at 0: curve c's
                                      observations are t/f/sigma[obs_offsets[c] ..
                                      obs_offsets[c+1])                                 */
    const int64_t *period_offsets; /* host [n_curves + 1], starting at 0: the same for
                                      periods and for the per-period outputs            */
    int64_t shuffle_seed;          /* 0: curves queued by descending fold cost; else a
                                      permutation drawn from this seed (results do not
                                      depend on the order)                              */
    int32_t pop_items;             /* work items a workgroup takes per pop of the
                                      queue, 1-64; 0 = chosen at launch (up to 8, fewer
                                      when the batch is small).  Results do not depend
                                      on it                                            */
    int32_t reserved1;
} cetra_batch_desc;

typedef struct cetra_batch_info {
    size_t workspace_bytes;  /* device workspace cetra_batch_search needs          */
    size_t tables_bytes;     /* leading workspace bytes that hold the plan's tables */
    int64_t n_curves;
    int64_t total_periods;
    int64_t n_launches;      /* kernel launches per cetra_batch_search (2)         */
    int64_t n_items;         /* work-queue items of one search                     */
    int32_t n_slots;         /* curves whose device slots are live at once          */
    int32_t period_block;
    int32_t lds_bytes;       /* dynamic LDS per workgroup of the persistent kernel */
    int32_t reserved;
} cetra_batch_info;

/* Flags of cetra_batch_search. */
#define CETRA_BATCH_RESUME 1      /* skip curves whose done flag is already set       */

/* Device status bits written by cetra_batch_search (0 = every curve searched). */
#define CETRA_BATCH_CANCELLED 1   /* the cancel flag stopped the launch early          */
#define CETRA_BATCH_WAIT_LIMIT 2  /* a dependency wait exceeded 30 s (results invalid)  */
#define CETRA_BATCH_BAD_TABLES 4  /* the workspace does not hold this plan's tables    */
#define CETRA_BATCH_UNSORTED 8    /* some curve's times were not finite and ascending  */

/* Opaque host-side plan. */
typedef struct cetra_batch_plan cetra_batch_plan;

/* Plan a batch (host only): validates the grids and offsets, orders the
 * curves (descending fold cost = sum over periods of allowed durations times
 * reference times, or a seeded shuffle), cuts every curve's stages into work
 * items (resampling, linear search, fold units, decode), groups consecutive
 * curves until a group's fold has enough items (a long curve is a group of
 * one), and lays out the queue so that each item's inputs come from items
 * queued before it: group g+2's resampling and linear search and group g-3's
 * decode are queued around group g's fold.  Each curve has a device slot
 * (resampled curve, fold-ready array, per-period table); min(8, groups) slot
 * sets are reused in queue order.  The plan
 * owns host memory only; free it with cetra_batch_plan_destroy. */
int cetra_batch_plan_create(const cetra_batch_desc *desc, cetra_batch_plan **out);
int cetra_batch_plan_destroy(cetra_batch_plan *plan);
int cetra_batch_plan_info(const cetra_batch_plan *plan, cetra_batch_info *info);
/* The queue order of the curves (host int32 [n], n = number of curves). */
int cetra_batch_plan_order(const cetra_batch_plan *plan, int32_t *order, int32_t n);

/* Device workspace of cetra_batch_search (host only): *bytes in all, of which
 * the first *tables_bytes (nullable) must hold the plan's tables image. */
int cetra_batch_workspace(const cetra_batch_plan *plan, size_t *bytes, size_t *tables_bytes);

/* Copies the plan's tables image (tables_bytes) to host memory; the caller
 * copies it once to the start of the device workspace before the first
 * search with that workspace (searches only read it). */
int cetra_batch_tables(const cetra_batch_plan *plan, void *host_dst, size_t bytes);

/* A cancel flag for the plan's searches in pinned host memory allocated by
 * this call on first use (hipHostMalloc) and freed by
 * cetra_batch_plan_destroy: writing a non-zero value while a search runs
 * stops it early (CETRA_BATCH_CANCELLED).  Searches poll it when their
 * cancel argument is NULL. */
int cetra_batch_cancel_flag(cetra_batch_plan *plan, int32_t **flag);

/* Search every curve of the batch: two launches on `stream`, a small kernel
 * that clears the counters (and the done flags, unless resuming), then one
 * persistent grid whose workgroups pop work items from an atomic counter in
 * queue order, wait for the items they depend on (acquire/release counters
 * per curve and stage), and run the same per-item code as the single-curve
 * calls, so every curve's records are bit-identical to cetra_resample +
 * cetra_linear_search + cetra_periodic_search + cetra_best on that curve.
 * Nothing is allocated and nothing synchronises, so the call can be
 * captured in a HIP graph and replayed.
 * t, f, sigma: device CSR observations (each curve's times finite and
 *   ascending; a curve that is not gets done = -1, undefined records and
 *   CETRA_BATCH_UNSORTED).  model[M]: device template.  periods: device CSR.
 * jrange: NULL, or device int32 [total periods][2] (CSR like the periods):
 *   each period's inclusive duration-index range, as cetra_periodic_search.
 * cancel: NULL (then the plan's flag, if cetra_batch_cancel_flag made one), or
 *   an int32 in device memory or pinned host memory, polled as items are
 *   taken; non-zero stops the launch after the items in progress.
 * flags: 0 or CETRA_BATCH_RESUME (curves with done[c] != 0 are skipped and
 *   keep their earlier outputs).
 * work: device workspace of cetra_batch_workspace bytes holding the tables.
 * Outputs: per-period lr, epoch, dur, depth, depth_var (device, CSR like the
 * periods), best[n_curves] (device; a curve without periods gets the null
 * record), done[n_curves] (device int32: 1 searched, -1 searched on unsorted
 * input, 0 not reached), status (device int32, CETRA_BATCH_* bits). */
int cetra_batch_search(const cetra_batch_plan *plan, void *stream, const double *t, const float *f,
                       const float *sigma, const float *model, const double *periods,
                       const int32_t *jrange, const int32_t *cancel, int32_t flags, void *work,
                       size_t work_bytes, float *lr,
                       int32_t *epoch, int32_t *dur, float *depth, float *depth_var,
                       cetra_best_record *best, int32_t *done, int32_t *status);

/* ------------------------------------------------------------------------
 * Period-window proposal network (an addition, not part of the paper).
 *
 * A small 1-D convolutional network reads the linear search's single-event
 * statistics (Sec. 2.2), downsampled to L bins, and scores W log-spaced
 * period windows; the periodic search (Sec. 2.3) then folds only the periods
 * of the K best-scored windows (cetra_periodic_search's subset argument).
 * The calls below are the network's forward and backward stages and its
 * optimiser, so that training and inference run on the device; the host
 * only sequences them.  Conventions:
 *   bf16   device buffers of IEEE bfloat16 values (passed as void*)
 *   x      input [batch][L][16] bf16 (channel-last; channels = durations)
 *   h      trunk activations [batch][L][64] bf16 (after ReLU)
 *   conv weights, packed: [64][k32] bf16, element (co, tap*cin + ci) is
 *          W[co][ci][tap] of the cross-correlation y[t] = sum W x[t+tap-4]
 *          (zero padding 4), k32 = 9*cin rounded up to a multiple of 32,
 *          padding columns zero (tap-major, channel-minor; FP32 masters and
 *          weight gradients use the same [64][k32] layout)
 *   e      event channels [batch][L][E] FP32, E <= 16 (linear projection)
 *   f      window features [batch][W][E+1] FP32 = (best fold score per
 *          channel, window position q in [0, 1])
 *   z      logits [batch][W]
 * Gradient outputs named d* / g* that are parameters accumulate (+=): the
 * caller clears them before each step; activation gradients are overwritten.
 * Every call only enqueues work on `stream`; errors as for the other calls.
 * ---------------------------------------------------------------------- */

/* One v_mfma_f32_16x16x32_bf16: c[16][16] (FP32) = a[16][32] b[32][16]
 * (bf16, row-major); pins the operand layout the convolutions assume. */
int cetra_net_mfma_probe(void *stream, const void *a, const void *b, float *c);

/* x[bin][j] (bf16) = min(sqrt(max over the bin's reference times of
 * S_fm^2 / S_mm), 30) / 8 from a fold-ready array [n_dur][n_t0][2] (device);
 * bins split the reference times evenly (bin b covers i in
 * [b n_t0 / n_bins, (b+1) n_t0 / n_bins)).  x is [n_bins][n_dur]. */
int cetra_net_downsample(void *stream, const float *fold, int32_t n_dur, int64_t n_t0, int32_t n_bins, void *x);

/* The signed form of the same input: x[bin][j] (bf16) = clamp(z, -30, 30) / 8
 * with z the largest S_fm / sqrt(S_mm) over the bin's reference times (the
 * single-event depth over its error, Sec. 2.2, keeping its sign: a dimming is
 * positive); a bin whose elements are all null gives 0.  Same layout, bins and
 * errors as cetra_net_downsample. */
int cetra_net_downsample_signed(void *stream, const float *fold, int32_t n_dur, int64_t n_t0, int32_t n_bins,
                                void *x);

/* y = relu(conv(x, w) + bias): x [batch][L][cin] bf16 (cin 16 or 64),
 * w packed bf16, bias[64] FP32, y [batch][L][64] bf16.  MFMA implicit GEMM. */
int cetra_conv1d_fwd(void *stream, const void *x, int32_t cin, int32_t L, int32_t batch, const void *w,
                     int32_t k32, const float *bias, void *y);

/* Backward of cetra_conv1d_fwd given dy [batch][L][64] FP32 (gradient of the
 * post-ReLU output y): dw [64][k32] FP32 and db[64] accumulate; dx
 * [batch][L][cin] FP32 is overwritten (dx = NULL skips it).  Scratch:
 * g_scratch batch*L*64 bf16, wt_scratch 64*9*cin bf16 (device).
 * dw_partial (device FP32, 16-byte aligned, dw_partial_floats >=
 * cetra_conv1d_bwd_partial_floats(cin, L, batch), else CETRA_ERR_INVALID):
 * each weight-gradient workgroup stores its sums there and a second kernel
 * adds them into dw and db in a fixed order, so the gradients do not depend
 * on timing.  dw_partial = NULL adds them with FP32 atomics instead (no
 * workspace; the order of the additions, and so the rounding, may vary). */
int cetra_conv1d_bwd(void *stream, const float *dy, const void *y, const void *x, int32_t cin, int32_t L,
                     int32_t batch, const void *w, int32_t k32, void *g_scratch, void *wt_scratch,
                     float *dw_partial, int64_t dw_partial_floats, float *dx, float *dw, float *db);

/* Floats of the dw_partial workspace of cetra_conv1d_bwd for these sizes
 * (-1 for sizes it rejects).  Host only. */
int64_t cetra_conv1d_bwd_partial_floats(int32_t cin, int32_t L, int32_t batch);

/* e[pos][c] = P[c][:] . h[pos][:] + p[c] over n_pos = batch*L positions;
 * P [E][64], p[E] FP32. */
int cetra_net_project_fwd(void *stream, const void *h, int64_t n_pos, const float *P, const float *p, int32_t E,
                          float *e);
/* Backward of the projection given ge [n_pos][E]: dh [n_pos][64] FP32
 * (overwritten; 16-byte aligned, else CETRA_ERR_INVALID), dP [E][64] and
 * dp[E] accumulate.  n_pos <= 2^31. */
int cetra_net_project_bwd(void *stream, const void *h, const float *ge, int64_t n_pos, const float *P, int32_t E,
                          float *dh, float *dP, float *dp);

/* Fold pooling: a coarse version of the periodic search on the event series.
 * For window w and trial t < S, T = trials[w][t] bins (device FP64 [W][S];
 * a trial that is not finite or shorter than one bin is skipped) has the
 * 32.32 step R = floor(2^32 T + 1/2); each phase phi < min(L, ceil(R/2^32))
 * sums e over the positions phi + ((k R + 2^31) >> 32) < L (the nearest-
 * epoch rule of Sec. 2.3 at bin resolution) and scores sum / sqrt(count).
 * f [B][W][E+1]: the maximum score over the window's trials and phases per
 * channel (ties: first trial, then smallest phase), then win_q[w];
 * arg [B][W][E] = trial * 65536 + phase (-1 if no trial is valid, feature 0).
 * e [B][L][E] FP32 (channel-last), L <= 8192, E <= 16, S <= 32. */
int cetra_net_foldpool_fwd(void *stream, const float *e, int32_t B, int32_t L, int32_t E, const double *trials,
                           int32_t W, int32_t S, const float *win_q, float *f, int32_t *arg);
/* Backward of the fold pooling: ge [B][L][E] (overwritten) collects
 * gf[b][w][c] / sqrt(count) at every position of each window's winner. */
int cetra_net_foldpool_bwd(void *stream, const float *gf, const int32_t *arg, const double *trials, int32_t B,
                           int32_t L, int32_t E, int32_t W, int32_t S, float *ge);

/* z = v . relu(U f + u) + v0 per (example, window); U [H][nf], H <= 128,
 * nf = E+1. */
int cetra_net_head_fwd(void *stream, const float *f, int64_t n_bw, int32_t nf, const float *U, const float *u,
                       const float *v, const float *v0, int32_t H, float *z);
/* Weighted binary cross-entropy with logits, mean over the n logits:
 * loss[0] += value (device), gz = d loss / d z (overwritten); labels y in
 * {0, 1}, positives weighted by pos_weight. */
int cetra_net_bce(void *stream, const float *z, const float *y, int64_t n, float pos_weight, float *gz,
                  float *loss);
/* Head backward: gU, gu, gv, gv0 accumulate; gf [n_bw][nf] overwritten. */
int cetra_net_head_bwd(void *stream, const float *f, int64_t n_bw, int32_t nf, const float *U, const float *u,
                       const float *v, int32_t H, const float *gz, float *gU, float *gu, float *gv, float *gv0,
                       float *gf);
/* One Adam step (bias-corrected, step >= 1) on n FP32 parameters p with
 * gradient g and moments m, v (device, updated in place). */
int cetra_adam_step(void *stream, float *p, const float *g, float *m, float *v, int64_t n, float lr, float beta1,
                    float beta2, float eps, int64_t step);
/* Packed bf16 conv weights (layout above) from FP32 masters w [64][k32] in
 * the same layout (padding columns are written as zero whatever w holds). */
int cetra_net_pack_conv_w(void *stream, const float *w, int32_t cin, int32_t k32, void *out);

/* out[b][r] = index of the window with the r-th largest score of example b
 * (ties: smaller index first); 1 <= K <= W <= 1024. */
int cetra_topk_windows(void *stream, const float *scores, int32_t B, int32_t W, int32_t K, int32_t *out);
/* Ascending indices k of the periods[K] (device, ascending) that fall in a
 * selected window, edges[w] <= P < edges[w+1] (edges: device double[W+1],
 * ascending; W <= 4096); sel[n_sel] device window indices (out-of-range
 * entries ignored).  subset must hold K entries; *n_out (device) = count.
 * The result is cetra_periodic_search's subset argument. */
int cetra_windows_to_periods(void *stream, const double *periods, int64_t K, const double *edges, int32_t W,
                             const int32_t *sel, int32_t n_sel, int64_t *subset, int64_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* CETRA_H */
