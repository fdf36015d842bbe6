/*
 * FP64 CPU oracle for the two-stage transit search (linear search, then
 * periodic search) of Smith et al. 2025, "CETRA" (arXiv:2503.20875).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition that the
 * GPU library is checked against.  Only the test suite, the package's smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU library
 * never calls it and shares no code, header, table or constant with it.
 *
 * Everything is IEEE FP64 (compiled without FMA contraction or fast-math).
 * Index rules that the paper leaves open are evaluated exactly as written in
 * the comments below ("reading"), as plain FP64 operations followed by
 * integer arithmetic.
 *
 * Layout conventions of this oracle:
 *   resampled light curve   flux[N], ivar[N]          (ivar = 1/sigma^2, 0 = null)
 *   linear-search outputs   depth/var/lr/aabs [J][I]  (duration-major)
 *   null linear element     depth = NaN, var = +inf, lr = 0, aabs = 0
 *   null periodic record    lr = 0, i = j = -1, z = NaN, zvar = +inf
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAX_DUR 64
#define TWO32 4294967296.0

typedef struct {
    double t_first;   /* time of the first observation (days)            */
    double cadence;   /* resampled cadence c (days)                      */
    double t_origin;  /* time of resampled point 0 = t_first - n_pad*c   */
    double t0_step;   /* reference-time step dt (days)                   */
    int64_t n_pad;    /* null points padded at each end                  */
    int64_t n_data;   /* points from first to last observation           */
    int64_t n;        /* N = n_data + 2 n_pad                            */
    int64_t n_t0;     /* I, number of reference times                    */
    int32_t n_dur;    /* J                                               */
    int32_t n_model;  /* M, template samples                             */
    double durations[ORA_MAX_DUR];
    uint64_t dur_step_fx[ORA_MAX_DUR]; /* template samples per grid point, 32.32 */
} ora_grid;

void ora_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ora_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Grids (Sec. 2.1.1 padding, Sec. 2.1.3 reference-time grid).
 * Reading: the resampled grid starts n_pad = ceil(max(D)/2 / c) points before
 * the first observation and ends n_pad points after the grid point nearest
 * the last observation.  Reference times t_i = i*dt (relative to the grid
 * origin) are transit mid-points, dt = frac * min(D) by default, and span
 * [0, (N-1) c].  Returns 0 on success, -1 on invalid input. */
int ora_grid_plan(double t_first, double t_last, double cadence, const double *durations,
                  int32_t n_dur, double t0_step, int32_t n_model, ora_grid *g) {
    if (!(cadence > 0.0) || n_dur < 1 || n_dur > ORA_MAX_DUR || n_model < 1 || !(t_last >= t_first))
        return -1;
    for (int j = 0; j < n_dur; ++j) {
        if (!(durations[j] > 0.0)) return -1;
        if (j > 0 && !(durations[j] > durations[j - 1])) return -1;
    }
    memset(g, 0, sizeof(*g));
    double dmax = durations[n_dur - 1];
    double dmin = durations[0];
    g->t_first = t_first;
    g->cadence = cadence;
    g->n_pad = (int64_t)ceil((dmax / 2.0) / cadence);
    g->n_data = (int64_t)floor((t_last - t_first) / cadence + 0.5) + 1;
    g->n = g->n_data + 2 * g->n_pad;
    g->t_origin = t_first - (double)g->n_pad * cadence;
    g->t0_step = (t0_step > 0.0) ? t0_step : 0.01 * dmin;
    g->n_t0 = (int64_t)floor((double)(g->n - 1) * cadence / g->t0_step) + 1;
    g->n_dur = n_dur;
    g->n_model = n_model;
    for (int j = 0; j < n_dur; ++j) {
        g->durations[j] = durations[j];
        g->dur_step_fx[j] = (uint64_t)llround(TWO32 * (((double)n_model * cadence) / durations[j]));
    }
    return 0;
}

/* Template resampling (Sec. 2.1.2): the dense template is resampled to M
 * samples by linear interpolation.  Reading: sample k sits at the centre of
 * the k-th of M equal cells of contact-normalised time, tau_k = (k + 1/2)/M,
 * and the dense samples are equally spaced over [0, 1].  Output rounded to
 * FP32 once (it is the FP32 table the search reads). */
void ora_template(const double *dense, int64_t n_dense, int32_t n_model, float *model) {
    for (int32_t k = 0; k < n_model; ++k) {
        double tau = ((double)k + 0.5) / (double)n_model;
        double x = tau * (double)(n_dense - 1);
        int64_t a = (int64_t)floor(x);
        if (a >= n_dense - 1) a = n_dense - 2;
        if (a < 0) a = 0;
        double fr = x - (double)a;
        double v = dense[a] + fr * (dense[a + 1] - dense[a]);
        model[k] = (float)v;
    }
}

/* Resampling (Sec. 2.1.1): every observation goes to the nearest grid point;
 * co-located observations are combined by their inverse-variance weighted
 * mean and formal uncertainty (sigma = (sum sigma^-2)^-1/2); grid points with
 * no observation are null (infinite sigma, stored as ivar = 0, flux 0).
 * Reading: nearest point by round-half-up, q = n_pad + floor((t-t_first)/c + 1/2);
 * observations with non-finite t, f or sigma, or sigma <= 0, are missing. */
void ora_resample(const ora_grid *g, const double *t, const float *f, const float *sigma,
                  int64_t n_obs, double *flux, double *ivar) {
    double *wsum = (double *)calloc((size_t)g->n, sizeof(double));
    double *fsum = (double *)calloc((size_t)g->n, sizeof(double));
    for (int64_t n = 0; n < n_obs; ++n) {
        double tn = t[n], fn = (double)f[n], sn = (double)sigma[n];
        if (!isfinite(tn) || !isfinite(fn) || !isfinite(sn) || !(sn > 0.0)) continue;
        int64_t q = g->n_pad + (int64_t)floor((tn - g->t_first) / g->cadence + 0.5);
        if (q < 0 || q >= g->n) continue;
        double w = 1.0 / (sn * sn);
        wsum[q] += w;
        fsum[q] += w * fn;
    }
    for (int64_t q = 0; q < g->n; ++q) {
        if (wsum[q] > 0.0) {
            flux[q] = fsum[q] / wsum[q];
            ivar[q] = wsum[q];
        } else {
            flux[q] = 0.0;
            ivar[q] = 0.0;
        }
    }
    free(wsum);
    free(fsum);
}

/* Transit window of reference time i and duration j (Sec. 2.1.1 index rule,
 * Sec. 2.2).  Reading: the window is [t_i - D/2, t_i + D/2]; its first and
 * last grid points are ceil(t_s/c) and floor(t_e/c); a window that leaves
 * [0, (N-1)c] is null.  The template sample for grid point n_lo + q is
 * floor(tau*M) (nearest cell centre), tau = (n*c - t_s)/D, evaluated in 32.32
 * fixed point: phase = llround(2^32 * ((n_lo*c - t_s)/D * M)) (clamped at 0),
 * k = min(M-1, (phase + q*G_j) >> 32) with G_j = llround(2^32 * M*c/D_j).
 * Returns 0 if null, else 1 and fills n_lo, n_hi, phase. */
static int window(const ora_grid *g, int64_t i, int j, int64_t *n_lo, int64_t *n_hi, int64_t *phase) {
    double c = g->cadence;
    double d = g->durations[j];
    double ts = (double)i * g->t0_step - 0.5 * d;
    double te = ts + d;
    if (ts < 0.0 || te > (double)(g->n - 1) * c) return 0;
    *n_lo = (int64_t)ceil(ts / c);
    *n_hi = (int64_t)floor(te / c);
    if (*n_lo > *n_hi) return 0;
    int64_t ph = llround(TWO32 * ((((double)(*n_lo) * c - ts) / d) * (double)g->n_model));
    *phase = ph < 0 ? 0 : ph;
    return 1;
}

static int template_index(const ora_grid *g, int j, int64_t phase, int64_t q) {
    uint64_t fx = (uint64_t)phase + (uint64_t)q * g->dur_step_fx[j];
    uint64_t k = fx >> 32;
    if (k > (uint64_t)(g->n_model - 1)) k = (uint64_t)(g->n_model - 1);
    return (int)k;
}

/* One element of the linear search (Sec. 2.2).
 * Pass 1: each point gives a depth estimate f_n/m_n with uncertainty
 * sigma_n/m_n; the maximum-likelihood depth is their inverse-variance
 * weighted mean and its variance is the reciprocal of the sum of weights.
 * Pass 2: the likelihood ratio against the constant (zero-offset) model over
 * the window only (Eq. 2), as a log-likelihood difference.
 * aabs = sum over the window of w |f| m (used only to scale parity errors). */
static void linear_one(const ora_grid *g, const double *flux, const double *ivar, const float *model,
                       int64_t i, int j, double *depth, double *var, double *lr, double *aabs) {
    int64_t n_lo, n_hi, phase;
    *depth = NAN;
    *var = INFINITY;
    *lr = 0.0;
    *aabs = 0.0;
    if (!window(g, i, j, &n_lo, &n_hi, &phase)) return;
    /* pass 1 */
    double sum_u = 0.0, sum_ud = 0.0, sum_abs = 0.0;
    for (int64_t n = n_lo; n <= n_hi; ++n) {
        double w = ivar[n];
        double m = (double)model[template_index(g, j, phase, n - n_lo)];
        if (w <= 0.0 || m == 0.0) continue;
        double dn = flux[n] / m;          /* depth implied by this point   */
        double un = w * m * m;            /* 1 / (sigma_n / m_n)^2         */
        sum_u += un;
        sum_ud += un * dn;
        sum_abs += w * fabs(flux[n]) * fabs(m);
    }
    if (!(sum_u > 0.0)) return;
    double dep = sum_ud / sum_u;
    /* pass 2: Eq. 2 */
    double l = 0.0;
    for (int64_t n = n_lo; n <= n_hi; ++n) {
        double w = ivar[n];
        if (w <= 0.0) continue;
        double m = (double)model[template_index(g, j, phase, n - n_lo)];
        double r = dep * m - flux[n];
        l += -0.5 * w * r * r - (-0.5 * w * flux[n] * flux[n]);
    }
    *depth = dep;
    *var = 1.0 / sum_u;
    *lr = l;
    *aabs = sum_abs;
}

void ora_linear(const ora_grid *g, const double *flux, const double *ivar, const float *model,
                double *depth, double *var, double *lr, double *aabs) {
    int64_t I = g->n_t0;
    int J = g->n_dur;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t e = 0; e < (int64_t)J * I; ++e) {
        int j = (int)(e / I);
        int64_t i = e % I;
        linear_one(g, flux, ivar, model, i, j, depth + e, var + e, lr + e, aabs + e);
    }
}

/* Linear search at selected (j, i) elements only (idx = j*I + i). */
void ora_linear_at(const ora_grid *g, const double *flux, const double *ivar, const float *model,
                   const int64_t *idx, int64_t n_idx, double *depth, double *var, double *lr, double *aabs) {
    int64_t I = g->n_t0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < n_idx; ++s) {
        int j = (int)(idx[s] / I);
        int64_t i = idx[s] % I;
        linear_one(g, flux, ivar, model, i, j, depth + s, var + s, lr + s, aabs + s);
    }
}

/* Log-likelihood of the constant (zero-offset) model (Eq. 1 at depth 0), over
 * the non-null resampled points; adding it to a likelihood ratio gives the
 * full log-likelihood (Sec. 2.2, Sec. 2.3). */
double ora_loglike0(const ora_grid *g, const double *flux, const double *ivar) {
    double s = 0.0;
    for (int64_t q = 0; q < g->n; ++q) {
        double w = ivar[q];
        if (w <= 0.0) continue;
        s += -0.5 * w * flux[q] * flux[q] - 0.5 * log(2.0 * M_PI / w);
    }
    return s;
}

/* Period fixed-point step R = llround(2^32 * P/dt) and epoch count
 * I_P = min(I, ceil(R / 2^32)) (reference times beyond one period duplicate
 * earlier ones, Sec. 2.3).  Transit m of epoch i maps to the nearest grid
 * reference time i + o_m, o_m = (m R + 2^31) >> 32 (nearest-neighbour mapping,
 * Sec. 2.3).
 * Reading for the edges of the period range: a period shorter than the
 * reference-time step, or not finite, is not evaluated (its transits would
 * land on the same grid epoch more than once) and gets the null record; a
 * period of at least I steps has exactly one transit per epoch inside the
 * grid (transit 1 would fall at or beyond reference time I), so its step is
 * taken as I * 2^32, which keeps R inside 64 bits for any such period.
 * Returns 0 if the period is not evaluated, else 1 with *R and *IP set. */
static int period_plan(const ora_grid *g, double period, uint64_t *R, int64_t *IP) {
    if (!isfinite(period) || !(period >= g->t0_step)) return 0;
    double steps = period / g->t0_step;
    if (steps >= (double)g->n_t0)
        *R = (uint64_t)g->n_t0 << 32;
    else
        *R = (uint64_t)llround(TWO32 * steps);
    int64_t ip = (int64_t)((*R + 4294967295ULL) >> 32);
    *IP = ip > g->n_t0 ? g->n_t0 : ip;
    return 1;
}

static int64_t transit_offset(uint64_t R, int64_t m) {
    return (int64_t)(((uint64_t)m * R + 2147483648ULL) >> 32);
}

/* One candidate (i, j, k) of the periodic search (Sec. 2.3): the common depth
 * Z is the inverse-variance weighted mean of the transits' depths and its
 * variance is the reciprocal of the sum of weights; the periodic likelihood
 * ratio is the sum over transits of Eq. 4 at that common depth.  Null
 * single-transit elements are skipped.  Returns 0 if every transit is null. */
static int fold_one(const ora_grid *g, const double *depth, const double *var, const double *lr,
                    const double *aabs, uint64_t R, int64_t i, int j,
                    double *lr_out, double *z_out, double *zvar_out, double *aabs_out) {
    int64_t I = g->n_t0;
    const double *dep = depth + (int64_t)j * I;
    const double *va = var + (int64_t)j * I;
    const double *l = lr + (int64_t)j * I;
    const double *ab = aabs + (int64_t)j * I;
    double sw = 0.0, swd = 0.0, sab = 0.0;
    if (R < 4294967296ULL) return 0; /* transits would not advance: not a period */
    for (int64_t m = 0;; ++m) {
        int64_t x = i + transit_offset(R, m);
        if (x >= I) break;
        if (!isfinite(va[x])) continue;
        sw += 1.0 / va[x];
        swd += dep[x] / va[x];
        sab += ab[x];
    }
    if (!(sw > 0.0)) return 0;
    double z = swd / sw;
    double s = 0.0;
    for (int64_t m = 0;; ++m) {
        int64_t x = i + transit_offset(R, m);
        if (x >= I) break;
        if (!isfinite(va[x])) continue;
        double dz = dep[x] - z;
        s += l[x] - 0.5 * dz * dz / va[x];
    }
    *lr_out = s;
    *z_out = z;
    *zvar_out = 1.0 / sw;
    *aabs_out = sab;
    return 1;
}

/* Allowed durations for period k: D_j < P_k (windows must not overlap,
 * Sec. 2.3), intersected with an optional caller range [jr[2k], jr[2k+1]]. */
static void allowed_range(const ora_grid *g, double period, const int32_t *jrange, int64_t k,
                          int *jlo, int *jhi) {
    int lo = 0, hi = g->n_dur - 1;
    if (jrange) {
        if (jrange[2 * k] > lo) lo = jrange[2 * k];
        if (jrange[2 * k + 1] < hi) hi = jrange[2 * k + 1];
    }
    while (hi >= lo && !(g->durations[hi] < period)) --hi;
    *jlo = lo;
    *jhi = hi;
}

/* Periodic search for the periods listed in sel[0..n_sel) (indices into
 * periods[]); results are written at position s of the output arrays.
 * Per period the maximum likelihood-ratio candidate is kept, ties going to
 * the smallest duration index, then the smallest epoch. */
void ora_periodic(const ora_grid *g, const double *depth, const double *var, const double *lr,
                  const double *aabs, const double *periods, const int32_t *jrange,
                  const int64_t *sel, int64_t n_sel, const int32_t *stride, double *lr_out, int32_t *i_out,
                  int32_t *j_out, double *z_out, double *zvar_out, double *aabs_out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t k = sel[s];
        double P = periods[k];
        uint64_t R = 0;
        int64_t IP = 0;
        int jlo = 0, jhi = -1;
        if (period_plan(g, P, &R, &IP)) allowed_range(g, P, jrange, k, &jlo, &jhi);
        double best = -1.0, bz = NAN, bzv = INFINITY, bab = 0.0;
        int32_t bi = -1, bj = -1;
        for (int j = jlo; j <= jhi; ++j) {
            /* optional coarser epoch grid for duration j: only the epochs that
               are multiples of stride[j] (a TLS-style reference-time step
               that grows with the duration, Sec. 2.1.3) */
            int64_t di = stride ? stride[j] : 1;
            for (int64_t i = 0; i < IP; i += di) {
                double l, z, zv, ab;
                if (!fold_one(g, depth, var, lr, aabs, R, i, j, &l, &z, &zv, &ab)) continue;
                if (l > best) {
                    best = l; bz = z; bzv = zv; bab = ab; bi = (int32_t)i; bj = j;
                }
            }
        }
        lr_out[s] = bi >= 0 ? best : 0.0;
        i_out[s] = bi;
        j_out[s] = bj;
        z_out[s] = bz;
        zvar_out[s] = bzv;
        aabs_out[s] = bab;
    }
}

/* A single periodic candidate, for checking another implementation's choice. */
int ora_fold_at(const ora_grid *g, const double *depth, const double *var, const double *lr,
                const double *aabs, double period, int64_t i, int32_t j,
                double *lr_out, double *z_out, double *zvar_out, double *aabs_out) {
    uint64_t R = 0;
    int64_t IP = 0;
    if (!period_plan(g, period, &R, &IP)) return 0;
    return fold_one(g, depth, var, lr, aabs, R, i, j, lr_out, z_out, zvar_out, aabs_out);
}

/* Best period over the periodogram (Sec. 2.3 outputs): maximum likelihood
 * ratio, ties to the smallest period index; -1 if every period is null. */
int64_t ora_best(const double *lr_k, const int32_t *i_k, int64_t n) {
    int64_t kb = -1;
    double best = -1.0;
    for (int64_t k = 0; k < n; ++k) {
        if (i_k[k] < 0) continue;
        if (lr_k[k] > best) {
            best = lr_k[k];
            kb = k;
        }
    }
    return kb;
}
