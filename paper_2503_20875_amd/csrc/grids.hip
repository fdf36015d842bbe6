// Host-side period and duration grids (Sec. 2.1.3): the optimally sampled
// period grid and the Keplerian duration range per period that the paper
// takes over as its defaults.  Pure FP64 host code; nothing here touches the
// device.
#include <cmath>

#include "common.h"

namespace cetra {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kGravity = 6.67430e-8;  // cm^3 g^-1 s^-2
constexpr double kDay = 86400.0;         // s

// Semi-major axis in stellar radii of a circular orbit of period P (days)
// around a star of mean density rho (g cm^-3): Kepler's third law with
// M = 4/3 pi R^3 rho gives (a/R)^3 = G rho P^2 / (3 pi).
double a_over_r(double period, double rho) {
    const double p = period * kDay;
    return std::cbrt(kGravity * rho * p * p / (3.0 * kPi));
}

// First-to-last-contact duration (days) of a circular orbit with radius
// ratio k and impact parameter b: T = (P/pi) asin(sqrt((1+k)^2 - b^2) /
// (a/R sin i)), cos i = b / (a/R).  A chord that does not fit (the orbit
// inside the star) gives half the period.
double t14(double period, double rho, double k, double b) {
    const double ar = a_over_r(period, rho);
    const double chord2 = (1.0 + k) * (1.0 + k) - b * b;
    if (chord2 <= 0.0) return 0.0;
    const double cos_i = b / ar;
    if (cos_i >= 1.0) return 0.0;
    const double x = std::sqrt(chord2) / (ar * std::sqrt(1.0 - cos_i * cos_i));
    if (x >= 1.0) return 0.5 * period;
    return period / kPi * std::asin(x);
}

int check_star(double rho_min, double rho_max, double k_max, double b_max) {
    CETRA_REQUIRE(std::isfinite(rho_min) && rho_min > 0.0 && std::isfinite(rho_max) && rho_max >= rho_min,
                  "stellar density range [%g, %g] g/cm^3 is not valid", rho_min, rho_max);
    CETRA_REQUIRE(std::isfinite(k_max) && k_max >= 0.0 && k_max < 1.0, "k_max = %g must lie in [0, 1)", k_max);
    CETRA_REQUIRE(std::isfinite(b_max) && b_max >= 0.0 && b_max < 1.0, "b_max = %g must lie in [0, 1)", b_max);
    return CETRA_OK;
}

}  // namespace
}  // namespace cetra

using namespace cetra;

extern "C" int cetra_period_grid(double span, double p_min, double p_max, double rho, double oversample,
                                 double *periods, int64_t cap, int64_t *n_out) {
    clear_error();
    CETRA_REQUIRE(n_out != nullptr, "period_grid: n_out is NULL");
    CETRA_REQUIRE(std::isfinite(span) && span > 0.0, "period_grid: span %g must be positive", span);
    CETRA_REQUIRE(std::isfinite(p_min) && std::isfinite(p_max) && p_min > 0.0 && p_max > p_min,
                  "period_grid: need 0 < p_min < p_max (got %g, %g)", p_min, p_max);
    CETRA_REQUIRE(std::isfinite(rho) && rho > 0.0, "period_grid: stellar density %g must be positive", rho);
    CETRA_REQUIRE(std::isfinite(oversample) && oversample > 0.0, "period_grid: oversampling %g must be positive",
                  oversample);
    // Frequencies in s^-1.  The duty cycle of a central transit is
    // q(f) = (3 pi / (G rho))^(1/3) f^(2/3) / pi; a step that moves the last
    // transit of the span by q / oversample of a phase, df = q / (S os),
    // is a constant step in f^(1/3) of (3 pi / (G rho))^(1/3) / (3 pi S os).
    const double S = span * kDay;
    const double step = std::cbrt(3.0 * kPi / (kGravity * rho)) / (3.0 * kPi * S * oversample);
    const double x_lo = std::cbrt(1.0 / (p_max * kDay));
    const double x_hi = std::cbrt(1.0 / (p_min * kDay));
    const double n_real = std::floor((x_hi - x_lo) / step) + 1.0;
    CETRA_REQUIRE(n_real <= 1.0e9, "period_grid: %g periods is too many", n_real);
    const int64_t n = (int64_t)n_real;
    *n_out = n;
    if (!periods) return CETRA_OK;
    CETRA_REQUIRE(cap >= n, "period_grid: the output holds %lld periods, %lld are needed", (long long)cap,
                  (long long)n);
    // ascending periods: the lowest frequency last
    for (int64_t m = 0; m < n; ++m) {
        const double x = x_lo + (double)(n - 1 - m) * step;
        periods[m] = 1.0 / (x * x * x) / kDay;
    }
    return CETRA_OK;
}

extern "C" int cetra_duration_limits(double period, double rho_min, double rho_max, double k_max, double b_max,
                                     double *d_min, double *d_max) {
    clear_error();
    CETRA_REQUIRE(d_min != nullptr && d_max != nullptr, "duration_limits: output is NULL");
    CETRA_REQUIRE(std::isfinite(period) && period > 0.0, "duration_limits: period %g must be positive", period);
    int rc = check_star(rho_min, rho_max, k_max, b_max);
    if (rc) return rc;
    *d_max = t14(period, rho_min, k_max, 0.0);
    *d_min = t14(period, rho_max, 0.0, b_max);
    return CETRA_OK;
}

extern "C" int cetra_keplerian_jrange(const double *periods, int64_t n_periods, const double *durations,
                                      int32_t n_dur, double rho_min, double rho_max, double k_max, double b_max,
                                      int32_t *jrange) {
    clear_error();
    CETRA_REQUIRE(n_periods >= 0 && (n_periods == 0 || (periods && jrange)), "keplerian_jrange: NULL array");
    CETRA_REQUIRE(n_dur >= 1 && n_dur <= CETRA_MAX_DURATIONS && durations, "keplerian_jrange: bad durations");
    for (int32_t j = 1; j < n_dur; ++j)
        CETRA_REQUIRE(durations[j] > durations[j - 1], "keplerian_jrange: durations must be ascending");
    int rc = check_star(rho_min, rho_max, k_max, b_max);
    if (rc) return rc;
    for (int64_t k = 0; k < n_periods; ++k) {
        const double P = periods[k];
        int32_t lo = 0, hi = -1;
        if (std::isfinite(P) && P > 0.0) {
            const double d_hi = t14(P, rho_min, k_max, 0.0);
            const double d_lo = t14(P, rho_max, 0.0, b_max);
            lo = n_dur;
            for (int32_t j = 0; j < n_dur; ++j)
                if (durations[j] >= d_lo) {
                    lo = j;
                    break;
                }
            for (int32_t j = n_dur - 1; j >= 0; --j)
                if (durations[j] <= d_hi) {
                    hi = j;
                    break;
                }
        }
        jrange[2 * k] = lo;
        jrange[2 * k + 1] = hi;
    }
    return CETRA_OK;
}

// Epoch strides of a reference-time step that grows with the duration (the
// TLS-style grid Sec. 2.1.3 mentions adopting), on the fixed grid of step dt:
// the largest whole number of steps not above `fraction` of each duration.
extern "C" int cetra_epoch_strides(const cetra_grid *grid, double fraction, int32_t *stride) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(stride != nullptr, "epoch_strides: NULL output");
    CETRA_REQUIRE(std::isfinite(fraction) && fraction > 0.0, "epoch_strides: fraction must be finite and > 0");
    for (int32_t j = 0; j < grid->n_dur; ++j) {
        const double q = fraction * grid->durations[j] / grid->t0_step;
        const double f = std::floor(q + 1e-9);
        stride[j] = f < 1.0 ? 1 : f > (double)INT32_MAX ? INT32_MAX : (int32_t)f;
    }
    return CETRA_OK;
}
