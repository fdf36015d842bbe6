// Service entry points, error handling and the host-side grid plan.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace cetra {

static thread_local std::string g_last_error;

int set_error(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

void clear_error() { g_last_error.clear(); }

int device_cu_count() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CETRA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return CETRA_OK;
}

static std::mutex g_tuning_mu;
static cetra_tuning g_tuning = {8, 8, 4, 2, 4, {0, 0, 0}};

cetra_tuning current_tuning() {
    std::lock_guard<std::mutex> lock(g_tuning_mu);
    return g_tuning;
}

int check_grid(const cetra_grid *g) {
    CETRA_REQUIRE(g != nullptr, "grid is NULL");
    CETRA_REQUIRE(g->n_dur >= 1 && g->n_dur <= CETRA_MAX_DURATIONS, "grid: bad n_dur %d", g->n_dur);
    CETRA_REQUIRE(g->n_model >= 1 && g->n_model <= CETRA_MAX_MODEL, "grid: bad n_model %d", g->n_model);
    CETRA_REQUIRE(g->n >= 1 && g->n_t0 >= 1 && g->cadence > 0 && g->t0_step > 0, "grid: not planned");
    if ((int64_t)g->n_dur * g->n_t0 > (int64_t)UINT32_MAX)
        return set_error(CETRA_ERR_RANGE, "grid: J*I = %lld exceeds 2^32",
                         (long long)((int64_t)g->n_dur * g->n_t0));
    return CETRA_OK;
}

}  // namespace cetra

using namespace cetra;

extern "C" int cetra_version(void) { return CETRA_VERSION; }

extern "C" const char *cetra_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *cetra_status_string(int status) {
    switch (status) {
        case CETRA_OK: return "ok";
        case CETRA_ERR_INVALID: return "invalid argument";
        case CETRA_ERR_RANGE: return "size out of supported range";
        case CETRA_ERR_WORKSPACE: return "workspace too small";
        case CETRA_ERR_HIP: return "HIP runtime error";
        case CETRA_ERR_DEVICE: return "no usable device";
        default: return "unknown status";
    }
}

extern "C" int cetra_get_tuning(cetra_tuning *out) {
    clear_error();
    CETRA_REQUIRE(out != nullptr, "get_tuning: NULL pointer");
    *out = current_tuning();
    return CETRA_OK;
}

extern "C" int cetra_set_tuning(const cetra_tuning *in) {
    clear_error();
    cetra_tuning t = {8, 8, 4, 2, 4, {0, 0, 0}};
    if (in) {
        CETRA_REQUIRE(in->fold_period_block == 4 || in->fold_period_block == 8 || in->fold_period_block == 16,
                      "set_tuning: fold_period_block must be 4, 8 or 16");
        CETRA_REQUIRE(in->fold_wgs_per_cu >= 1 && in->fold_wgs_per_cu <= 32, "set_tuning: fold_wgs_per_cu in [1, 32]");
        CETRA_REQUIRE(in->fold_units_per_wg >= 1 && in->fold_units_per_wg <= 64,
                      "set_tuning: fold_units_per_wg in [1, 64]");
        CETRA_REQUIRE(in->fold_variant == 0 || in->fold_variant == 2, "set_tuning: fold_variant must be 0 or 2");
        CETRA_REQUIRE(in->linear_windows == 0 || in->linear_windows == 1 || in->linear_windows == 2 ||
                          in->linear_windows == 4,
                      "set_tuning: linear_windows must be 1, 2 or 4 (0: the default)");
        t = *in;
        if (t.linear_windows == 0) t.linear_windows = 4;
    }
    std::lock_guard<std::mutex> lock(g_tuning_mu);
    g_tuning = t;
    return CETRA_OK;
}

// Grid plan: padding of half the longest duration at both ends (Sec. 2.1.1),
// reference-time step of 1% of the shortest duration by default (Sec. 2.1.3),
// template-sample step per grid point in 32.32 fixed point for the
// nearest-sample rule (Sec. 2.1.2).  Plain IEEE FP64, no contraction.
extern "C" int cetra_grid_plan(double t_first, double t_last, double cadence, const double *durations,
                               int32_t n_dur, double t0_step, int32_t n_model, cetra_grid *out) {
    clear_error();
    CETRA_REQUIRE(out != nullptr && durations != nullptr, "grid_plan: NULL pointer");
    CETRA_REQUIRE(std::isfinite(t_first) && std::isfinite(t_last) && t_last >= t_first,
                  "grid_plan: need finite t_last >= t_first");
    CETRA_REQUIRE(std::isfinite(cadence) && cadence > 0, "grid_plan: cadence must be > 0");
    CETRA_REQUIRE(n_dur >= 1 && n_dur <= CETRA_MAX_DURATIONS, "grid_plan: n_dur must be in [1, %d]",
                  CETRA_MAX_DURATIONS);
    CETRA_REQUIRE(n_model >= 1 && n_model <= CETRA_MAX_MODEL, "grid_plan: n_model must be in [1, %d]",
                  CETRA_MAX_MODEL);
    for (int j = 0; j < n_dur; ++j) {
        CETRA_REQUIRE(std::isfinite(durations[j]) && durations[j] > 0, "grid_plan: duration %d not > 0", j);
        CETRA_REQUIRE(j == 0 || durations[j] > durations[j - 1], "grid_plan: durations not ascending");
    }
    cetra_grid g;
    std::memset(&g, 0, sizeof g);
    const double d_max = durations[n_dur - 1];
    const double d_min = durations[0];
    g.t_first = t_first;
    g.cadence = cadence;
    g.n_pad = (int64_t)std::ceil((d_max / 2.0) / cadence);
    g.n_data = (int64_t)std::floor((t_last - t_first) / cadence + 0.5) + 1;
    g.n = g.n_data + 2 * g.n_pad;
    g.t_origin = t_first - (double)g.n_pad * cadence;
    g.t0_step = t0_step > 0 ? t0_step : 0.01 * d_min;
    const double span = (double)(g.n - 1) * cadence / g.t0_step;
    if (!(span < 4.0e9))
        return set_error(CETRA_ERR_RANGE, "grid_plan: too many reference times (%.3g)", span);
    g.n_t0 = (int64_t)std::floor(span) + 1;
    g.n_dur = n_dur;
    g.n_model = n_model;
    for (int j = 0; j < n_dur; ++j) {
        g.durations[j] = durations[j];
        g.dur_step_fx[j] = (uint64_t)std::llround(kTwo32 * (((double)n_model * cadence) / durations[j]));
    }
    int rc = check_grid(&g);
    if (rc != CETRA_OK) return rc;
    *out = g;
    return CETRA_OK;
}
