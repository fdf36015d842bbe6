// Single-event (monotransit) search over the linear search's results, the
// nulling of a found signal's transits for the next search (Sec. 1 and
// Sec. 5: single transits are searched for in the linear-search output; a
// multi-planet search re-runs after nulling the flux in and around the
// strongest signal), and the per-period merge of searches run with several
// templates (Sec. 2.1.2 suggests searching across a sequence of impact
// parameters).
#include <cmath>

#include "common.h"
#include "stages.h"

namespace {

using namespace cetra;

struct EventDurations {
    double d[CETRA_MAX_DURATIONS];
};

constexpr int kEventThreads = 256;

// Ranking key of candidate (j, i): FP32 LR bits (LR >= 0, so the bits are
// monotone) above the complement of the flat index j I + i, so that a 64-bit
// maximum prefers the larger LR and, on ties, the smaller index.
__device__ __forceinline__ uint64_t event_key(float lr, uint32_t flat) {
    return ((uint64_t)__float_as_uint(lr) << 32) | (uint64_t)(0xFFFFFFFFu - flat);
}

__global__ void events_clear_kernel(uint64_t *keys, int32_t n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) keys[t] = 0;
}

// Strongest candidate whose window overlaps none of the events already
// found: |t_i - t_e| < (D_j + D_e) / 2 with t = i dt excludes (j, i).
__global__ void __launch_bounds__(kEventThreads) events_reduce_kernel(const float2 *__restrict__ fold, int64_t I,
                                                                      int32_t J, double dt, EventDurations dur,
                                                                      const cetra_event *__restrict__ found,
                                                                      int32_t n_found, uint64_t *key) {
    __shared__ double s_t[64];
    __shared__ double s_half[64];
    const int n_ex = min(n_found, 64);
    for (int q = threadIdx.x; q < n_ex; q += blockDim.x) {
        const cetra_event ev = found[q];
        s_t[q] = ev.epoch >= 0 ? (double)ev.epoch * dt : __builtin_inf();
        s_half[q] = ev.epoch >= 0 ? 0.5 * ev.duration : 0.0;
    }
    __syncthreads();
    uint64_t best = 0;
    const int64_t total = (int64_t)J * I;
    for (int64_t flat = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; flat < total;
         flat += (int64_t)gridDim.x * blockDim.x) {
        const float2 p = fold[flat];
        if (!(p.y > 0.0f)) continue;
        const int32_t j = (int32_t)(flat / I);
        const int64_t i = flat - (int64_t)j * I;
        const double t = (double)i * dt;
        bool free = true;
        for (int q = 0; q < n_ex; ++q) free &= !(fabs(t - s_t[q]) < s_half[q] + 0.5 * dur.d[j]);
        if (!free) continue;
        const uint64_t k = event_key(0.5f * p.x * (p.x / p.y), (uint32_t)flat);
        best = k > best ? k : best;
    }
    const uint64_t m = cetra::dev::wave_max_u64(best);
    if ((threadIdx.x & 63) == 0 && m != 0) atomicMax((unsigned long long *)key, (unsigned long long)m);
}

// The winner's record from its fold-ready pair, in FP64.
__global__ void events_decode_kernel(const float2 *__restrict__ fold, int64_t I, double dt, double t_origin,
                                     EventDurations dur, const uint64_t *key, cetra_event *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    cetra_event ev;
    const uint64_t k = *key;
    if (k == 0) {
        ev.epoch = -1;
        ev.dur = -1;
        ev.t0 = ev.t0_abs = ev.duration = __builtin_nan("");
        ev.lr = 0.0;
        ev.depth = __builtin_nan("");
        ev.depth_var = __builtin_inf();
        ev.snr = 0.0;
    } else {
        const uint32_t flat = 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull);
        const int32_t j = (int32_t)(flat / (uint64_t)I);
        const int64_t i = (int64_t)flat - (int64_t)j * I;
        const float2 p = fold[flat];
        const double sfm = p.x, smm = p.y;
        ev.epoch = (int32_t)i;
        ev.dur = j;
        ev.t0 = (double)i * dt;
        ev.t0_abs = t_origin + ev.t0;
        ev.duration = dur.d[j];
        ev.depth = sfm / smm;
        ev.depth_var = 1.0 / smm;
        ev.lr = 0.5 * sfm * sfm / smm;
        ev.snr = ev.depth / sqrt(ev.depth_var);
    }
    *out = ev;
}

// Null every resampled point within half_width of a transit mid-time
// t0 + n P (nearest n), or of t0 alone for a single event (P not > 0).
__global__ void mask_kernel(int64_t n, double cadence, double period, double t0, double half_width, float *flux,
                            float *ivar) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double d = (double)q * cadence - t0;
    if (period > 0.0) d -= floor(d / period + 0.5) * period;
    if (fabs(d) <= half_width) {
        flux[q] = 0.0f;
        ivar[q] = 0.0f;
    }
}

// Per period, the record with the largest LR over n_sets stacked period
// searches (ties: the first set); null records never win over a valid one.
__global__ void merge_kernel(int32_t n_sets, int64_t n, const float *__restrict__ lr, const int32_t *__restrict__ ep,
                             const int32_t *__restrict__ du, const float *__restrict__ z,
                             const float *__restrict__ zv, float *__restrict__ o_lr, int32_t *__restrict__ o_ep,
                             int32_t *__restrict__ o_du, float *__restrict__ o_z, float *__restrict__ o_zv,
                             int32_t *__restrict__ o_set) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t best = -1;
    for (int32_t s = 0; s < n_sets; ++s) {
        const int64_t q = (int64_t)s * n + k;
        if (ep[q] < 0) continue;
        if (best < 0 || lr[q] > lr[(int64_t)best * n + k]) best = s;
    }
    if (best < 0) {
        o_lr[k] = 0.0f;
        o_ep[k] = -1;
        o_du[k] = -1;
        o_z[k] = __builtin_nanf("");
        o_zv[k] = __builtin_inff();
        o_set[k] = -1;
        return;
    }
    const int64_t q = (int64_t)best * n + k;
    o_lr[k] = lr[q];
    o_ep[k] = ep[q];
    o_du[k] = du[q];
    o_z[k] = z[q];
    o_zv[k] = zv[q];
    o_set[k] = best;
}

}  // namespace

extern "C" int cetra_periodic_merge(void *stream, int32_t n_sets, int64_t n_periods, const float *lr,
                                    const int32_t *epoch, const int32_t *dur, const float *depth,
                                    const float *depth_var, float *out_lr, int32_t *out_epoch, int32_t *out_dur,
                                    float *out_depth, float *out_depth_var, int32_t *out_set) {
    clear_error();
    CETRA_REQUIRE(n_sets >= 1 && n_periods >= 0, "periodic_merge: bad sizes");
    CETRA_REQUIRE(n_periods == 0 || (lr && epoch && dur && depth && depth_var && out_lr && out_epoch && out_dur &&
                                     out_depth && out_depth_var && out_set),
                  "periodic_merge: NULL pointer");
    if (n_periods == 0) return CETRA_OK;
    hipLaunchKernelGGL(merge_kernel, dim3((unsigned)ceil_div(n_periods, 256)), dim3(256), 0, as_stream(stream),
                       n_sets, n_periods, lr, epoch, dur, depth, depth_var, out_lr, out_epoch, out_dur, out_depth,
                       out_depth_var, out_set);
    return check_launch("periodic_merge");
}

extern "C" int cetra_single_events_workspace(int32_t n_events, size_t *bytes) {
    clear_error();
    CETRA_REQUIRE(bytes != nullptr, "single_events_workspace: bytes is NULL");
    CETRA_REQUIRE(n_events >= 1 && n_events <= CETRA_MAX_EVENTS, "single_events: n_events %d not in [1, %d]",
                  n_events, CETRA_MAX_EVENTS);
    *bytes = sizeof(uint64_t) * (size_t)n_events;
    return CETRA_OK;
}

extern "C" int cetra_single_events(void *stream, const cetra_grid *grid, const float *fold, int32_t n_events,
                                   void *work, size_t work_bytes, cetra_event *out) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(fold && out, "single_events: NULL pointer");
    CETRA_REQUIRE(n_events >= 1 && n_events <= CETRA_MAX_EVENTS, "single_events: n_events %d not in [1, %d]",
                  n_events, CETRA_MAX_EVENTS);
    CETRA_REQUIRE(work && work_bytes >= sizeof(uint64_t) * (size_t)n_events,
                  "single_events: workspace needs %zu bytes", sizeof(uint64_t) * (size_t)n_events);
    hipStream_t s = as_stream(stream);
    EventDurations d;
    for (int j = 0; j < CETRA_MAX_DURATIONS; ++j) d.d[j] = j < grid->n_dur ? grid->durations[j] : 0.0;
    auto *keys = static_cast<uint64_t *>(work);
    const auto *f2 = reinterpret_cast<const float2 *>(fold);
    const int64_t I = grid->n_t0;
    const int64_t total = (int64_t)grid->n_dur * I;
    const int64_t wgs = std::min<int64_t>(ceil_div(total, kEventThreads), (int64_t)device_cu_count() * 8);
    hipLaunchKernelGGL(events_clear_kernel, dim3(1), dim3(CETRA_MAX_EVENTS), 0, s, keys, n_events);
    if ((rc = check_launch("single_events/clear"))) return rc;
    for (int32_t e = 0; e < n_events; ++e) {
        hipLaunchKernelGGL(events_reduce_kernel, dim3((unsigned)wgs), dim3(kEventThreads), 0, s, f2, I,
                           grid->n_dur, grid->t0_step, d, out, e, keys + e);
        if ((rc = check_launch("single_events/reduce"))) return rc;
        hipLaunchKernelGGL(events_decode_kernel, dim3(1), dim3(64), 0, s, f2, I, grid->t0_step, grid->t_origin, d,
                           keys + e, out + e);
        if ((rc = check_launch("single_events/decode"))) return rc;
    }
    return CETRA_OK;
}

extern "C" int cetra_mask_transits(void *stream, const cetra_grid *grid, double period, double t0, double duration,
                                   double width, float *flux, float *ivar) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(flux && ivar, "mask_transits: NULL pointer");
    CETRA_REQUIRE(std::isfinite(t0) && std::isfinite(duration) && duration > 0.0 && std::isfinite(width) &&
                      width > 0.0,
                  "mask_transits: t0, duration and width must be finite, duration and width positive");
    const int64_t n = grid->n;
    if (n == 0) return CETRA_OK;
    const double p = (period > 0.0 && std::isfinite(period)) ? period : 0.0;  // else a single event
    hipLaunchKernelGGL(mask_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, as_stream(stream), n,
                       grid->cadence, p, t0, 0.5 * width * duration, flux, ivar);
    return check_launch("mask_transits");
}
