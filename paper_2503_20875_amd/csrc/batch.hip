// Batched search: many light curves of uneven length searched with one call
// (the per-curve method is unchanged: Sec. 2.1 setup, Sec. 2.2 linear search,
// Sec. 2.3 periodic search and best period).
//
// The plan (host only) orders the curves by descending fold cost -- the sum
// over periods of allowed durations times reference times -- and sizes one
// device slot for the largest curve: resampled flux and inverse variance, the
// fold-ready array and the fold workspace.  The search enqueues, curve after
// curve on the caller's stream, the single-curve kernels with outputs written
// at the curve's CSR offsets; stream order makes reusing the slot safe.
// Nothing is allocated and nothing synchronises, so the whole batch can be
// captured in one HIP graph and replayed.  Results are bit-identical to
// separate single-curve calls because they are the same kernels on the same
// inputs.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "common.h"

namespace {

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__global__ void batch_status_kernel(int32_t *status) {
    if (threadIdx.x == 0) status[0] = 0;
}

}  // namespace

struct cetra_batch_plan {
    std::vector<cetra_grid> grids;
    std::vector<int64_t> obs_off, per_off;
    std::vector<int32_t> order;
    size_t off_ivar, off_fold, off_fold_work, fold_work_bytes, workspace_bytes;
    int64_t launches;
};

using namespace cetra;

extern "C" int cetra_batch_plan_create(const cetra_batch_desc *d, cetra_batch_plan **out) {
    clear_error();
    CETRA_REQUIRE(d && out && d->grids && d->obs_offsets && d->period_offsets, "batch_plan: NULL pointer");
    CETRA_REQUIRE(d->n_curves >= 1, "batch_plan: n_curves must be >= 1");
    CETRA_REQUIRE(d->reserved0 == 0 && d->reserved1 == 0, "batch_plan: reserved fields must be 0");
    const int n = d->n_curves;
    const cetra_grid &g0 = d->grids[0];
    int rc;
    size_t max_n = 0, max_fold = 0, max_work = 0;
    std::vector<double> cost(n);
    for (int c = 0; c < n; ++c) {
        if ((rc = check_grid(&d->grids[c]))) return rc;
        const cetra_grid &g = d->grids[c];
        CETRA_REQUIRE(g.n_dur == g0.n_dur && g.n_model == g0.n_model, "batch_plan: curves must share J and M");
        for (int j = 0; j < g.n_dur; ++j)
            CETRA_REQUIRE(g.durations[j] == g0.durations[j], "batch_plan: curves must share the durations");
        CETRA_REQUIRE(d->obs_offsets[c] >= 0 && d->obs_offsets[c + 1] >= d->obs_offsets[c],
                      "batch_plan: obs_offsets not ascending");
        CETRA_REQUIRE(d->period_offsets[c] >= 0 && d->period_offsets[c + 1] >= d->period_offsets[c],
                      "batch_plan: period_offsets not ascending");
        if (g.n_t0 >= ((int64_t)1 << 28))
            return set_error(CETRA_ERR_RANGE, "batch_plan: curve %d: I must be < 2^28", c);
        const int64_t K = d->period_offsets[c + 1] - d->period_offsets[c];
        size_t wb = 0;
        if ((rc = cetra_periodic_workspace(&g, K, &wb))) return rc;
        max_n = std::max(max_n, (size_t)g.n);
        max_fold = std::max(max_fold, (size_t)8 * (size_t)g.n_dur * (size_t)g.n_t0);
        max_work = std::max(max_work, wb);
        cost[c] = (double)K * g.n_dur * (double)g.n_t0;
    }
    auto *plan = new (std::nothrow) cetra_batch_plan;
    if (!plan) return set_error(CETRA_ERR_INVALID, "batch_plan: out of host memory");
    plan->grids.assign(d->grids, d->grids + n);
    plan->obs_off.assign(d->obs_offsets, d->obs_offsets + n + 1);
    plan->per_off.assign(d->period_offsets, d->period_offsets + n + 1);
    plan->order.resize(n);
    std::iota(plan->order.begin(), plan->order.end(), 0);
    std::stable_sort(plan->order.begin(), plan->order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    // slot layout: flux [N] | ivar [N] | fold [J][I][2] | fold workspace
    plan->off_ivar = align256(4 * max_n);
    plan->off_fold = plan->off_ivar + align256(4 * max_n);
    plan->off_fold_work = plan->off_fold + align256(max_fold);
    plan->fold_work_bytes = max_work;
    plan->workspace_bytes = plan->off_fold_work + align256(std::max<size_t>(max_work, 1));
    int64_t launches = 1;  // status kernel
    for (int c = 0; c < n; ++c) {
        const int64_t K = plan->per_off[c + 1] - plan->per_off[c];
        launches += 1 + plan->grids[c].n_dur + (K > 0 ? 3 : 0) + 1;  // resample, linear per duration, fold, best
    }
    plan->launches = launches;
    *out = plan;
    return CETRA_OK;
}

extern "C" int cetra_batch_plan_destroy(cetra_batch_plan *plan) {
    clear_error();
    delete plan;
    return CETRA_OK;
}

extern "C" int cetra_batch_plan_info(const cetra_batch_plan *plan, cetra_batch_info *info) {
    clear_error();
    CETRA_REQUIRE(plan && info, "batch_plan_info: NULL pointer");
    std::memset(info, 0, sizeof *info);
    info->workspace_bytes = plan->workspace_bytes;
    info->n_curves = (int64_t)plan->grids.size();
    info->total_periods = plan->per_off.back() - plan->per_off.front();
    info->n_launches = plan->launches;
    return CETRA_OK;
}

extern "C" int cetra_batch_plan_order(const cetra_batch_plan *plan, int32_t *order, int32_t n) {
    clear_error();
    CETRA_REQUIRE(plan && order, "batch_plan_order: NULL pointer");
    CETRA_REQUIRE(n == (int32_t)plan->order.size(), "batch_plan_order: n must equal the number of curves");
    std::copy(plan->order.begin(), plan->order.end(), order);
    return CETRA_OK;
}

extern "C" int cetra_batch_search(const cetra_batch_plan *plan, void *stream, const double *t, const float *f,
                                  const float *sigma, const float *model, const double *periods, void *work,
                                  size_t work_bytes, float *lr, int32_t *epoch, int32_t *dur, float *depth,
                                  float *depth_var, cetra_best_record *best, int32_t *status) {
    clear_error();
    CETRA_REQUIRE(plan, "batch_search: NULL plan");
    CETRA_REQUIRE(model && work && best && status && t && f && sigma, "batch_search: NULL pointer");
    const bool any_periods = plan->per_off.back() > plan->per_off.front();
    CETRA_REQUIRE(!any_periods || (periods && lr && epoch && dur && depth && depth_var),
                  "batch_search: NULL period pointer");
    if (work_bytes < plan->workspace_bytes)
        return set_error(CETRA_ERR_WORKSPACE, "batch_search: workspace needs %zu bytes", plan->workspace_bytes);
    char *w = static_cast<char *>(work);
    float *flux = reinterpret_cast<float *>(w);
    float *ivar = reinterpret_cast<float *>(w + plan->off_ivar);
    float *fold = reinterpret_cast<float *>(w + plan->off_fold);
    void *fwork = w + plan->off_fold_work;
    int rc;
    for (const int32_t c : plan->order) {
        const cetra_grid *g = &plan->grids[c];
        const int64_t o0 = plan->obs_off[c], n_obs = plan->obs_off[c + 1] - o0;
        const int64_t p0 = plan->per_off[c], K = plan->per_off[c + 1] - p0;
        if ((rc = cetra_resample(stream, g, t + o0, f + o0, sigma + o0, n_obs, flux, ivar, nullptr))) return rc;
        if ((rc = cetra_linear_search(stream, g, flux, ivar, model, fold, nullptr, nullptr, nullptr))) return rc;
        if (K > 0 &&
            (rc = cetra_periodic_search(stream, g, fold, periods + p0, K, nullptr, nullptr, 0, fwork,
                                        plan->fold_work_bytes, lr + p0, epoch + p0, dur + p0, depth + p0,
                                        depth_var + p0)))
            return rc;
        if (K > 0)
            rc = cetra_best(stream, g, periods + p0, K, lr + p0, epoch + p0, dur + p0, depth + p0, depth_var + p0,
                            best + c);
        else
            rc = cetra_best(stream, g, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, best + c);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(batch_status_kernel, dim3(1), dim3(64), 0, as_stream(stream), status);
    return check_launch("batch_search/status");
}
