// Linear search (Sec. 2.2): for every (reference time i, duration j) window,
// the inverse-variance weighted template fit S_fm = sum w f m,
// S_mm = sum w m^2, from which depth = S_fm/S_mm, var = 1/S_mm and the
// likelihood ratio of Eq. 2, S_fm^2 / (2 S_mm), follow in closed form.
//
// Work mapping (gfx950, wave64): one workgroup of 256 lanes takes 256 W
// consecutive reference times of one duration, W adjacent ones per lane
// (W = 1, 2 or 4, the launch tuning's linear_windows); one launch covers
// every duration.  Their windows overlap almost entirely, so the workgroup
// stages the light-curve span they cover, as (w f, w) pairs, plus the
// template in LDS; a lane then walks the union of its W windows once,
// reading each point's pair once for all of them (dev::linear_tile).  Per
// window and point: one LDS read of the template, a multiply, two FMAs and
// the 64-bit phase step.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "stages.h"

namespace {

using cetra::dev::kThreads;

// Per-duration parameters of one launch over every duration.
struct LinearLaunch {
    double cadence, t0_step, t_end;
    int64_t n_t0, n_tiles;
    int32_t n_model, n_dur;
    double duration[CETRA_MAX_DURATIONS];
    uint64_t step_fx[CETRA_MAX_DURATIONS];
    int32_t span_cap[CETRA_MAX_DURATIONS];
};

// One launch for every duration: workgroup b takes tile b mod n_tiles of
// duration J - 1 - b / n_tiles (the longest windows first, so the costliest
// workgroups start first).
template <int W>
__global__ void __launch_bounds__(kThreads) linear_kernel(const LinearLaunch L, const float *__restrict__ flux,
                                                          const float *__restrict__ ivar,
                                                          const float *__restrict__ model, float2 *__restrict__ fold,
                                                          float *__restrict__ depth, float *__restrict__ var,
                                                          float *__restrict__ lr) {
    extern __shared__ float lds[];
    __shared__ int s_bounds[2];
    const int32_t j = L.n_dur - 1 - (int32_t)(blockIdx.x / L.n_tiles);
    const int64_t tile = blockIdx.x % L.n_tiles;
    cetra::dev::LinearParams p;
    p.cadence = L.cadence;
    p.t0_step = L.t0_step;
    p.duration = L.duration[j];
    p.t_end = L.t_end;
    p.n_t0 = L.n_t0;
    p.step_fx = L.step_fx[j];
    p.n_model = L.n_model;
    p.span_cap = L.span_cap[j];
    const int64_t row = (int64_t)j * L.n_t0;
    cetra::dev::linear_tile<W>(p, tile * kThreads * W, flux, ivar, model, fold + row, depth ? depth + row : nullptr,
                               var ? var + row : nullptr, lr ? lr + row : nullptr, lds, s_bounds);
}

}  // namespace

namespace cetra {

size_t linear_lds_bytes(const cetra_grid *g, int j, int W, size_t cap, int32_t *span_cap) {
    const size_t tab_bytes = (size_t)dev::template_table_entries(g->n_model) * sizeof(float);
    const double span = dev::linear_span(g->t0_step, g->durations[j], g->cadence, W);
    const size_t staged_bytes = tab_bytes + (size_t)std::ceil(span) * sizeof(float2);
    if (staged_bytes <= cap) {
        *span_cap = (int32_t)std::ceil(span);
        return staged_bytes;
    }
    *span_cap = 0;
    return tab_bytes;
}

}  // namespace cetra

using namespace cetra;

extern "C" int cetra_linear_search(void *stream, const cetra_grid *grid, const float *flux, const float *ivar,
                                   const float *model, float *fold, float *depth, float *var, float *lr) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(flux && ivar && model && fold, "linear_search: NULL pointer");
    if (grid->n >= INT32_MAX) return set_error(CETRA_ERR_RANGE, "linear_search: N must be < 2^31");
    const int W = current_tuning().linear_windows;
    LinearLaunch L;
    std::memset(&L, 0, sizeof L);
    L.cadence = grid->cadence;
    L.t0_step = grid->t0_step;
    L.t_end = (double)(grid->n - 1) * grid->cadence;
    L.n_t0 = grid->n_t0;
    L.n_tiles = ceil_div(grid->n_t0, (int64_t)kThreads * W);
    L.n_model = grid->n_model;
    L.n_dur = grid->n_dur;
    size_t lds = 0;
    for (int j = 0; j < grid->n_dur; ++j) {
        L.duration[j] = grid->durations[j];
        L.step_fx[j] = grid->dur_step_fx[j];
        lds = std::max(lds, linear_lds_bytes(grid, j, W, kMaxLinearLdsBytes, &L.span_cap[j]));
    }
    const int64_t blocks = L.n_tiles * grid->n_dur;
    if (blocks > INT32_MAX) return set_error(CETRA_ERR_RANGE, "linear_search: too many reference times");
    const void *kern = W == 1 ? (const void *)linear_kernel<1>
                     : W == 2 ? (const void *)linear_kernel<2>
                              : (const void *)linear_kernel<4>;
    auto *fold2 = reinterpret_cast<float2 *>(fold);
    void *args[] = {(void *)&L, (void *)&flux, (void *)&ivar, (void *)&model, (void *)&fold2,
                    (void *)&depth, (void *)&var, (void *)&lr};
    const hipError_t le = hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(kThreads), args, lds, as_stream(stream));
    if (le != hipSuccess) return set_error(CETRA_ERR_HIP, "linear_search: %s", hipGetErrorString(le));
    return CETRA_OK;
}
