// Linear search (Sec. 2.2): for every (reference time i, duration j) window,
// the inverse-variance weighted template fit S_fm = sum w f m,
// S_mm = sum w m^2, from which depth = S_fm/S_mm, var = 1/S_mm and the
// likelihood ratio of Eq. 2, S_fm^2 / (2 S_mm), follow in closed form.
//
// Work mapping (gfx950, wave64): one workgroup of 256 lanes takes 256 W
// consecutive reference times of one duration, W adjacent ones per lane
// (W = 1, 2 or 4, the launch tuning's linear_windows).  Their windows overlap
// almost entirely, so the workgroup stages the light-curve span they cover,
// as (w f, w) pairs, plus the template table (m, m^2) in LDS; a lane then
// walks the union of its W windows once, reading each point's pair once for
// all of them (dev::linear_tile).  Per window and point: one LDS read of the
// template pair, two FMAs and the 64-bit phase step.
#include <cmath>

#include "common.h"
#include "stages.h"

namespace {

using cetra::dev::kThreads;

template <int W>
__global__ void __launch_bounds__(kThreads) linear_kernel(cetra::dev::LinearParams p, const float *__restrict__ flux,
                                                          const float *__restrict__ ivar,
                                                          const float *__restrict__ model, float2 *__restrict__ fold,
                                                          float *__restrict__ depth, float *__restrict__ var,
                                                          float *__restrict__ lr, int64_t row_offset) {
    extern __shared__ float lds[];
    __shared__ int s_bounds[2];
    cetra::dev::linear_tile<W>(p, (int64_t)blockIdx.x * kThreads * W, flux, ivar, model, fold + row_offset,
                               depth ? depth + row_offset : nullptr, var ? var + row_offset : nullptr,
                               lr ? lr + row_offset : nullptr, lds, s_bounds);
}

}  // namespace

namespace cetra {

size_t linear_lds_bytes(const cetra_grid *g, int j, int W, size_t cap, int32_t *span_cap) {
    const size_t tab_bytes = (size_t)dev::template_table_entries(g->n_model) * sizeof(float2);
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
    hipStream_t s = as_stream(stream);
    const int W = current_tuning().linear_windows;
    const int64_t blocks = ceil_div(grid->n_t0, (int64_t)kThreads * W);
    if (blocks > INT32_MAX) return set_error(CETRA_ERR_RANGE, "linear_search: too many reference times");
    const void *kern = W == 1 ? (const void *)linear_kernel<1>
                     : W == 2 ? (const void *)linear_kernel<2>
                              : (const void *)linear_kernel<4>;
    for (int j = 0; j < grid->n_dur; ++j) {
        dev::LinearParams p = dev::linear_params(*grid, j);
        size_t lds = linear_lds_bytes(grid, j, W, kMaxLinearLdsBytes, &p.span_cap);
        auto *fold2 = reinterpret_cast<float2 *>(fold);
        int64_t row = (int64_t)j * grid->n_t0;
        void *args[] = {(void *)&p,   (void *)&flux, (void *)&ivar, (void *)&model, (void *)&fold2,
                        (void *)&depth, (void *)&var, (void *)&lr,   (void *)&row};
        const hipError_t le = hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(kThreads), args, lds, s);
        if (le != hipSuccess) return set_error(CETRA_ERR_HIP, "linear_search: %s", hipGetErrorString(le));
    }
    return CETRA_OK;
}
