// Linear search (Sec. 2.2): for every (reference time i, duration j) window,
// the inverse-variance weighted template fit S_fm = sum w f m,
// S_mm = sum w m^2, from which depth = S_fm/S_mm, var = 1/S_mm and the
// likelihood ratio of Eq. 2, S_fm^2 / (2 S_mm), follow in closed form.
//
// Work mapping (gfx950, wave64): one workgroup of 256 lanes takes 256
// consecutive reference times of one duration.  Their windows overlap almost
// entirely, so the workgroup stages the light-curve span they cover, as
// (w f, w) pairs, plus the template in LDS, and every lane then walks its own
// window out of LDS (dev::linear_tile).
#include <cmath>

#include "common.h"
#include "stages.h"

namespace {

using cetra::dev::kThreads;

__global__ void __launch_bounds__(kThreads) linear_kernel(cetra::dev::LinearParams p, const float *__restrict__ flux,
                                                          const float *__restrict__ ivar,
                                                          const float *__restrict__ model, float2 *__restrict__ fold,
                                                          float *__restrict__ depth, float *__restrict__ var,
                                                          float *__restrict__ lr, int64_t row_offset) {
    extern __shared__ float lds[];
    __shared__ int s_bounds[2];
    cetra::dev::linear_tile(p, (int64_t)blockIdx.x * kThreads, flux, ivar, model, fold + row_offset,
                            depth ? depth + row_offset : nullptr, var ? var + row_offset : nullptr,
                            lr ? lr + row_offset : nullptr, lds, s_bounds);
}

}  // namespace

namespace cetra {

// LDS bytes of the linear tile for duration j, and its staged span
// (0 = the span does not fit and the tile reads the light curve directly).
size_t linear_lds_bytes(const cetra_grid *g, int j, int32_t *span_cap) {
    const size_t model_bytes = (size_t)((g->n_model + 1) & ~1) * sizeof(float);
    const double span = dev::linear_span(g->t0_step, g->durations[j], g->cadence);
    const size_t staged_bytes = model_bytes + (size_t)std::ceil(span) * sizeof(float2);
    if (staged_bytes <= (size_t)kMaxLinearLdsBytes) {
        *span_cap = (int32_t)std::ceil(span);
        return staged_bytes;
    }
    *span_cap = 0;
    return model_bytes;
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
    const int64_t blocks = ceil_div(grid->n_t0, kThreads);
    if (blocks > INT32_MAX) return set_error(CETRA_ERR_RANGE, "linear_search: too many reference times");
    for (int j = 0; j < grid->n_dur; ++j) {
        dev::LinearParams p = dev::linear_params(*grid, j);
        const size_t lds = linear_lds_bytes(grid, j, &p.span_cap);
        hipLaunchKernelGGL(linear_kernel, dim3((unsigned)blocks), dim3(kThreads), lds, s, p, flux, ivar, model,
                           reinterpret_cast<float2 *>(fold), depth, var, lr, (int64_t)j * grid->n_t0);
        if ((rc = check_launch("linear_search"))) return rc;
    }
    return CETRA_OK;
}
