// Setup stages on the device: template resampling (Sec. 2.1.2), light-curve
// resampling onto the regular grid (Sec. 2.1.1) and the constant-model
// log-likelihood (Eq. 1 at zero depth).
#include <cmath>

#include "common.h"
#include "stages.h"

namespace {

// --- template: linear interpolation of the dense template at cell centres.
__global__ void template_kernel(const double *__restrict__ dense, int64_t n_dense, int32_t n_model,
                                float *__restrict__ model) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_model) return;
    const double tau = ((double)k + 0.5) / (double)n_model;
    const double x = tau * (double)(n_dense - 1);
    int64_t a = (int64_t)floor(x);
    if (a >= n_dense - 1) a = n_dense - 2;
    if (a < 0) a = 0;
    const double fr = x - (double)a;
    model[k] = (float)(dense[a] + fr * (dense[a + 1] - dense[a]));
}

// --- input check: times finite and non-decreasing.  One workgroup, so the
// flag is reduced in-kernel and written once (no pre-clearing needed).
__global__ void __launch_bounds__(1024) check_sorted_kernel(const double *__restrict__ t, int64_t n_obs,
                                                            int32_t *__restrict__ status) {
    __shared__ int bad_any;
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t n = threadIdx.x; n < n_obs; n += blockDim.x) {
        const double tn = t[n];
        if (!isfinite(tn)) bad = 1;
        if (n > 0 && !(tn >= t[n - 1])) bad = 1;
    }
    if (bad) atomicOr(&bad_any, 1);
    __syncthreads();
    if (threadIdx.x == 0) status[0] = bad_any;
}

// --- resampling: one thread per grid point gathers the (sorted) observations
// whose nearest grid point it is (dev::resample_point).
__global__ void resample_kernel(const double *__restrict__ t, const float *__restrict__ f,
                                const float *__restrict__ sigma, int64_t n_obs, double t_first, double c,
                                int64_t n_pad, int64_t n_grid, float *__restrict__ flux,
                                float *__restrict__ ivar) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_grid) return;
    cetra::dev::resample_point(t, f, sigma, n_obs, t_first, c, n_pad, q, flux, ivar);
}

// --- constant-model log-likelihood: one workgroup, fixed reduction order.
__global__ void __launch_bounds__(1024) loglike0_kernel(const float *__restrict__ flux,
                                                        const float *__restrict__ ivar, int64_t n,
                                                        double *__restrict__ out) {
    __shared__ double part[1024];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += blockDim.x) {
        const double w = (double)ivar[q];
        if (!(w > 0.0)) continue;
        const double fq = (double)flux[q];
        s += -0.5 * w * fq * fq - 0.5 * log(2.0 * M_PI / w);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

}  // namespace

using namespace cetra;

extern "C" int cetra_template_resample(void *stream, const double *dense, int64_t n_dense, int32_t n_model,
                                       float *model) {
    clear_error();
    CETRA_REQUIRE(dense && model, "template_resample: NULL pointer");
    CETRA_REQUIRE(n_dense >= 2, "template_resample: need at least 2 dense samples");
    CETRA_REQUIRE(n_model >= 1 && n_model <= CETRA_MAX_MODEL, "template_resample: bad n_model");
    const int threads = 256;
    hipLaunchKernelGGL(template_kernel, dim3((unsigned)ceil_div(n_model, threads)), dim3(threads), 0,
                       as_stream(stream), dense, n_dense, n_model, model);
    return check_launch("template_resample");
}

extern "C" int cetra_resample(void *stream, const cetra_grid *grid, const double *t, const float *f,
                              const float *sigma, int64_t n_obs, float *flux, float *ivar, int32_t *status) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(flux && ivar, "resample: NULL output");
    CETRA_REQUIRE(n_obs >= 0, "resample: n_obs < 0");
    CETRA_REQUIRE(n_obs == 0 || (t && f && sigma), "resample: NULL input");
    hipStream_t s = as_stream(stream);
    if (status) {
        hipLaunchKernelGGL(check_sorted_kernel, dim3(1), dim3(1024), 0, s, t, n_obs, status);
        if ((rc = check_launch("resample/check"))) return rc;
    }
    const int threads = 256;
    hipLaunchKernelGGL(resample_kernel, dim3((unsigned)ceil_div(grid->n, threads)), dim3(threads), 0, s, t, f,
                       sigma, n_obs, grid->t_first, grid->cadence, grid->n_pad, grid->n, flux, ivar);
    return check_launch("resample");
}

extern "C" int cetra_loglike0(void *stream, const cetra_grid *grid, const float *flux, const float *ivar,
                              double *out) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(flux && ivar && out, "loglike0: NULL pointer");
    hipLaunchKernelGGL(loglike0_kernel, dim3(1), dim3(1024), 0, as_stream(stream), flux, ivar, grid->n, out);
    return check_launch("loglike0");
}
