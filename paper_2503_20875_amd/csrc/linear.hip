// Linear search (Sec. 2.2): for every (reference time i, duration j) window,
// the inverse-variance weighted template fit S_fm = sum w f m,
// S_mm = sum w m^2, from which depth = S_fm/S_mm, var = 1/S_mm and the
// likelihood ratio of Eq. 2, S_fm^2 / (2 S_mm), follow in closed form.
//
// Work mapping (gfx950, wave64): one workgroup of 256 lanes takes 256
// consecutive reference times of one duration.  Their windows overlap almost
// entirely, so the workgroup stages the light-curve span they cover, as
// (w f, w) pairs, plus the template in LDS, and every lane then walks its own
// window out of LDS.  Template indices advance in 32.32 fixed point (two
// integer adds per point).  Partial sums are kept in FP32 registers for 32
// points at a time and folded into FP64, which bounds the rounding of windows
// with thousands of points.
#include <climits>
#include <cmath>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 32;                    // FP32 partial-sum length
constexpr int kMaxLdsBytes = 64 * 1024;       // staging limit per workgroup

struct LinearParams {
    double cadence, t0_step, duration, t_end;  // t_end = (N-1) c
    int64_t n_t0;
    uint64_t step_fx;                           // G_j
    int32_t n_model;
    int32_t span_cap;                           // staged points (0 = not staged)
};

struct Window {
    int64_t lo, hi;
    uint64_t phase;
    bool ok;
};

// Window of reference time i: [t_i - D/2, t_i + D/2], null if it leaves
// [0, (N-1) c]; first/last grid points ceil(t_s/c), floor(t_e/c); template
// phase of the first point in 32.32 fixed point (plain FP64 operations).
__device__ __forceinline__ Window make_window(const LinearParams &p, int64_t i) {
    Window w;
    const double ts = (double)i * p.t0_step - 0.5 * p.duration;
    const double te = ts + p.duration;
    w.ok = !(ts < 0.0 || te > p.t_end);
    w.lo = 0;
    w.hi = -1;
    w.phase = 0;
    if (!w.ok) return w;
    w.lo = (int64_t)ceil(ts / p.cadence);
    w.hi = (int64_t)floor(te / p.cadence);
    if (w.lo > w.hi) {
        w.ok = false;
        return w;
    }
    const long long ph = llround(4294967296.0 * ((((double)w.lo * p.cadence - ts) / p.duration) * (double)p.n_model));
    w.phase = ph < 0 ? 0ull : (uint64_t)ph;
    return w;
}

template <bool kStaged>
__global__ void __launch_bounds__(kThreads) linear_kernel(LinearParams p, const float *__restrict__ flux,
                                                          const float *__restrict__ ivar,
                                                          const float *__restrict__ model, float2 *__restrict__ fold,
                                                          float *__restrict__ depth, float *__restrict__ var,
                                                          float *__restrict__ lr, int64_t row_offset) {
    extern __shared__ float lds[];
    float *s_model = lds;                                           // [M]
    float2 *s_data = reinterpret_cast<float2 *>(lds + ((p.n_model + 1) & ~1));  // [span_cap]
    __shared__ int s_lo, s_hi;

    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool in_range = i < p.n_t0;
    Window w = make_window(p, in_range ? i : 0);
    w.ok = w.ok && in_range;

    for (int k = threadIdx.x; k < p.n_model; k += kThreads) s_model[k] = model[k];

    int64_t base = 0;
    if (kStaged) {
        if (threadIdx.x == 0) {
            s_lo = INT_MAX;
            s_hi = -1;
        }
        __syncthreads();
        if (w.ok) {
            atomicMin(&s_lo, (int)w.lo);
            atomicMax(&s_hi, (int)w.hi);
        }
        __syncthreads();
        base = s_lo;
        // (255 dt + D)/c + 1 points at most; span_cap carries a margin of 3
        const int64_t count = min((int64_t)s_hi - (int64_t)s_lo + 1, (int64_t)p.span_cap);
        for (int64_t q = threadIdx.x; q < count; q += kThreads) {
            const float wq = ivar[base + q];
            s_data[q] = make_float2(flux[base + q] * wq, wq);
        }
    }
    __syncthreads();

    double dfm = 0.0, dmm = 0.0;
    if (w.ok) {
        const int32_t last = p.n_model - 1;
        uint64_t ph = w.phase;
        int64_t n = w.lo;
        while (n <= w.hi) {
            const int64_t stop = min(w.hi + 1, n + kChunk);
            float sfm = 0.0f, smm = 0.0f;
            for (; n < stop; ++n) {
                const uint32_t k = min((uint32_t)(ph >> 32), (uint32_t)last);
                const float mk = s_model[k];
                float wf, wq;
                if (kStaged) {
                    const float2 d = s_data[n - base];
                    wf = d.x;
                    wq = d.y;
                } else {
                    wq = ivar[n];
                    wf = flux[n] * wq;
                }
                sfm = fmaf(wf, mk, sfm);
                smm = fmaf(wq * mk, mk, smm);
                ph += p.step_fx;
            }
            dfm += (double)sfm;
            dmm += (double)smm;
        }
    }
    if (!in_range) return;
    const int64_t e = row_offset + i;
    if (w.ok && dmm > 0.0) {
        fold[e] = make_float2((float)dfm, (float)dmm);
        if (depth) depth[e] = (float)(dfm / dmm);
        if (var) var[e] = (float)(1.0 / dmm);
        if (lr) lr[e] = (float)(0.5 * dfm * dfm / dmm);
    } else {
        fold[e] = make_float2(0.0f, 0.0f);
        if (depth) depth[e] = __builtin_nanf("");
        if (var) var[e] = __builtin_inff();
        if (lr) lr[e] = 0.0f;
    }
}

}  // namespace

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
    const size_t model_bytes = (size_t)((grid->n_model + 1) & ~1) * sizeof(float);
    for (int j = 0; j < grid->n_dur; ++j) {
        LinearParams p;
        p.cadence = grid->cadence;
        p.t0_step = grid->t0_step;
        p.duration = grid->durations[j];
        p.t_end = (double)(grid->n - 1) * grid->cadence;
        p.n_t0 = grid->n_t0;
        p.step_fx = grid->dur_step_fx[j];
        p.n_model = grid->n_model;
        // points covered by 256 consecutive windows, with margin for rounding
        const double span = ((double)(kThreads - 1) * grid->t0_step + p.duration) / grid->cadence + 4.0;
        const size_t staged_bytes = model_bytes + (size_t)std::ceil(span) * sizeof(float2);
        const bool staged = staged_bytes <= (size_t)kMaxLdsBytes;
        p.span_cap = staged ? (int32_t)std::ceil(span) : 0;
        const size_t lds = staged ? staged_bytes : model_bytes;
        const int64_t row = (int64_t)j * grid->n_t0;
        auto *f2 = reinterpret_cast<float2 *>(fold);
        if (staged)
            hipLaunchKernelGGL(linear_kernel<true>, dim3((unsigned)blocks), dim3(kThreads), lds, s, p, flux, ivar,
                               model, f2, depth, var, lr, row);
        else
            hipLaunchKernelGGL(linear_kernel<false>, dim3((unsigned)blocks), dim3(kThreads), lds, s, p, flux, ivar,
                               model, f2, depth, var, lr, row);
        if ((rc = check_launch("linear_search"))) return rc;
    }
    return CETRA_OK;
}
