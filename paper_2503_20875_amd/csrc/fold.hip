// Periodic search (Sec. 2.3) and best period.
//
// For period P_k, duration j and epoch i in [0, ceil(P_k/dt)), the transits
// sit at reference times i + o_m with o_m = round_half_up(m P_k/dt)
// (nearest-neighbour mapping, 32.32 fixed point).  Summing Eq. 4 over the
// transits at the inverse-variance common depth Z gives, with the linear
// search's per-window sums, LR = (sum S_fm)^2 / (2 sum S_mm), Z = sum S_fm /
// sum S_mm and var_Z = 1 / sum S_mm.  So the fold reads one float pair per
// (period, duration, transit) and the per-period reduction keeps the maximum.
//
// Work mapping (gfx950): a persistent grid of workgroups strides over units
// (period block of up to B periods, duration j, epoch chunk).  Every unit
// costs about B * I element reads whatever the period, because the transits
// of all epochs of one period tile the whole row.  A lane owns epochs and
// sums all B periods of its block at once: the B loads of one transit step
// are independent (memory-level parallelism) and hit nearly the same
// addresses, since neighbouring trial periods shift the transits by a few
// elements, so the block's periods share cache lines in L1/L2.  The sums
// that rank candidates are FP32 chunks of 32 transits folded into FP32
// totals; only each period's winner is recomputed in FP64 (epilogue).  Units
// are ordered period-block fastest, so the workgroups running at once sweep
// the same duration row, which then stays resident in each XCD's L2.
//
// Argmax: LR >= 0, so its FP32 bit pattern is monotone; the key
// (bits(LR) << 32) | (2^32 - 1 - (j I + i)) under a 64-bit atomicMax gives
// the maximum with ties to the smallest (j, i).  An epilogue recomputes the
// winner's sums in the same order to emit LR, Z and var_Z.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"
#include "stages.h"

namespace {

using cetra::dev::kThreads;

// Fold workspace of cetra_periodic_search_noalloc: one copy per device, held
// until the process ends.  Host code never passes this name to a kernel (on
// the host it is a stand-in, not a device address); it uses the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct FoldWork {
    uint64_t *key;     // [n_eval] argmax keys
    uint64_t *step;    // [n_eval] R_k = llround(2^32 P_k/dt)
    int32_t *n_ep;     // [n_eval] I_P
    int32_t *jr;       // [n_eval][2] allowed duration range after D_j < P_k
    int64_t *kidx;     // [n_eval] period index (-1 = invalid subset entry)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t workspace_bytes(int64_t n_eval) {
    size_t b = 0;
    b += align256(sizeof(uint64_t) * n_eval);
    b += align256(sizeof(uint64_t) * n_eval);
    b += align256(sizeof(int32_t) * n_eval);
    b += align256(sizeof(int32_t) * 2 * n_eval);
    b += align256(sizeof(int64_t) * n_eval);
    return b;
}

FoldWork carve(void *work, int64_t n_eval) {
    char *p = static_cast<char *>(work);
    FoldWork w;
    w.key = reinterpret_cast<uint64_t *>(p);
    p += align256(sizeof(uint64_t) * n_eval);
    w.step = reinterpret_cast<uint64_t *>(p);
    p += align256(sizeof(uint64_t) * n_eval);
    w.n_ep = reinterpret_cast<int32_t *>(p);
    p += align256(sizeof(int32_t) * n_eval);
    w.jr = reinterpret_cast<int32_t *>(p);
    p += align256(sizeof(int32_t) * 2 * n_eval);
    w.kidx = reinterpret_cast<int64_t *>(p);
    return w;
}

struct Durations {
    double d[CETRA_MAX_DURATIONS];
};

// Per-duration epoch strides of a coarser fold epoch grid; any = 0 when
// every stride is 1 (the fixed grid).
struct Strides {
    int32_t s[CETRA_MAX_DURATIONS];
    int32_t any;
};

// Per evaluated period: fixed-point step, epoch count, allowed durations
// (D_j < P_k, Sec. 2.3, intersected with the caller's range); clears its key.
__global__ void fold_setup_kernel(const double *__restrict__ periods, int64_t n_periods,
                                  const int32_t *__restrict__ jrange, const int64_t *__restrict__ subset,
                                  int64_t n_eval, double t0_step, int64_t n_t0, int32_t n_dur, Durations dur,
                                  FoldWork w) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_eval) return;
    const int64_t k = subset ? subset[s] : s;
    w.key[s] = 0;
    if (k < 0 || k >= n_periods) {
        w.kidx[s] = -1;
        w.step[s] = 0;
        w.n_ep[s] = 0;
        w.jr[2 * s] = 0;
        w.jr[2 * s + 1] = -1;
        return;
    }
    const cetra::dev::PeriodInfo pi = cetra::dev::period_info(
        periods[k], t0_step, n_t0, n_dur, dur.d, jrange ? jrange[2 * k] : 0,
        jrange ? jrange[2 * k + 1] : n_dur - 1);
    w.kidx[s] = k;
    w.step[s] = pi.step;
    w.n_ep[s] = pi.n_ep;
    w.jr[2 * s] = pi.jlo;
    w.jr[2 * s + 1] = pi.jhi;
}

// Persistent grid over units (period block of B periods, duration j, epoch
// chunk), ordered block-fastest; each unit is one dev::fold_unit (variant 0:
// lane epochs 64 apart; 2: adjacent lane epochs, 16-byte loads).  kStrided:
// rows whose epoch stride exceeds 1 run dev::fold_unit_strided on the
// coarser epoch grid (a separate instantiation, so the plain kernels keep
// their register budget).
template <int B, int kVariant, bool kStrided = false>
__global__ void __launch_bounds__(kThreads) fold_kernel(const float2 *__restrict__ fold, FoldWork w, int64_t n_eval,
                                                        int32_t I, int32_t n_chunks, int64_t n_units, Strides st) {
    const int64_t n_pblk = (n_eval + B - 1) / B;
    for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        const int64_t pb = u % n_pblk;
        const int64_t rest = u / n_pblk;
        const int32_t c = (int32_t)(rest % n_chunks);
        const int32_t j = (int32_t)(rest / n_chunks);
        const int64_t s0 = pb * B;
        uint64_t R[B];
        int32_t ipb[B];
        int32_t ipmax = 0;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t s = s0 + b;
            bool ok = s < n_eval;
            if (ok) ok = w.kidx[s] >= 0 && j >= w.jr[2 * s] && j <= w.jr[2 * s + 1];
            R[b] = ok ? w.step[s] : 0;
            ipb[b] = ok ? w.n_ep[s] : 0;
            ipmax = max(ipmax, ipb[b]);
        }
        if (ipmax == 0) continue;
        if (kStrided && st.s[j] > 1) {
            // coarser epoch grid for this duration: count epochs in strides
            const int32_t sj = st.s[j];
#pragma unroll
            for (int b = 0; b < B; ++b) ipb[b] = (int32_t)(((int64_t)ipb[b] + sj - 1) / sj);
            const int32_t ipc = (int32_t)(((int64_t)ipmax + sj - 1) / sj);
            const int32_t chunk = (ipc + n_chunks - 1) / n_chunks;
            const int32_t e_lo = c * chunk;
            const int32_t e_hi = min(ipc, e_lo + chunk);
            if (e_lo < e_hi)
                cetra::dev::fold_unit_strided<B>(fold + (int64_t)j * I, j, I, sj, R, ipb, e_lo, e_hi, w.key + s0);
            continue;
        }
        const int32_t chunk = (ipmax + n_chunks - 1) / n_chunks;
        const int32_t e_lo = c * chunk;
        const int32_t e_hi = min(ipmax, e_lo + chunk);
        if (e_lo >= e_hi) continue;
        cetra::dev::fold_unit<B, kVariant == 2>(fold + (int64_t)j * I, j, I, R, ipb, e_lo, e_hi, w.key + s0);
    }
}

// Null record for every period (used before a subset search).
__global__ void fold_null_kernel(int64_t n, float *lr, int32_t *ep, int32_t *du, float *z, float *zv) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    lr[k] = 0.0f;
    ep[k] = -1;
    du[k] = -1;
    z[k] = __builtin_nanf("");
    zv[k] = __builtin_inff();
}

// Decode each period's winner and recompute its sums in the fold's order.
__global__ void fold_epilogue_kernel(const float2 *__restrict__ fold, FoldWork w, int64_t n_eval, int64_t n_t0,
                                     int32_t n_dur, float *lr, int32_t *ep, int32_t *du, float *z, float *zv) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_eval) return;
    const int64_t k = w.kidx[s];
    if (k < 0) return;
    cetra::dev::fold_decode(fold, n_t0, n_dur, w.step[s], w.key[s], lr + k, ep + k, du + k, z + k, zv + k);
}

__global__ void __launch_bounds__(1024) best_kernel(const double *__restrict__ periods, int64_t n,
                                                    const float *__restrict__ lr, const int32_t *__restrict__ ep,
                                                    const int32_t *__restrict__ du, const float *__restrict__ z,
                                                    const float *__restrict__ zv, double t0_step, double t_origin,
                                                    Durations dur, cetra_best_record *out) {
    __shared__ float s_lr[1024];
    __shared__ int64_t s_k[1024];
    float bl = -1.0f;
    int64_t bk = -1;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
        if (ep[k] < 0) continue;
        if (lr[k] > bl) {
            bl = lr[k];
            bk = k;
        }
    }
    s_lr[threadIdx.x] = bl;
    s_k[threadIdx.x] = bk;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const float ol = s_lr[threadIdx.x + h];
            const int64_t ok = s_k[threadIdx.x + h];
            const int64_t mk = s_k[threadIdx.x];
            if (ok >= 0 && (mk < 0 || ol > s_lr[threadIdx.x] || (ol == s_lr[threadIdx.x] && ok < mk))) {
                s_lr[threadIdx.x] = ol;
                s_k[threadIdx.x] = ok;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    cetra_best_record b;
    const int64_t k = s_k[0];
    b.k = k;
    if (k < 0) {
        b.epoch = -1;
        b.dur = -1;
        b.period = b.duration = b.t0 = b.t0_abs = __builtin_nan("");
        b.lr = 0.0;
        b.depth = __builtin_nan("");
        b.depth_var = __builtin_inf();
        b.snr = 0.0;
    } else {
        b.epoch = ep[k];
        b.dur = du[k];
        b.period = periods[k];
        b.duration = dur.d[b.dur];
        b.t0 = (double)b.epoch * t0_step;
        b.t0_abs = t_origin + b.t0;
        b.lr = (double)lr[k];
        b.depth = (double)z[k];
        b.depth_var = (double)zv[k];
        b.snr = b.depth / sqrt(b.depth_var);
    }
    *out = b;
}

Durations pack_durations(const cetra_grid *g) {
    Durations d;
    for (int j = 0; j < CETRA_MAX_DURATIONS; ++j) d.d[j] = j < g->n_dur ? g->durations[j] : 0.0;
    return d;
}

}  // namespace

using namespace cetra;

extern "C" int cetra_periodic_workspace(const cetra_grid *grid, int64_t n_eval, size_t *bytes) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(bytes != nullptr, "periodic_workspace: NULL output");
    CETRA_REQUIRE(n_eval >= 0, "periodic_workspace: n_eval < 0");
    *bytes = workspace_bytes(n_eval);
    return CETRA_OK;
}

namespace {

int periodic_search(void *stream, const cetra_grid *grid, const float *fold, const double *periods,
                    int64_t n_periods, const int32_t *jrange, const int64_t *subset, int64_t n_subset,
                    const int32_t *stride, void *work, size_t work_bytes, float *lr, int32_t *epoch, int32_t *dur,
                    float *depth, float *depth_var) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    Strides st{};
    st.any = 0;
    for (int j = 0; j < CETRA_MAX_DURATIONS; ++j) st.s[j] = 1;
    if (stride) {
        for (int j = 0; j < grid->n_dur; ++j) {
            if (stride[j] < 1) return set_error(CETRA_ERR_INVALID, "periodic_search: stride[%d] = %d < 1", j, stride[j]);
            st.s[j] = stride[j];
            st.any |= stride[j] > 1;
        }
    }
    CETRA_REQUIRE(fold && lr && epoch && dur && depth && depth_var, "periodic_search: NULL pointer");
    CETRA_REQUIRE(n_periods >= 0 && (n_periods == 0 || periods), "periodic_search: bad periods");
    CETRA_REQUIRE(!subset || n_subset >= 0, "periodic_search: bad subset");
    // buffer byte offsets (element index + saturated transit offset) * 8 must fit 32 bits
    if (grid->n_t0 >= (int64_t)1 << 28)
        return set_error(CETRA_ERR_RANGE, "periodic_search: I must be < 2^28");
    const int64_t n_eval = subset ? n_subset : n_periods;
    if (work_bytes < workspace_bytes(n_eval) || (n_eval > 0 && !work))
        return set_error(CETRA_ERR_WORKSPACE, "periodic_search: workspace needs %zu bytes",
                         workspace_bytes(n_eval));
    hipStream_t s = as_stream(stream);
    if (subset && n_periods > 0) {
        hipLaunchKernelGGL(fold_null_kernel, dim3((unsigned)ceil_div(n_periods, 256)), dim3(256), 0, s, n_periods,
                           lr, epoch, dur, depth, depth_var);
        if ((rc = check_launch("periodic_search/null"))) return rc;
    }
    if (n_eval == 0) return CETRA_OK;
    FoldWork w = carve(work, n_eval);
    const Durations d = pack_durations(grid);
    hipLaunchKernelGGL(fold_setup_kernel, dim3((unsigned)ceil_div(n_eval, 256)), dim3(256), 0, s, periods,
                       n_periods, jrange, subset, n_eval, grid->t0_step, grid->n_t0, grid->n_dur, d, w);
    if ((rc = check_launch("periodic_search/setup"))) return rc;

    const cetra_tuning tu = current_tuning();
    const int B = tu.fold_period_block;
    const int64_t n_pblk = ceil_div(n_eval, B);
    // persistent grid: no more workgroups than can be resident at once
    const void *kern = nullptr;
    switch ((tu.fold_variant == 2 ? 3 : 0) + (B == 4 ? 0 : B == 8 ? 1 : 2)) {
        case 0: kern = (const void *)fold_kernel<4, 0>; break;
        case 1: kern = (const void *)fold_kernel<8, 0>; break;
        case 2: kern = (const void *)fold_kernel<16, 0>; break;
        case 3: kern = (const void *)fold_kernel<4, 2>; break;
        case 4: kern = (const void *)fold_kernel<8, 2>; break;
        default: kern = (const void *)fold_kernel<16, 2>; break;
    }
    if (st.any)  // a coarser epoch grid: its own instantiation, variant 2 for the rows of stride 1
        kern = B == 4 ? (const void *)fold_kernel<4, 2, true>
             : B == 8 ? (const void *)fold_kernel<8, 2, true>
                      : (const void *)fold_kernel<16, 2, true>;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kThreads, 0) != hipSuccess || occ <= 0) occ = 1;
    const int64_t wgs = (int64_t)device_cu_count() * std::min(tu.fold_wgs_per_cu, occ);
    const int64_t base_units = n_pblk * grid->n_dur;
    int64_t n_chunks = ceil_div((int64_t)tu.fold_units_per_wg * wgs, base_units);
    n_chunks = std::max<int64_t>(1, std::min<int64_t>(n_chunks, 64));
    const int64_t n_units = base_units * n_chunks;
    const int64_t grid_wgs = std::min<int64_t>(wgs, n_units);
    const auto *f2 = reinterpret_cast<const float2 *>(fold);
    const int32_t I = (int32_t)grid->n_t0;
    const int32_t n_chunks32 = (int32_t)n_chunks;
    void *args[] = {(void *)&f2,         (void *)&w,       (void *)&n_eval, (void *)&I,
                    (void *)&n_chunks32, (void *)&n_units, (void *)&st};
    const hipError_t le = hipLaunchKernel(kern, dim3((unsigned)grid_wgs), dim3(kThreads), args, 0, s);
    if (le != hipSuccess) return set_error(CETRA_ERR_HIP, "periodic_search/fold: %s", hipGetErrorString(le));
    hipLaunchKernelGGL(fold_epilogue_kernel, dim3((unsigned)ceil_div(n_eval, 256)), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(fold), w, n_eval, grid->n_t0, grid->n_dur, lr, epoch, dur,
                       depth, depth_var);
    return check_launch("periodic_search/epilogue");
}

}  // namespace

extern "C" int cetra_periodic_search(void *stream, const cetra_grid *grid, const float *fold, const double *periods,
                                     int64_t n_periods, const int32_t *jrange, const int64_t *subset,
                                     int64_t n_subset, void *work, size_t work_bytes, float *lr, int32_t *epoch,
                                     int32_t *dur, float *depth, float *depth_var) {
    return periodic_search(stream, grid, fold, periods, n_periods, jrange, subset, n_subset, nullptr, work,
                           work_bytes, lr, epoch, dur, depth, depth_var);
}

extern "C" int cetra_periodic_search_strided(void *stream, const cetra_grid *grid, const float *fold,
                                             const double *periods, int64_t n_periods, const int32_t *jrange,
                                             const int64_t *subset, int64_t n_subset, const int32_t *stride,
                                             void *work, size_t work_bytes, float *lr, int32_t *epoch, int32_t *dur,
                                             float *depth, float *depth_var) {
    return periodic_search(stream, grid, fold, periods, n_periods, jrange, subset, n_subset, stride, work,
                           work_bytes, lr, epoch, dur, depth, depth_var);
}

namespace {

// Device address of `scratch` on the current device, resolved once per device
// (each GPU holds its own copy of the array at its own address).
int scratch_address(void **out) {
    static std::mutex mu;
    static std::vector<void *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(CETRA_ERR_HIP, "periodic_search_noalloc: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(CETRA_ERR_HIP, "periodic_search_noalloc: scratch address: %s", hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return CETRA_OK;
}

}  // namespace

extern "C" int cetra_periodic_search_noalloc_limit(const cetra_grid *grid, int64_t *max_eval) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(max_eval != nullptr, "periodic_search_noalloc_limit: NULL output");
    int64_t lo = 0, hi = (int64_t)(kScratchBytes / 8);  // workspace_bytes grows with n_eval
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (workspace_bytes(mid) <= kScratchBytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    *max_eval = lo;
    return CETRA_OK;
}

extern "C" int cetra_periodic_search_noalloc(void *stream, const cetra_grid *grid, const float *fold,
                                             const double *periods, int64_t n_periods, const int32_t *jrange,
                                             const int64_t *subset, int64_t n_subset, float *lr, int32_t *epoch,
                                             int32_t *dur, float *depth, float *depth_var) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(n_periods >= 0 && (!subset || n_subset >= 0), "periodic_search_noalloc: negative size");
    const int64_t n_eval = subset ? n_subset : n_periods;
    if (workspace_bytes(n_eval) > kScratchBytes) {
        int64_t lim = 0;
        cetra_periodic_search_noalloc_limit(grid, &lim);
        return set_error(CETRA_ERR_RANGE,
                         "periodic_search_noalloc: %lld evaluated periods exceed the fixed scratch of %zu bytes "
                         "(at most %lld periods)", (long long)n_eval, kScratchBytes, (long long)lim);
    }
    void *work = nullptr;
    if ((rc = scratch_address(&work))) return rc;
    return periodic_search(stream, grid, fold, periods, n_periods, jrange, subset, n_subset, nullptr, work,
                           kScratchBytes, lr, epoch, dur, depth, depth_var);
}

extern "C" int cetra_best(void *stream, const cetra_grid *grid, const double *periods, int64_t n_periods,
                          const float *lr, const int32_t *epoch, const int32_t *dur, const float *depth,
                          const float *depth_var, cetra_best_record *out) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(out && (n_periods == 0 || (periods && lr && epoch && dur && depth && depth_var)),
                  "best: NULL pointer");
    CETRA_REQUIRE(n_periods >= 0, "best: n_periods < 0");
    hipLaunchKernelGGL(best_kernel, dim3(1), dim3(1024), 0, as_stream(stream), periods, n_periods, lr, epoch, dur,
                       depth, depth_var, grid->t0_step, grid->t_origin, pack_durations(grid), out);
    return check_launch("best");
}
