// Batched search: many light curves of uneven length searched by a short
// sequence of persistent work-queue launches (the method is the same per
// curve: Sec. 2.1 setup, Sec. 2.2 linear search, Sec. 2.3 periodic search).
//
// Host plan.  Curves are ordered by descending fold cost (longest first) and
// packed into generations whose resampled light curves and fold-ready arrays
// fit one half of a caller-sized arena; generations alternate between the two
// halves.  Work items:
//   RES  (curve, 1024 grid points)       resampling; also clears the curve's
//                                         argmax keys
//   LIN  (curve, duration, 64 tiles)     linear search, 16 384 reference times
//   FOLD (curve, duration, B periods)    fold + argmax over all epochs
//   EPI  (curve, 256 periods)            decode winners, per-curve best key
//   FIN  (curve)                         best-period record
// Launches (one stream; each a persistent grid draining its own item range
// through one atomic counter; the items of a launch are independent):
//   RES(0); LIN(0); then for each generation g:
//   FOLD(g)+RES(g+1); EPI(g)+LIN(g+1); FIN(g).
// Stream order provides every dependency (stage s of a curve after stage s-1;
// RES(g+2) reuses the arena half of generation g after EPI(g)), and kernel
// boundaries make each launch's writes visible to every XCD, so no workgroup
// ever waits on another.  The whole sequence can be captured in one HIP graph.
//
// Every item runs the same per-item device code as the single-curve entry
// points (stages.h), so batched results are bit-identical to single calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "common.h"
#include "stages.h"

namespace {

using cetra::dev::kThreads;

enum Stage : int32_t { kRes = 0, kLin = 1, kFold = 2, kEpi = 3, kFin = 4, kStages = 5 };
constexpr int kResPoints = 1024;
constexpr int kLinTilesPerItem = 64;
constexpr int kEpiPeriods = 256;
constexpr bool kBatchSearchEnabled = false;

struct CurveDesc {
    int64_t obs_off, n_obs;
    int64_t per_off, n_per;
    int64_t arena_off;       // bytes from the start of the arena (both halves)
    int64_t n_items[kStages];
    int32_t gen;
    int32_t n_lin_per_dur;   // LIN items per duration
    int32_t n_pblk;          // period blocks
    int32_t pad;
};

struct Segment {
    int64_t first;   // first item index
    int64_t count;
    int32_t curve;
    int32_t stage;
};

struct Launch {
    int64_t first, end;  // item range [first, end)
};

struct TablesHeader {
    int64_t n_curves, n_segments, n_items, n_gens, n_launches;
    int64_t off_curves, off_grids, off_segments, off_launches;  // byte offsets in the tables
    int64_t tables_bytes;
    int64_t off_counters, off_keys, off_best_keys, off_arena;   // byte offsets in the workspace
    int64_t workspace_bytes, total_periods;
    int32_t period_block, lds_bytes;
};

struct BatchArgs {
    const double *t;
    const float *f, *sigma, *model;
    const double *periods;
    char *work;
    const int32_t *cancel;
    float *lr, *depth, *depth_var;
    int32_t *epoch, *dur;
    cetra_best_record *best;
    int32_t *status;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------- device side
struct Tables {
    const TablesHeader *h;
    const CurveDesc *curves;
    const cetra_grid *grids;
    const Segment *segs;
    const Launch *launches;
    unsigned long long *heads;  // [n_launches] work-queue counters
    uint64_t *keys;             // [total periods]
    uint64_t *best_keys;        // [n_curves]
    char *arena;
};

__device__ __forceinline__ Tables bind(char *work) {
    Tables tb;
    tb.h = reinterpret_cast<const TablesHeader *>(work);
    tb.curves = reinterpret_cast<const CurveDesc *>(work + tb.h->off_curves);
    tb.grids = reinterpret_cast<const cetra_grid *>(work + tb.h->off_grids);
    tb.segs = reinterpret_cast<const Segment *>(work + tb.h->off_segments);
    tb.launches = reinterpret_cast<const Launch *>(work + tb.h->off_launches);
    tb.heads = reinterpret_cast<unsigned long long *>(work + tb.h->off_counters);
    tb.keys = reinterpret_cast<uint64_t *>(work + tb.h->off_keys);
    tb.best_keys = reinterpret_cast<uint64_t *>(work + tb.h->off_best_keys);
    tb.arena = work + tb.h->off_arena;
    return tb;
}

// Clears the work-queue counters and the status word (a kernel, not a
// memset, so the launch sequence can be captured in a graph).
__global__ void batch_init_kernel(char *work, int32_t *status) {
    const Tables tb = bind(work);
    for (int64_t i = threadIdx.x; i < tb.h->n_launches; i += blockDim.x) tb.heads[i] = 0ull;
    if (threadIdx.x == 0) status[0] = 0;
}

__device__ __forceinline__ float2 *curve_fold(const Tables &tb, const CurveDesc &cd, const cetra_grid &g) {
    return reinterpret_cast<float2 *>(tb.arena + cd.arena_off + align256(sizeof(float) * 2 * (size_t)g.n));
}

template <int B>
__device__ void run_item(const Tables &tb, const BatchArgs &a, int32_t c, int32_t stage, int64_t idx, float *lds,
                         int *s_bounds) {
    const CurveDesc &cd = tb.curves[c];
    const cetra_grid &g = tb.grids[c];
    float *flux = reinterpret_cast<float *>(tb.arena + cd.arena_off);
    float *ivar = flux + g.n;
    float2 *fold = curve_fold(tb, cd, g);
    const int64_t I = g.n_t0;
    if (stage == kRes) {
        const int64_t q0 = idx * kResPoints;
        for (int64_t q = q0 + threadIdx.x; q < min(q0 + kResPoints, g.n); q += kThreads)
            cetra::dev::resample_point(a.t + cd.obs_off, a.f + cd.obs_off, a.sigma + cd.obs_off, cd.n_obs,
                                       g.t_first, g.cadence, g.n_pad, q, flux, ivar);
        const int64_t nres = cd.n_items[kRes];
        const int64_t k0 = cd.n_per * idx / nres, k1 = cd.n_per * (idx + 1) / nres;
        for (int64_t k = k0 + threadIdx.x; k < k1; k += kThreads) tb.keys[cd.per_off + k] = 0;
        if (idx == 0 && threadIdx.x == 0) tb.best_keys[c] = 0;
    } else if (stage == kLin) {
        const int32_t j = (int32_t)(idx / cd.n_lin_per_dur);
        const int64_t t0 = (idx % cd.n_lin_per_dur) * kLinTilesPerItem;
        cetra::dev::LinearParams p = cetra::dev::linear_params(g, j);
        const double span = cetra::dev::linear_span(g.t0_step, g.durations[j], g.cadence);
        const int64_t need = (int64_t)((g.n_model + 1) & ~1) * 4 + (int64_t)ceil(span) * 8;
        p.span_cap = need <= tb.h->lds_bytes ? (int32_t)ceil(span) : 0;
        const int64_t n_tiles = (I + kThreads - 1) / kThreads;
        for (int64_t tile = t0; tile < min(t0 + kLinTilesPerItem, n_tiles); ++tile)
            cetra::dev::linear_tile(p, tile * kThreads, flux, ivar, a.model, fold + (int64_t)j * I, nullptr,
                                    nullptr, nullptr, lds, s_bounds);
    } else if (stage == kFold) {
        const int32_t j = (int32_t)(idx / cd.n_pblk);
        const int64_t pb = idx % cd.n_pblk;
        uint64_t R[B];
        int32_t ipb[B];
        int32_t ipmax = 0;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t k = pb * B + b;
            R[b] = 0;
            ipb[b] = 0;
            if (k < cd.n_per) {
                const cetra::dev::PeriodInfo pi = cetra::dev::period_info(a.periods[cd.per_off + k], g.t0_step, I,
                                                                          g.n_dur, g.durations, 0, g.n_dur - 1);
                if (j >= pi.jlo && j <= pi.jhi) {
                    R[b] = pi.step;
                    ipb[b] = pi.n_ep;
                }
            }
            ipmax = max(ipmax, ipb[b]);
        }
        if (ipmax > 0)
            cetra::dev::fold_unit<B>(fold + (int64_t)j * I, j, (int32_t)I, R, ipb, 0, ipmax,
                                     tb.keys + cd.per_off + pb * B);
    } else if (stage == kEpi) {
        const int64_t k = idx * kEpiPeriods + threadIdx.x;
        uint64_t bk = 0;
        if (k < cd.n_per) {
            const int64_t o = cd.per_off + k;
            const cetra::dev::PeriodInfo pi =
                cetra::dev::period_info(a.periods[o], g.t0_step, I, g.n_dur, g.durations, 0, g.n_dur - 1);
            const float l = cetra::dev::fold_decode(fold, I, g.n_dur, pi.step, tb.keys[o], a.lr + o, a.epoch + o,
                                                    a.dur + o, a.depth + o, a.depth_var + o);
            if (a.epoch[o] >= 0) bk = ((uint64_t)__float_as_uint(l) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
        }
        bk = cetra::dev::wave_max_u64(bk);
        if ((threadIdx.x & 63) == 0 && bk != 0) atomicMax((unsigned long long *)&tb.best_keys[c], bk);
    } else if (threadIdx.x == 0) {  // kFin
        const uint64_t bk = tb.best_keys[c];
        cetra_best_record r;
        if (bk == 0) {
            r.k = -1;
            r.epoch = -1;
            r.dur = -1;
            r.period = r.duration = r.t0 = r.t0_abs = __builtin_nan("");
            r.lr = 0.0;
            r.depth = __builtin_nan("");
            r.depth_var = __builtin_inf();
            r.snr = 0.0;
        } else {
            const int64_t k = (int64_t)(0xFFFFFFFFu - (uint32_t)(bk & 0xFFFFFFFFull));
            const int64_t o = cd.per_off + k;
            r.k = k;
            r.epoch = a.epoch[o];
            r.dur = a.dur[o];
            r.period = a.periods[o];
            r.duration = g.durations[r.dur];
            r.t0 = (double)r.epoch * g.t0_step;
            r.t0_abs = g.t_origin + r.t0;
            r.lr = (double)a.lr[o];
            r.depth = (double)a.depth[o];
            r.depth_var = (double)a.depth_var[o];
            r.snr = r.depth / sqrt(r.depth_var);
        }
        a.best[c] = r;
    }
}

// One launch of the sequence: drain the item range of launch `li`.
template <int B>
__global__ void __launch_bounds__(kThreads) batch_kernel(BatchArgs a, int32_t li) {
    extern __shared__ float lds[];
    __shared__ int s_bounds[2];
    __shared__ long long s_item;
    const Tables tb = bind(a.work);
    const Launch L = tb.launches[li];
    for (;;) {
        if (threadIdx.x == 0) {
            long long item = -1;
            if (a.cancel && __hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0) {
                atomicOr(a.status, 1);
            } else {
                const unsigned long long v = atomicAdd(&tb.heads[li], 1ull);
                if ((long long)v < L.end - L.first) item = L.first + (long long)v;
            }
            s_item = item;
        }
        __syncthreads();
        const long long item = s_item;
        __syncthreads();  // s_item is rewritten at the top of the next round
        if (item < 0) break;
        // segment of the item: last segment whose first index is <= item
        int64_t lo = 0, hi = tb.h->n_segments - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (tb.segs[mid].first <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const Segment sg = tb.segs[lo];
        run_item<B>(tb, a, sg.curve, sg.stage, item - sg.first, lds, s_bounds);
    }
}

}  // namespace

// --------------------------------------------------------------- host side
struct cetra_batch_plan {
    std::vector<char> tables;  // header, curves, grids, segments, launches
    TablesHeader h;
    int64_t arena_bytes;
};

using namespace cetra;

extern "C" int cetra_batch_plan_create(const cetra_batch_desc *d, cetra_batch_plan **out) {
    clear_error();
    CETRA_REQUIRE(d && out && d->grids && d->obs_offsets && d->period_offsets, "batch_plan: NULL pointer");
    CETRA_REQUIRE(d->n_curves >= 1, "batch_plan: n_curves must be >= 1");
    const int n = d->n_curves;
    const cetra_grid &g0 = d->grids[0];
    int rc;
    for (int c = 0; c < n; ++c) {
        if ((rc = check_grid(&d->grids[c]))) return rc;
        const cetra_grid &g = d->grids[c];
        CETRA_REQUIRE(g.n_dur == g0.n_dur && g.n_model == g0.n_model, "batch_plan: curves must share J and M");
        for (int j = 0; j < g.n_dur; ++j)
            CETRA_REQUIRE(g.durations[j] == g0.durations[j], "batch_plan: curves must share the durations");
        CETRA_REQUIRE(d->obs_offsets[c + 1] >= d->obs_offsets[c], "batch_plan: obs_offsets not ascending");
        CETRA_REQUIRE(d->period_offsets[c + 1] >= d->period_offsets[c], "batch_plan: period_offsets not ascending");
        if (g.n_t0 >= ((int64_t)1 << 28) || g.n >= INT32_MAX)
            return set_error(CETRA_ERR_RANGE, "batch_plan: curve %d too long", c);
    }
    const int B = d->fold_period_block ? d->fold_period_block : current_tuning().fold_period_block;
    CETRA_REQUIRE(B == 4 || B == 8, "batch_plan: fold_period_block must be 4 or 8");
    const int J = g0.n_dur;

    std::vector<CurveDesc> cds(n);
    std::vector<int64_t> need(n);
    std::vector<double> cost(n);
    int64_t lds = 0;
    for (int c = 0; c < n; ++c) {
        const cetra_grid &g = d->grids[c];
        CurveDesc &cd = cds[c];
        std::memset(&cd, 0, sizeof cd);
        cd.obs_off = d->obs_offsets[c];
        cd.n_obs = d->obs_offsets[c + 1] - d->obs_offsets[c];
        cd.per_off = d->period_offsets[c];
        cd.n_per = d->period_offsets[c + 1] - d->period_offsets[c];
        const int64_t n_tiles = ceil_div(g.n_t0, kThreads);
        cd.n_lin_per_dur = (int32_t)ceil_div(n_tiles, kLinTilesPerItem);
        cd.n_pblk = (int32_t)ceil_div(std::max<int64_t>(cd.n_per, 1), B);
        cd.n_items[kRes] = ceil_div(g.n, kResPoints);
        cd.n_items[kLin] = (int64_t)J * cd.n_lin_per_dur;
        cd.n_items[kFold] = (int64_t)J * cd.n_pblk;
        cd.n_items[kEpi] = ceil_div(std::max<int64_t>(cd.n_per, 1), kEpiPeriods);
        cd.n_items[kFin] = 1;
        need[c] = (int64_t)align256(sizeof(float) * 2 * (size_t)g.n) + (int64_t)align256(8 * (size_t)J * g.n_t0);
        cost[c] = (double)cd.n_per * J * (double)g.n_t0;
        for (int j = 0; j < J; ++j) {
            int32_t span_cap = 0;
            lds = std::max<int64_t>(lds, (int64_t)linear_lds_bytes(&g, j, &span_cap));
        }
    }
    const int64_t biggest = *std::max_element(need.begin(), need.end());
    int64_t arena = d->arena_bytes > 0 ? d->arena_bytes : 2 * biggest;
    if (arena < 2 * biggest)
        return set_error(CETRA_ERR_WORKSPACE, "batch_plan: arena of %lld bytes cannot hold the longest curve "
                         "twice (%lld bytes)", (long long)arena, (long long)(2 * biggest));
    const int64_t half = (arena / 2) & ~(int64_t)255;

    // longest first, packed into generations that fit one arena half
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<std::vector<int>> gens;
    int64_t used = half;  // forces a new generation at the first curve
    for (int c : order) {
        if (used + need[c] > half) {
            gens.emplace_back();
            used = 0;
        }
        cds[c].gen = (int32_t)gens.size() - 1;
        cds[c].arena_off = (gens.size() - 1) % 2 * half + used;
        used += need[c];
        gens.back().push_back(c);
    }
    // Queue order: RES(0) LIN(0) | RES(1) LIN(1) FOLD(0) EPI(0) FIN(0) |
    // RES(2) LIN(2) FOLD(1) EPI(1) FIN(1) | ... so the next generation's
    // resampling and linear search are queued ahead of this generation's fold.
    // RES(g+1) waits for FIN(g-1) (same arena half), which is queued earlier.
    // Launch sequence: RES(0); LIN(0); then per generation g:
    // FOLD(g)+RES(g+1); EPI(g)+LIN(g+1); FIN(g).  Segments are listed in
    // launch order, so every launch owns a contiguous item range.
    std::vector<Segment> segs;
    std::vector<Launch> launches;
    int64_t item = 0;
    auto emit = [&](int g, int st) {
        for (int c : gens[g]) {
            Segment sg;
            sg.first = item;
            sg.count = cds[c].n_items[st];
            sg.curve = c;
            sg.stage = st;
            segs.push_back(sg);
            item += sg.count;
        }
    };
    const int G = (int)gens.size();
    int64_t f0 = item;
    emit(0, kRes);
    launches.push_back(Launch{f0, item});
    f0 = item;
    emit(0, kLin);
    launches.push_back(Launch{f0, item});
    for (int g = 0; g < G; ++g) {
        f0 = item;
        emit(g, kFold);
        if (g + 1 < G) emit(g + 1, kRes);
        launches.push_back(Launch{f0, item});
        f0 = item;
        emit(g, kEpi);
        if (g + 1 < G) emit(g + 1, kLin);
        launches.push_back(Launch{f0, item});
        f0 = item;
        emit(g, kFin);
        launches.push_back(Launch{f0, item});
    }

    TablesHeader h;
    std::memset(&h, 0, sizeof h);
    h.n_curves = n;
    h.n_segments = (int64_t)segs.size();
    h.n_items = item;
    h.n_gens = G;
    h.n_launches = (int64_t)launches.size();
    size_t off = align256(sizeof(TablesHeader));
    h.off_curves = off;
    off += align256(sizeof(CurveDesc) * n);
    h.off_grids = off;
    off += align256(sizeof(cetra_grid) * n);
    h.off_segments = off;
    off += align256(sizeof(Segment) * segs.size());
    h.off_launches = off;
    off += align256(sizeof(Launch) * launches.size());
    h.tables_bytes = off;
    h.off_counters = off;
    off += align256(sizeof(unsigned long long) * launches.size());
    h.total_periods = d->period_offsets[n] - d->period_offsets[0];
    h.off_keys = off;
    off += align256(sizeof(uint64_t) * std::max<int64_t>(d->period_offsets[n], 1));
    h.off_best_keys = off;
    off += align256(sizeof(uint64_t) * n);
    h.off_arena = off;
    off += 2 * half;
    h.workspace_bytes = off;
    h.period_block = B;
    h.lds_bytes = (int32_t)lds;

    auto *plan = new (std::nothrow) cetra_batch_plan;
    if (!plan) return set_error(CETRA_ERR_INVALID, "batch_plan: out of host memory");
    plan->h = h;
    plan->arena_bytes = 2 * half;
    plan->tables.assign(h.tables_bytes, 0);
    std::memcpy(plan->tables.data(), &h, sizeof h);
    std::memcpy(plan->tables.data() + h.off_curves, cds.data(), sizeof(CurveDesc) * n);
    std::memcpy(plan->tables.data() + h.off_grids, d->grids, sizeof(cetra_grid) * n);
    std::memcpy(plan->tables.data() + h.off_segments, segs.data(), sizeof(Segment) * segs.size());
    std::memcpy(plan->tables.data() + h.off_launches, launches.data(), sizeof(Launch) * launches.size());
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
    info->workspace_bytes = (size_t)plan->h.workspace_bytes;
    info->tables_bytes = (size_t)plan->h.tables_bytes;
    info->arena_bytes = (size_t)plan->arena_bytes;
    info->n_items = plan->h.n_items;
    info->n_generations = plan->h.n_gens;
    info->n_launches = plan->h.n_launches;
    info->total_periods = plan->h.total_periods;
    info->period_block = plan->h.period_block;
    info->lds_bytes = plan->h.lds_bytes;
    return CETRA_OK;
}

extern "C" int cetra_batch_tables(const cetra_batch_plan *plan, void *host_dst, size_t bytes) {
    clear_error();
    CETRA_REQUIRE(plan && host_dst, "batch_tables: NULL pointer");
    if (bytes < plan->tables.size())
        return set_error(CETRA_ERR_WORKSPACE, "batch_tables: need %zu bytes", plan->tables.size());
    std::memcpy(host_dst, plan->tables.data(), plan->tables.size());
    return CETRA_OK;
}

extern "C" int cetra_batch_search(const cetra_batch_plan *plan, void *stream, const double *t, const float *f,
                                  const float *sigma, const float *model, const double *periods, void *work,
                                  size_t work_bytes, const int32_t *cancel, float *lr, int32_t *epoch, int32_t *dur,
                                  float *depth, float *depth_var, cetra_best_record *best, int32_t *status) {
    clear_error();
    // Switched off: on the MI355X both launch designs of this path (a single
    // persistent launch with per-curve dependency waits, and the present
    // sequence of wait-free launches) failed to finish a 10-curve batch
    // within the time limit, and the cause has not been found.  Nothing is
    // enqueued until it is.
    if (!kBatchSearchEnabled)
        return set_error(CETRA_ERR_INVALID, "batch_search: switched off (did not complete on the GPU; "
                         "cause under investigation)");
    CETRA_REQUIRE(plan, "batch_search: NULL plan");
    CETRA_REQUIRE(model && work && best && status && lr && epoch && dur && depth && depth_var,
                  "batch_search: NULL pointer");
    CETRA_REQUIRE(plan->h.total_periods == 0 || periods, "batch_search: NULL periods");
    if (work_bytes < (size_t)plan->h.workspace_bytes)
        return set_error(CETRA_ERR_WORKSPACE, "batch_search: workspace needs %lld bytes",
                         (long long)plan->h.workspace_bytes);
    hipStream_t s = as_stream(stream);
    BatchArgs a;
    a.t = t;
    a.f = f;
    a.sigma = sigma;
    a.model = model;
    a.periods = periods;
    a.work = static_cast<char *>(work);
    a.cancel = cancel;
    a.lr = lr;
    a.depth = depth;
    a.depth_var = depth_var;
    a.epoch = epoch;
    a.dur = dur;
    a.best = best;
    a.status = status;
    hipLaunchKernelGGL(batch_init_kernel, dim3(1), dim3(256), 0, s, a.work, status);
    int rc = check_launch("batch_search/init");
    if (rc) return rc;
    const size_t lds = (size_t)plan->h.lds_bytes;
    int occ = 0;
    hipError_t oe = plan->h.period_block == 4
                        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_kernel<4>, kThreads, lds)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_kernel<8>, kThreads, lds);
    if (oe != hipSuccess || occ <= 0) occ = 1;
    const int64_t resident = (int64_t)device_cu_count() * occ;
    const Launch *ls = reinterpret_cast<const Launch *>(plan->tables.data() + plan->h.off_launches);
    for (int64_t li = 0; li < plan->h.n_launches; ++li) {
        const int64_t n_items = ls[li].end - ls[li].first;
        if (n_items <= 0) continue;
        const unsigned wgs = (unsigned)std::min<int64_t>(resident, n_items);
        if (plan->h.period_block == 4)
            hipLaunchKernelGGL(batch_kernel<4>, dim3(wgs), dim3(kThreads), lds, s, a, (int32_t)li);
        else
            hipLaunchKernelGGL(batch_kernel<8>, dim3(wgs), dim3(kThreads), lds, s, a, (int32_t)li);
        if ((rc = check_launch("batch_search"))) return rc;
    }
    return CETRA_OK;
}
