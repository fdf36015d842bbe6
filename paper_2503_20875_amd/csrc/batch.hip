// Batched search: many light curves of uneven length searched by one
// persistent launch that drains a work queue (the per-curve method is Sec. 2.1
// setup, Sec. 2.2 linear search, Sec. 2.3 periodic search and best period,
// unchanged; batching is this library's addition).
//
// Plan (host).  Curves are ordered by descending fold cost (sum over periods
// of allowed durations times reference times), or by a seeded permutation.
// Each curve has four stages, cut into work items:
//   RES  resampling of 2048 grid points; also clears a share of the curve's
//        argmax keys, computes the same share of its periods' fold steps,
//        epoch counts and duration ranges (for the fold and decode items),
//        and checks a share of its times for order
//   LIN  linear search of 4 tiles of 256 W reference times of one duration
//   FOLD one fold unit: a block of B periods, one duration, one epoch chunk
//   EPI  decode of 256 periods' winners (FP64 recompute); the last EPI item of
//        a curve writes its best-period record and its done flag
// Consecutive curves in queue order form groups: a group closes once its
// fold has enough items (long curves are groups of one).  Dependencies and
// completion counts are per (group, stage), so a workgroup waits on, and
// acquires, one counter per group and stage rather than per curve.  The
// queue lists the items of group r in the order
//   RES(0) LIN(0) RES(1) LIN(1), then for r = 0, 1, ...:
//   FOLD(r) EPI(r-3) RES(r+2) LIN(r+2), and the last three EPI at the end,
// so the linear search of group r+2 and the decode of group r-3 run while
// group r folds.  Each curve's resampled light curve, fold-ready array and
// per-period table live in its own slot of slot set r mod S, S =
// min(8, groups); a set is sized for the largest group it serves.
//
// Dependencies.  An item may start only when the items it reads from are
// complete: LIN after every RES of its group, FOLD after every LIN of its
// group, EPI after every FOLD of its group, and RES after every EPI of the
// group that used the slot set before (group r-8).  Every such item sits
// earlier in the queue, and items are popped in queue order by workgroups
// that keep running until they finish them, so the earliest unfinished item
// never waits and the queue always drains.  The distances leave slack: a
// decode is queued three folds after its own fold, and the resampling that
// reuses a slot set three steps after that decode.
// Completion is counted per (group, stage): after a run of items the
// workgroup synchronises and one lane adds the run's count with release
// semantics at agent scope; a waiting workgroup's first wave polls the
// counter and acquires once it is complete (device-scope coherence across
// the XCDs' separate L2 caches), then the workgroup synchronises.  Every wait is bounded: a host-set cancel flag,
// another workgroup's abort, or a wall-clock limit ends it, and the limit
// marks the status so no result is trusted.
//
// Every item runs the same per-item device code as the single-curve entry
// points (stages.h), so each curve's records are bit-identical to separate
// single-curve calls whatever the queue order or the interleaving.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "common.h"
#include "stages.h"

namespace {

using cetra::dev::kThreads;

enum Stage : int32_t { kRes = 0, kLin = 1, kFold = 2, kEpi = 3, kStages = 4 };
constexpr int kResPoints = 2048;                 // grid points per RES item
constexpr int kLinTiles = 4;                     // 256-reference-time tiles per LIN item
constexpr int kEpiPeriods = kThreads;            // periods per EPI item
constexpr int kMaxSlots = 8;                     // groups of curves resident at once
constexpr int kLinAhead = 2;                     // RES/LIN of group r+2 are queued with FOLD(r)
constexpr int kEpiLag = 3;                       // EPI of group r-3 is queued with FOLD(r)
constexpr int kMaxGroup = 16;                    // curves per group at most
constexpr int64_t kGroupFoldItems = 49152;       // a group closes once its fold has this many items
constexpr int kLdsCapBytes = 40 * 1024;          // dynamic LDS of the persistent kernel
constexpr int64_t kFoldItemsTarget = 8192;       // fold items per curve to aim for (epoch chunks)
constexpr int32_t kPopMax = 64;                  // largest run of items one queue pop may take
constexpr int32_t kPopAuto = 8;                  // the automatic choice's largest run
constexpr uint64_t kMagic = 0x31484354414254ull; // tables image tag

struct Segment {
    int64_t first;  // first item index
    int32_t curve;
    int32_t stage;
};

struct CurveDesc {
    int64_t obs_off, n_obs, per_off, n_per;
    int64_t slot_off;                      // byte offset of the curve's slot in the arena
    int64_t ivar_off, fold_off, ptab_off;  // inside the slot: flux at 0, then ivar, the
                                           // fold-ready array, the per-period steps, epoch
                                           // counts and duration ranges
    int64_t n_items[kStages];
    int32_t group;                         // the curve's group (consecutive in queue order)
    int32_t n_res, n_lin_per_dur, n_pblk, n_chunks, n_tiles;
};

struct GroupDesc {
    int64_t n_items[kStages];  // items of the group's curves per stage (what a dependency waits for)
    int32_t prev_group;        // group that used the same slots before, whose decode must finish
                               // before this group resamples; -1 if none
    int32_t n_curves;
};

struct Header {
    uint64_t magic, plan_id;
    int64_t n_curves, n_groups, n_segments, n_items;
    int64_t off_curves, off_groups, off_grids, off_segments, tables_bytes;
    int32_t period_block, lds_bytes, lds_cap;
    int32_t linear_windows;  // W: reference times per lane of a LIN tile (256 W per tile)
    int32_t pop_items;       // items a workgroup takes per queue pop; 0 = chosen at launch
    int32_t reserved;
};

// Device status bits of cetra_batch_search.
constexpr int32_t kCancelled = CETRA_BATCH_CANCELLED;
constexpr int32_t kWaitLimit = CETRA_BATCH_WAIT_LIMIT;
constexpr int32_t kBadTables = CETRA_BATCH_BAD_TABLES;
constexpr int32_t kUnsorted = CETRA_BATCH_UNSORTED;

struct Counters {  // cleared by batch_init_kernel at every call
    unsigned long long head;
    uint32_t abort_flag;
    uint32_t pad;
};

struct BatchArgs {
    const char *tables;
    uint64_t plan_id;
    Counters *ctr;
    uint32_t *group_done;  // [n_groups][kStages]: finished items per group and stage
    uint32_t *curve_epi;   // [n_curves]: finished decode items per curve
    uint32_t *bad;         // [n_curves]
    uint64_t *best_keys;   // [n_curves]
    uint64_t *keys;        // [total periods]
    char *arena;
    const double *t;
    const float *f, *sigma, *model;
    const double *periods;
    const int32_t *jrange;  // nullable: [total periods][2] inclusive duration-index ranges
    const int32_t *cancel;  // nullable; polled at system scope
    float *lr, *depth, *depth_var;
    int32_t *epoch, *dur;
    cetra_best_record *best;
    int32_t *done;          // [n_curves]
    int32_t *status;
    int64_t n_curves, n_groups, n_items;
    uint64_t wait_ticks;    // wall-clock limit of one dependency wait
    int32_t resume;
    int32_t pop;            // items taken per queue pop (>= 1)
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Clears the counters, keys of the best periods, the status and (unless
// resuming) the done flags: a kernel rather than memsets, so the call can be
// captured in a graph.
__global__ void batch_init_kernel(BatchArgs a) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (tid == 0) {
        a.ctr->head = 0ull;
        a.ctr->abort_flag = 0u;
        a.status[0] = 0;
    }
    for (int64_t i = tid; i < a.n_groups * kStages; i += stride) a.group_done[i] = 0u;
    for (int64_t c = tid; c < a.n_curves; c += stride) {
        a.curve_epi[c] = 0u;
        a.bad[c] = 0u;
        a.best_keys[c] = 0ull;
        if (!a.resume) a.done[c] = 0;
    }
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ bool lane_zero() { return (threadIdx.x & 63) == 0; }

// Called by every lane of one wave: whether the host's cancel flag or another
// workgroup's abort stops the batch (the loaded flags are made wave-uniform,
// so every branch on the result is uniform).
__device__ __forceinline__ bool stop_requested(const BatchArgs &a) {
    if (a.cancel) {
        const int32_t c = __hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (__builtin_amdgcn_readfirstlane(c) != 0) {
            if (lane_zero()) atomicOr(a.status, kCancelled);
            return true;
        }
    }
    const uint32_t ab = __hip_atomic_load(&a.ctr->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(ab) != 0u;
}

// Called by every lane of one wave: wait until *counter >= need (acquire);
// false when the batch is being stopped or the wait exceeded its limit.  The
// loop's exit conditions are wave-uniform.  The counter is polled with
// relaxed loads and the acquire is one fence after the load that sees the
// count complete (an acquire load per poll would invalidate the XCD's L2 on
// every iteration of a spinning workgroup).
__device__ bool wait_for(const BatchArgs &a, const uint32_t *counter, uint32_t need) {
    if (need == 0) return true;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const uint32_t v = __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(v) >= need) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return true;
        }
        if (stop_requested(a)) return false;
        if (wall_clock64() - t0 > a.wait_ticks) {
            if (lane_zero()) {
                atomicOr(a.status, kWaitLimit);
                __hip_atomic_store(&a.ctr->abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

struct ItemRef {
    int32_t curve, stage;
    int64_t idx;
};

// Segment of an item: the last segment whose first item is <= item.  A
// workgroup pops items in increasing order, so the search starts from the
// segment of its previous item (`hint`, updated): usually the same one or a
// few later, which saves a chain of dependent loads per item.
__device__ ItemRef locate(const Header *h, const Segment *segs, int64_t item, int64_t &hint) {
    const int64_t last = h->n_segments - 1;
    int64_t lo = hint;
    if (lo < last && segs[lo + 1].first <= item) {
        int64_t hi = last;
        ++lo;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (segs[mid].first <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
    }
    lo = uniform64(lo);
    hint = lo;
    ItemRef r;
    r.curve = segs[lo].curve;
    r.stage = segs[lo].stage;
    r.idx = item - segs[lo].first;
    return r;
}

template <int B, int W>
__device__ void run_item(const BatchArgs &a, const Header *h, const CurveDesc &cd, const cetra_grid &g, int32_t c,
                         int32_t stage, int64_t idx, float *lds, int *s_bounds) {
    char *slot = a.arena + cd.slot_off;
    float *flux = reinterpret_cast<float *>(slot);
    float *ivar = reinterpret_cast<float *>(slot + cd.ivar_off);
    float2 *fold = reinterpret_cast<float2 *>(slot + cd.fold_off);
    cetra::dev::PeriodInfo *ptab = reinterpret_cast<cetra::dev::PeriodInfo *>(slot + cd.ptab_off);
    const int64_t I = g.n_t0;
    if (stage == kRes) {
        const int64_t q0 = idx * kResPoints;
        const int64_t q1 = min(q0 + kResPoints, g.n);
        for (int64_t q = q0 + threadIdx.x; q < q1; q += kThreads)
            cetra::dev::resample_point(a.t + cd.obs_off, a.f + cd.obs_off, a.sigma + cd.obs_off, cd.n_obs,
                                       g.t_first, g.cadence, g.n_pad, q, flux, ivar);
        // a share of the argmax keys, and of the order check of the times
        const int64_t nres = cd.n_res;
        const int64_t k0 = cd.n_per * idx / nres, k1 = cd.n_per * (idx + 1) / nres;
        for (int64_t k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const int64_t o = cd.per_off + k;
            a.keys[o] = 0ull;
            ptab[k] = cetra::dev::period_info(a.periods[o], g.t0_step, I, g.n_dur, g.durations,
                                              a.jrange ? a.jrange[2 * o] : 0,
                                              a.jrange ? a.jrange[2 * o + 1] : g.n_dur - 1);
        }
        const int64_t o0 = cd.n_obs * idx / nres, o1 = cd.n_obs * (idx + 1) / nres;
        const double *t = a.t + cd.obs_off;
        bool bad = false;
        for (int64_t n = o0 + threadIdx.x; n < o1; n += kThreads) {
            const double tn = t[n];
            if (!isfinite(tn) || (n > 0 && !(tn >= t[n - 1]))) bad = true;
        }
        if (bad) {
            atomicOr(&a.bad[c], 1u);
            atomicOr(a.status, kUnsorted);
        }
    } else if (stage == kLin) {
        // the tile loop and linear_tile's staged branch hold barriers: their
        // bounds and condition are made wave-uniform
        const int32_t per_dur = __builtin_amdgcn_readfirstlane(cd.n_lin_per_dur);
        const int32_t j = __builtin_amdgcn_readfirstlane((int32_t)(idx / per_dur));
        const int64_t tile0 = (idx % per_dur) * kLinTiles;
        cetra::dev::LinearParams p = cetra::dev::linear_params(g, j);
        const double span = cetra::dev::linear_span(g.t0_step, g.durations[j], g.cadence, W);
        const int64_t tab_bytes = (int64_t)cetra::dev::template_table_entries(g.n_model) * 8;
        const int64_t need = tab_bytes + (int64_t)ceil(span) * 8;
        p.span_cap = __builtin_amdgcn_readfirstlane(need <= h->lds_cap ? (int32_t)ceil(span) : 0);
        const int64_t tile1 = uniform64(min(tile0 + kLinTiles, (int64_t)cd.n_tiles));
        for (int64_t tile = tile0; tile < tile1; ++tile)
            cetra::dev::linear_tile<W>(p, tile * kThreads * W, flux, ivar, a.model, fold + (int64_t)j * I, nullptr,
                                       nullptr, nullptr, lds, s_bounds);
    } else if (stage == kFold) {
        const int64_t per_dur = (int64_t)cd.n_pblk * cd.n_chunks;
        const int32_t j = (int32_t)(idx / per_dur);
        const int64_t rest = idx % per_dur;
        const int64_t pb = rest % cd.n_pblk;
        const int32_t ch = (int32_t)(rest / cd.n_pblk);
        uint64_t R[B];
        int32_t ipb[B];
        int32_t ipmax = 0;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t k = pb * B + b;
            R[b] = 0;
            ipb[b] = 0;
            if (k < cd.n_per) {
                const cetra::dev::PeriodInfo pi = ptab[k];  // written by the curve's RES items
                if (j >= pi.jlo && j <= pi.jhi) {
                    R[b] = pi.step;
                    ipb[b] = pi.n_ep;
                }
            }
            ipmax = max(ipmax, ipb[b]);
        }
        if (ipmax == 0) return;
        const int32_t chunk = (ipmax + cd.n_chunks - 1) / cd.n_chunks;
        // the fold keeps its transit offsets and buffer resource in scalar
        // registers: every operand it takes must be wave-uniform
        const int32_t e_lo = __builtin_amdgcn_readfirstlane(ch * chunk);
        const int32_t e_hi = __builtin_amdgcn_readfirstlane(min(ipmax, ch * chunk + chunk));
        if (e_lo >= e_hi) return;
        const int32_t I32 = __builtin_amdgcn_readfirstlane((int32_t)I);
        const int32_t ju = __builtin_amdgcn_readfirstlane(j);
        const float2 *row = reinterpret_cast<const float2 *>(uniform64((int64_t)(fold + (int64_t)ju * I32)));
        uint64_t *keys = reinterpret_cast<uint64_t *>(uniform64((int64_t)(a.keys + cd.per_off + pb * B)));
        cetra::dev::fold_unit<B, true>(row, ju, I32, R, ipb, e_lo, e_hi, keys);
    } else {  // kEpi
        const int64_t k = idx * kEpiPeriods + threadIdx.x;
        uint64_t bk = 0;
        if (k < cd.n_per) {
            const int64_t o = cd.per_off + k;
            const cetra::dev::PeriodInfo pi = ptab[k];  // the step does not depend on the duration range
            const uint64_t key = __hip_atomic_load(&a.keys[o], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const float l = cetra::dev::fold_decode(fold, I, g.n_dur, pi.step, key, a.lr + o, a.epoch + o,
                                                    a.dur + o, a.depth + o, a.depth_var + o);
            if (a.epoch[o] >= 0) bk = ((uint64_t)__float_as_uint(l) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
        }
        bk = cetra::dev::wave_max_u64(bk);
        if ((threadIdx.x & 63) == 0 && bk != 0) atomicMax((unsigned long long *)&a.best_keys[c], bk);
    }
}

// Best-period record of curve c from its packed best key (the maximum LR,
// ties to the smallest period index, as cetra_best), and its done flag.
__device__ void finish_curve(const BatchArgs &a, const CurveDesc &cd, const cetra_grid &g, int32_t c) {
    const uint64_t bk = __hip_atomic_load(&a.best_keys[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    a.done[c] = __hip_atomic_load(&a.bad[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? -1 : 1;
}

// Called by every lane of one wave: adds n finished items of (curve c,
// stage) to the stage's counter of the curve's group; release orders the
// items' stores (and atomics) before the count.  Decode items also count per
// curve, with acquire and release: the call that completes a curve's decode
// writes its best-period record from the other items' records, before the
// group count.
__device__ void count_items(const BatchArgs &a, const CurveDesc *curves, const cetra_grid *grids, int32_t c,
                            int32_t stage, uint32_t n, int32_t skipped) {
    if (n == 0) return;
    const int32_t g = __builtin_amdgcn_readfirstlane(curves[c].group);
    if (stage == kEpi) {
        uint32_t prev = 0;
        if (lane_zero()) prev = __hip_atomic_fetch_add(&a.curve_epi[c], n, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        prev = __builtin_amdgcn_readfirstlane(prev);
        const uint32_t n_epi = __builtin_amdgcn_readfirstlane((uint32_t)curves[c].n_items[kEpi]);
        if (!skipped && prev + n == n_epi && lane_zero()) finish_curve(a, curves[c], grids[c], c);
    }
    if (lane_zero())
        (void)__hip_atomic_fetch_add(&a.group_done[(int64_t)g * kStages + stage], n, __ATOMIC_RELEASE,
                                     __HIP_MEMORY_SCOPE_AGENT);
}

template <int B, int W>
__global__ void __launch_bounds__(kThreads, 3) batch_kernel(BatchArgs a) {
    extern __shared__ float lds[];
    __shared__ int s_bounds[2];
    __shared__ long long s_item;
    __shared__ int s_go;
    const Header *h = reinterpret_cast<const Header *>(a.tables);
    if (h->magic != kMagic || h->plan_id != a.plan_id) {  // the workspace does not hold this plan's tables
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(a.status, kBadTables);
        return;
    }
    const CurveDesc *curves = reinterpret_cast<const CurveDesc *>(a.tables + h->off_curves);
    const GroupDesc *groups = reinterpret_cast<const GroupDesc *>(a.tables + h->off_groups);
    const cetra_grid *grids = reinterpret_cast<const cetra_grid *>(a.tables + h->off_grids);
    const Segment *segs = reinterpret_cast<const Segment *>(a.tables + h->off_segments);
    // The first wave takes items, waits on dependencies and counts
    // completions; a branch on the wave index is scalar, and every loop in
    // those regions exits on wave-uniform values, so the control flow around
    // the barriers below is uniform.  (A lane-0 region holding a loop between
    // barriers of this loop can be restructured by the compiler into an inner
    // loop that the wave's other lanes keep re-entering without lane 0: the
    // wave would then never leave it.)
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // the dependency this workgroup last saw complete: counters only grow and
    // the acquire that saw it already made its data visible here, so later
    // items with the same dependency skip the wait (and its cache
    // invalidation, which would otherwise evict the fold's working set from
    // L2 on every short item)
    const uint32_t *seen_counter = nullptr;
    int64_t seg_hint = 0;
    // One pop takes a run of a.pop consecutive items, [next, end): the queue
    // head and the per-stage counters are single words that every workgroup
    // updates, and one update per item saturates them when items are short.
    // Finished items of one (curve, stage) are counted together, before the
    // workgroup moves to another (curve, stage), waits on a dependency, or
    // pops again; so it never waits while holding uncounted items, and the
    // earliest unfinished item still never waits.
    int64_t next = 0, end = 0;
    int32_t pend_c = 0, pend_stage = 0, pend_skip = 0;
    uint32_t pend_n = 0;
    for (;;) {
        if (next >= end) {
            if (wave == 0) {
                count_items(a, curves, grids, pend_c, pend_stage, pend_n, pend_skip);
                long long it = -1;
                if (!stop_requested(a)) {
                    unsigned long long v = 0;
                    if (lane_zero()) v = atomicAdd(&a.ctr->head, (unsigned long long)a.pop);
                    v = (unsigned long long)uniform64((int64_t)v);
                    if (v < (unsigned long long)a.n_items) it = (long long)v;
                }
                if (lane_zero()) s_item = it;
            }
            pend_n = 0;
            __syncthreads();
            next = uniform64(s_item);
            if (next < 0) break;
            end = min(next + (int64_t)a.pop, a.n_items);
        }
        const int64_t item = next++;
        const ItemRef ir = locate(h, segs, item, seg_hint);
        const int32_t c = __builtin_amdgcn_readfirstlane(ir.curve);
        const int32_t stage = __builtin_amdgcn_readfirstlane(ir.stage);
        const int64_t idx = uniform64(ir.idx);
        const CurveDesc &cd = curves[c];
        const bool other_run = pend_n != 0 && (c != pend_c || stage != pend_stage);
        // dependency of the item: the previous stage of its curve's group,
        // or for RES the decode of the group that used its slots before
        if (wave == 0) {
            if (other_run) count_items(a, curves, grids, pend_c, pend_stage, pend_n, pend_skip);
            const int32_t g = __builtin_amdgcn_readfirstlane(cd.group);
            const uint32_t *counter = nullptr;
            uint32_t need = 0;
            if (stage == kRes) {
                const int32_t pg = __builtin_amdgcn_readfirstlane(groups[g].prev_group);
                if (pg >= 0) {
                    counter = &a.group_done[(int64_t)pg * kStages + kEpi];
                    need = __builtin_amdgcn_readfirstlane((uint32_t)groups[pg].n_items[kEpi]);
                }
            } else {
                counter = &a.group_done[(int64_t)g * kStages + stage - 1];
                need = __builtin_amdgcn_readfirstlane((uint32_t)groups[g].n_items[stage - 1]);
            }
            bool ok = true;
            if (counter && counter != seen_counter) {
                ok = wait_for(a, counter, need);
                if (ok) seen_counter = counter;
            }
            if (lane_zero()) s_go = ok ? 1 : 0;
        }
        if (other_run) pend_n = 0;
        __syncthreads();
        const int go = __builtin_amdgcn_readfirstlane(s_go);
        if (!go) break;
        const int skip = __builtin_amdgcn_readfirstlane(a.resume && a.done[c] != 0 ? 1 : 0);  // done earlier
        if (!skip) run_item<B, W>(a, h, cd, grids[c], c, stage, idx, lds, s_bounds);
        __syncthreads();  // every lane's stores of the item are complete before it is counted
        pend_c = c;
        pend_stage = stage;
        pend_skip = skip;
        ++pend_n;
    }
}

uint64_t next_plan_id() {
    static std::mutex mu;
    static uint64_t counter = 0x9E3779B97F4A7C15ull;
    std::lock_guard<std::mutex> lock(mu);
    counter += 0x9E3779B97F4A7C15ull;
    uint64_t z = counter;  // splitmix64 finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Device wall-clock ticks per second (cached per device).
double wall_clock_hz() {
    static std::mutex mu;
    static std::vector<double> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1.0e8;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0.0);
    if (cache[dev] == 0.0) {
        int khz = 0;
        cache[dev] = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0
                         ? 1.0e3 * khz
                         : 1.0e8;
    }
    return cache[dev];
}

}  // namespace

struct cetra_batch_plan {
    std::vector<char> tables;  // header, curves, grids, segments (the device image)
    Header h;
    std::vector<int32_t> order;
    int64_t n_curves, total_periods;
    size_t off_counters, off_group_done, off_curve_epi, off_bad, off_best_keys, off_keys, off_arena, arena_bytes;
    size_t workspace_bytes;
    int32_t n_slots;   // curves whose slots are live at once
    int32_t n_groups;
    int32_t *cancel_host;  // pinned flag of cetra_batch_cancel_flag, or NULL
};

using namespace cetra;

extern "C" int cetra_batch_plan_create(const cetra_batch_desc *d, cetra_batch_plan **out) {
    clear_error();
    CETRA_REQUIRE(d && out && d->grids && d->obs_offsets && d->period_offsets, "batch_plan: NULL pointer");
    CETRA_REQUIRE(d->n_curves >= 1, "batch_plan: n_curves must be >= 1");
    CETRA_REQUIRE(d->pop_items >= 0 && d->pop_items <= kPopMax, "batch_plan: pop_items must be 0-64");
    const int n = d->n_curves;
    const cetra_grid &g0 = d->grids[0];
    int rc;
    const cetra_tuning tu = current_tuning();
    const int B = d->fold_period_block ? d->fold_period_block : std::min(tu.fold_period_block, 8);
    CETRA_REQUIRE(B == 4 || B == 8, "batch_plan: fold_period_block must be 0, 4 or 8");
    // the persistent kernel's registers are the maximum over its stages: four
    // windows per lane would lift the linear stage above the fold's budget
    // (197 against 157 VGPRs, 2 waves per SIMD instead of 3); results do not
    // depend on W
    const int W = std::min(tu.linear_windows, 2);
    CETRA_REQUIRE(d->obs_offsets[0] == 0 && d->period_offsets[0] == 0, "batch_plan: offsets must start at 0");
    std::vector<CurveDesc> cds(n);
    std::vector<double> cost(n);
    const int64_t tab_bytes = (int64_t)dev::template_table_entries(g0.n_model) * 8;
    const int32_t lds_cap = (int32_t)std::max<int64_t>(kLdsCapBytes, tab_bytes);
    int32_t lds_bytes = (int32_t)tab_bytes;
    for (int c = 0; c < n; ++c) {
        if ((rc = check_grid(&d->grids[c]))) return rc;
        const cetra_grid &g = d->grids[c];
        CETRA_REQUIRE(g.n_dur == g0.n_dur && g.n_model == g0.n_model, "batch_plan: curves must share J and M");
        for (int j = 0; j < g.n_dur; ++j)
            CETRA_REQUIRE(g.durations[j] == g0.durations[j], "batch_plan: curves must share the durations");
        CETRA_REQUIRE(d->obs_offsets[c + 1] >= d->obs_offsets[c], "batch_plan: obs_offsets not ascending");
        CETRA_REQUIRE(d->period_offsets[c + 1] >= d->period_offsets[c], "batch_plan: period_offsets not ascending");
        if (g.n_t0 >= ((int64_t)1 << 28) || g.n >= INT32_MAX)
            return set_error(CETRA_ERR_RANGE, "batch_plan: curve %d: I must be < 2^28 and N < 2^31", c);
        CurveDesc &cd = cds[c];
        std::memset(&cd, 0, sizeof cd);
        cd.obs_off = d->obs_offsets[c];
        cd.n_obs = d->obs_offsets[c + 1] - d->obs_offsets[c];
        cd.per_off = d->period_offsets[c];
        cd.n_per = d->period_offsets[c + 1] - d->period_offsets[c];
        cd.n_tiles = (int32_t)ceil_div(g.n_t0, (int64_t)kThreads * W);
        cd.n_res = (int32_t)ceil_div(g.n, kResPoints);
        cd.n_lin_per_dur = (int32_t)ceil_div(cd.n_tiles, kLinTiles);
        cd.n_pblk = (int32_t)ceil_div(cd.n_per, B);
        const int64_t base = (int64_t)cd.n_pblk * g.n_dur;
        cd.n_chunks = base > 0 ? (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, ceil_div(kFoldItemsTarget, base)))
                               : 1;
        cd.n_items[kRes] = cd.n_res;
        cd.n_items[kLin] = (int64_t)g.n_dur * cd.n_lin_per_dur;
        cd.n_items[kFold] = base * cd.n_chunks;
        cd.n_items[kEpi] = std::max<int64_t>(1, ceil_div(cd.n_per, kEpiPeriods));
        for (int s = 0; s < kStages; ++s)
            if (cd.n_items[s] >= (int64_t)UINT32_MAX)
                return set_error(CETRA_ERR_RANGE, "batch_plan: curve %d has too many work items", c);
        cost[c] = (double)cd.n_per * g.n_dur * (double)g.n_t0;
        for (int j = 0; j < g.n_dur; ++j) {
            int32_t span_cap = 0;
            lds_bytes = std::max<int32_t>(lds_bytes, (int32_t)linear_lds_bytes(&g, j, W, lds_cap, &span_cap));
        }
    }
    // queue order
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    if (d->shuffle_seed != 0) {
        uint64_t s = (uint64_t)d->shuffle_seed;
        for (int i = n - 1; i > 0; --i) {  // Fisher-Yates with splitmix64 draws
            s += 0x9E3779B97F4A7C15ull;
            uint64_t z = s;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            std::swap(order[i], order[(int)(z % (uint64_t)(i + 1))]);
        }
    } else {
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    }
    // groups: consecutive curves in queue order, closed once their fold has
    // kGroupFoldItems items (long curves form groups of one); dependencies
    // and counters are per group, so a workgroup acquires once per group and
    // stage rather than per curve
    std::vector<int32_t> gfirst, gcount;
    {
        int64_t acc = 0;
        for (int p = 0; p < n; ++p) {
            if (gfirst.empty() || gcount.back() == kMaxGroup || acc >= kGroupFoldItems) {
                gfirst.push_back(p);
                gcount.push_back(0);
                acc = 0;
            }
            cds[order[p]].group = (int32_t)(gfirst.size() - 1);
            ++gcount.back();
            acc += cds[order[p]].n_items[kFold];
        }
    }
    const int n_groups = (int)gfirst.size();
    std::vector<GroupDesc> grp(n_groups);
    // slot sets: group gi uses set gi mod S, with one slot per curve sized
    // for that curve; a set holds the largest of the groups it serves
    const int n_sets = std::min(kMaxSlots, n_groups);
    std::vector<size_t> set_bytes(n_sets, 0), grp_bytes(n_groups, 0);
    for (int gi = 0; gi < n_groups; ++gi) {
        GroupDesc &gd = grp[gi];
        std::memset(&gd, 0, sizeof gd);
        gd.prev_group = gi >= n_sets ? gi - n_sets : -1;
        gd.n_curves = gcount[gi];
        size_t off_in_group = 0;
        for (int p = gfirst[gi]; p < gfirst[gi] + gcount[gi]; ++p) {
            CurveDesc &cd = cds[order[p]];
            const cetra_grid &g = d->grids[order[p]];
            cd.ivar_off = (int64_t)align256(4 * (size_t)g.n);
            cd.fold_off = cd.ivar_off + (int64_t)align256(4 * (size_t)g.n);
            cd.ptab_off = cd.fold_off + (int64_t)align256((size_t)8 * g.n_dur * (size_t)g.n_t0);
            cd.slot_off = (int64_t)off_in_group;  // relative to the set for now
            off_in_group += (size_t)cd.ptab_off + align256(sizeof(dev::PeriodInfo) * (size_t)std::max<int64_t>(cd.n_per, 1));
            for (int st = 0; st < kStages; ++st) gd.n_items[st] += cd.n_items[st];
        }
        for (int st = 0; st < kStages; ++st)
            if (gd.n_items[st] >= (int64_t)UINT32_MAX)
                return set_error(CETRA_ERR_RANGE, "batch_plan: group %d has too many work items", gi);
        grp_bytes[gi] = off_in_group;
        set_bytes[gi % n_sets] = std::max(set_bytes[gi % n_sets], off_in_group);
    }
    std::vector<size_t> set_off(n_sets, 0);
    size_t arena_bytes = 0;
    for (int si = 0; si < n_sets; ++si) {
        set_off[si] = arena_bytes;
        arena_bytes += set_bytes[si];
    }
    int32_t resident = 0;  // curves whose slots are live at once: the largest group of each set
    {
        std::vector<int32_t> set_max(n_sets, 0);
        for (int gi = 0; gi < n_groups; ++gi) set_max[gi % n_sets] = std::max(set_max[gi % n_sets], gcount[gi]);
        for (int si = 0; si < n_sets; ++si) resident += set_max[si];
    }
    for (int p = 0; p < n; ++p) {
        CurveDesc &cd = cds[order[p]];
        cd.slot_off += (int64_t)set_off[cd.group % n_sets];
    }
    // items in queue order
    std::vector<Segment> segs;
    int64_t item = 0;
    auto emit_group = [&](int gi, int st) {
        if (gi < 0 || gi >= n_groups) return;
        for (int p = gfirst[gi]; p < gfirst[gi] + gcount[gi]; ++p) {
            const int c = order[p];
            if (cds[c].n_items[st] == 0) continue;
            segs.push_back(Segment{item, c, st});
            item += cds[c].n_items[st];
        }
    };
    // slot reuse needs RES(group gi), queued at step gi - kLinAhead, after
    // EPI(group gi - S), queued at step gi - S + kEpiLag
    static_assert(kMaxSlots > kLinAhead + kEpiLag, "a slot's next user would be queued before its last");
    for (int gi = 0; gi < kLinAhead; ++gi) {
        emit_group(gi, kRes);
        emit_group(gi, kLin);
    }
    for (int r = 0; r < n_groups; ++r) {
        emit_group(r, kFold);
        emit_group(r - kEpiLag, kEpi);
        emit_group(r + kLinAhead, kRes);
        emit_group(r + kLinAhead, kLin);
    }
    for (int gi = std::max(0, n_groups - kEpiLag); gi < n_groups; ++gi) emit_group(gi, kEpi);

    auto *plan = new (std::nothrow) cetra_batch_plan;
    if (!plan) return set_error(CETRA_ERR_INVALID, "batch_plan: out of host memory");
    Header h;
    std::memset(&h, 0, sizeof h);
    h.magic = kMagic;
    h.plan_id = next_plan_id();
    h.n_curves = n;
    h.n_groups = n_groups;
    h.n_segments = (int64_t)segs.size();
    h.n_items = item;
    size_t off = align256(sizeof(Header));
    h.off_curves = (int64_t)off;
    off += align256(sizeof(CurveDesc) * n);
    h.off_groups = (int64_t)off;
    off += align256(sizeof(GroupDesc) * n_groups);
    h.off_grids = (int64_t)off;
    off += align256(sizeof(cetra_grid) * n);
    h.off_segments = (int64_t)off;
    off += align256(sizeof(Segment) * std::max<size_t>(segs.size(), 1));
    h.tables_bytes = (int64_t)off;
    h.period_block = B;
    h.linear_windows = W;
    h.pop_items = d->pop_items;
    h.lds_bytes = lds_bytes;
    h.lds_cap = lds_cap;
    plan->h = h;
    plan->tables.assign(off, 0);
    std::memcpy(plan->tables.data(), &h, sizeof h);
    std::memcpy(plan->tables.data() + h.off_curves, cds.data(), sizeof(CurveDesc) * n);
    std::memcpy(plan->tables.data() + h.off_groups, grp.data(), sizeof(GroupDesc) * n_groups);
    std::memcpy(plan->tables.data() + h.off_grids, d->grids, sizeof(cetra_grid) * n);
    if (!segs.empty()) std::memcpy(plan->tables.data() + h.off_segments, segs.data(), sizeof(Segment) * segs.size());
    plan->order = order;
    plan->n_curves = n;
    plan->n_groups = n_groups;
    plan->total_periods = d->period_offsets[n];
    // workspace: tables | counters | group stage counters | curve decode
    // counters | bad flags | best keys | keys | slots
    size_t w = off;
    plan->off_counters = w;
    w += align256(sizeof(Counters));
    plan->off_group_done = w;
    w += align256(sizeof(uint32_t) * kStages * (size_t)n_groups);
    plan->off_curve_epi = w;
    w += align256(sizeof(uint32_t) * (size_t)n);
    plan->off_bad = w;
    w += align256(sizeof(uint32_t) * (size_t)n);
    plan->off_best_keys = w;
    w += align256(sizeof(uint64_t) * (size_t)n);
    plan->off_keys = w;
    w += align256(sizeof(uint64_t) * (size_t)std::max<int64_t>(plan->total_periods, 1));
    plan->off_arena = w;
    w += arena_bytes;
    plan->arena_bytes = arena_bytes;
    plan->workspace_bytes = w;
    plan->n_slots = resident;
    plan->cancel_host = nullptr;
    *out = plan;
    return CETRA_OK;
}

extern "C" int cetra_batch_plan_destroy(cetra_batch_plan *plan) {
    clear_error();
    if (plan && plan->cancel_host) (void)hipHostFree(plan->cancel_host);
    delete plan;
    return CETRA_OK;
}

extern "C" int cetra_batch_plan_info(const cetra_batch_plan *plan, cetra_batch_info *info) {
    clear_error();
    CETRA_REQUIRE(plan && info, "batch_plan_info: NULL pointer");
    std::memset(info, 0, sizeof *info);
    info->workspace_bytes = plan->workspace_bytes;
    info->tables_bytes = (size_t)plan->h.tables_bytes;
    info->n_curves = plan->n_curves;
    info->total_periods = plan->total_periods;
    info->n_launches = 2;
    info->n_items = plan->h.n_items;
    info->n_slots = plan->n_slots;
    info->period_block = plan->h.period_block;
    info->lds_bytes = plan->h.lds_bytes;
    return CETRA_OK;
}

extern "C" int cetra_batch_workspace(const cetra_batch_plan *plan, size_t *bytes, size_t *tables_bytes) {
    clear_error();
    CETRA_REQUIRE(plan && bytes, "batch_workspace: NULL pointer");
    *bytes = plan->workspace_bytes;
    if (tables_bytes) *tables_bytes = (size_t)plan->h.tables_bytes;
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

extern "C" int cetra_batch_plan_order(const cetra_batch_plan *plan, int32_t *order, int32_t n) {
    clear_error();
    CETRA_REQUIRE(plan && order, "batch_plan_order: NULL pointer");
    CETRA_REQUIRE(n == (int32_t)plan->order.size(), "batch_plan_order: n must equal the number of curves");
    std::copy(plan->order.begin(), plan->order.end(), order);
    return CETRA_OK;
}

extern "C" int cetra_batch_cancel_flag(cetra_batch_plan *plan, int32_t **flag) {
    clear_error();
    CETRA_REQUIRE(plan && flag, "batch_cancel_flag: NULL pointer");
    if (!plan->cancel_host) {
        void *p = nullptr;
        const hipError_t e = hipHostMalloc(&p, sizeof(int32_t), hipHostMallocCoherent);
        if (e != hipSuccess || !p)
            return set_error(CETRA_ERR_HIP, "batch_cancel_flag: hipHostMalloc: %s", hipGetErrorString(e));
        plan->cancel_host = static_cast<int32_t *>(p);
        *plan->cancel_host = 0;
    }
    *flag = plan->cancel_host;
    return CETRA_OK;
}

extern "C" int cetra_batch_search(const cetra_batch_plan *plan, void *stream, const double *t, const float *f,
                                  const float *sigma, const float *model, const double *periods,
                                  const int32_t *jrange, const int32_t *cancel, int32_t flags, void *work, size_t work_bytes, float *lr,
                                  int32_t *epoch, int32_t *dur, float *depth, float *depth_var,
                                  cetra_best_record *best, int32_t *done, int32_t *status) {
    clear_error();
    CETRA_REQUIRE(plan, "batch_search: NULL plan");
    CETRA_REQUIRE(model && work && best && done && status, "batch_search: NULL pointer");
    CETRA_REQUIRE((flags & ~CETRA_BATCH_RESUME) == 0, "batch_search: unknown flags");
    CETRA_REQUIRE(t && f && sigma, "batch_search: NULL observations");
    CETRA_REQUIRE(plan->total_periods == 0 || (periods && lr && epoch && dur && depth && depth_var),
                  "batch_search: NULL period pointer");
    if (work_bytes < plan->workspace_bytes)
        return set_error(CETRA_ERR_WORKSPACE, "batch_search: workspace needs %zu bytes", plan->workspace_bytes);
    char *w = static_cast<char *>(work);
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.tables = w;
    a.plan_id = plan->h.plan_id;
    a.ctr = reinterpret_cast<Counters *>(w + plan->off_counters);
    a.group_done = reinterpret_cast<uint32_t *>(w + plan->off_group_done);
    a.curve_epi = reinterpret_cast<uint32_t *>(w + plan->off_curve_epi);
    a.bad = reinterpret_cast<uint32_t *>(w + plan->off_bad);
    a.best_keys = reinterpret_cast<uint64_t *>(w + plan->off_best_keys);
    a.keys = reinterpret_cast<uint64_t *>(w + plan->off_keys);
    a.arena = w + plan->off_arena;
    a.t = t;
    a.f = f;
    a.sigma = sigma;
    a.model = model;
    a.periods = periods;
    a.jrange = jrange;
    a.cancel = cancel ? cancel : plan->cancel_host;
    a.lr = lr;
    a.depth = depth;
    a.depth_var = depth_var;
    a.epoch = epoch;
    a.dur = dur;
    a.best = best;
    a.done = done;
    a.status = status;
    a.n_curves = plan->n_curves;
    a.n_groups = plan->n_groups;
    a.n_items = plan->h.n_items;
    a.resume = (flags & CETRA_BATCH_RESUME) ? 1 : 0;
    a.wait_ticks = (uint64_t)(wall_clock_hz() * 30.0);  // 30 s: far beyond any item's run time
    hipStream_t s = as_stream(stream);
    const unsigned init_blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(plan->n_curves * kStages, 256)));
    hipLaunchKernelGGL(batch_init_kernel, dim3(init_blocks), dim3(256), 0, s, a);
    int rc = check_launch("batch_search/init");
    if (rc) return rc;
    const int W = plan->h.linear_windows;
    const void *kern = plan->h.period_block == 4
                           ? (W == 1 ? (const void *)batch_kernel<4, 1> : W == 2 ? (const void *)batch_kernel<4, 2>
                                                                                 : (const void *)batch_kernel<4, 4>)
                           : (W == 1 ? (const void *)batch_kernel<8, 1> : W == 2 ? (const void *)batch_kernel<8, 2>
                                                                                 : (const void *)batch_kernel<8, 4>);
    const size_t lds = (size_t)plan->h.lds_bytes;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kThreads, lds) != hipSuccess || occ <= 0) occ = 1;
    const int per_cu = std::max(1, std::min(current_tuning().fold_wgs_per_cu, occ));
    const int64_t wgs = std::min<int64_t>((int64_t)device_cu_count() * per_cu, std::max<int64_t>(plan->h.n_items, 1));
    // runs of items per pop: up to kPopAuto, while every workgroup still
    // takes at least 32 runs (a lone curve keeps every workgroup busy)
    a.pop = plan->h.pop_items > 0
                ? plan->h.pop_items
                : (int32_t)std::max<int64_t>(1, std::min<int64_t>(kPopAuto, plan->h.n_items / (wgs * 32)));
    void *args[] = {(void *)&a};
    const hipError_t le = hipLaunchKernel(kern, dim3((unsigned)wgs), dim3(kThreads), args, lds, s);
    if (le != hipSuccess) return set_error(CETRA_ERR_HIP, "batch_search: %s", hipGetErrorString(le));
    return CETRA_OK;
}
