// Per-item device code of the search stages, shared by the single-curve
// kernels and the batched persistent kernel (so both produce bit-identical
// results).  Internal header.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#include "cetra.h"

namespace cetra {
namespace dev {

constexpr int kThreads = 256;          // lanes per workgroup in every stage
constexpr int kFoldChunk = 32;         // FP32 partial-sum length of the fold
constexpr int kFoldWaveEpochs = 128;   // epochs per wave in the fold
constexpr int kFoldTileEpochs = kFoldWaveEpochs * (kThreads / 64);

// ------------------------------------------------------------- resampling
// Nearest grid point of an observation, round half up (Sec. 2.1.1), FP64.
__device__ __forceinline__ int64_t obs_bin(double t, double t_first, double c, int64_t n_pad) {
    return n_pad + (int64_t)floor((t - t_first) / c + 0.5);
}

// Grid point q: inverse-variance weighted mean of the (time-sorted)
// observations whose nearest grid point it is, in input order, FP64.
__device__ __forceinline__ void resample_point(const double *__restrict__ t, const float *__restrict__ f,
                                               const float *__restrict__ sigma, int64_t n_obs, double t_first,
                                               double c, int64_t n_pad, int64_t q, float *__restrict__ flux,
                                               float *__restrict__ ivar) {
    int64_t lo = 0, hi = n_obs;
    while (lo < hi) {  // first observation whose bin is >= q
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (obs_bin(t[mid], t_first, c, n_pad) < q)
            lo = mid + 1;
        else
            hi = mid;
    }
    double wsum = 0.0, fsum = 0.0;
    for (int64_t n = lo; n < n_obs && obs_bin(t[n], t_first, c, n_pad) == q; ++n) {
        const double fn = (double)f[n];
        const double sn = (double)sigma[n];
        if (!isfinite(fn) || !isfinite(sn) || !(sn > 0.0)) continue;
        const double w = 1.0 / (sn * sn);
        wsum += w;
        fsum += w * fn;
    }
    if (wsum > 0.0) {
        flux[q] = (float)(fsum / wsum);
        ivar[q] = (float)wsum;
    } else {
        flux[q] = 0.0f;
        ivar[q] = 0.0f;
    }
}

// ----------------------------------------------------------- linear search
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

// Points covered by the 256 W consecutive windows of one duration that a
// workgroup computes (W windows per lane), with a margin of three for
// rounding: ((256 W - 1) dt + D)/c + 1 at most.
__host__ __device__ inline double linear_span(double t0_step, double duration, double cadence, int W) {
    return ((double)(kThreads * W - 1) * t0_step + duration) / cadence + 4.0;
}

// Template table entries in LDS: m_k for k < M, then copies of the last
// sample (rounded up to an even count, so the data pairs after it stay 8-byte
// aligned).  The nearest-sample index of a point inside its window never
// exceeds M (the last point lies at most D after the window start), so the
// copies stand in for the clamp to M - 1 of Sec. 2.1.2's table lookup.
constexpr int kTemplatePad = 4;
__host__ __device__ inline int template_table_entries(int n_model) { return (n_model + kTemplatePad + 1) & ~1; }

__host__ __device__ inline LinearParams linear_params(const cetra_grid &g, int j) {
    LinearParams p;
    p.cadence = g.cadence;
    p.t0_step = g.t0_step;
    p.duration = g.durations[j];
    p.t_end = (double)(g.n - 1) * g.cadence;
    p.n_t0 = g.n_t0;
    p.step_fx = g.dur_step_fx[j];
    p.n_model = g.n_model;
    p.span_cap = 0;
    return p;
}

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
    const long long ph =
        llround(4294967296.0 * ((((double)w.lo * p.cadence - ts) / p.duration) * (double)p.n_model));
    w.phase = ph < 0 ? 0ull : (uint64_t)ph;
    return w;
}

// FP32 partial sums are taken over aligned blocks of 32 grid points
// (n >> 5) and folded into FP64 block by block, so a window's sums do not
// depend on how many windows a lane computes or where they start.
constexpr int kLinearBlockShift = 5;

// One point of one window: template sample of 32.32 phase ph (integer part
// <= M), (w f, w) of the point.
__device__ __forceinline__ void linear_point(const float *__restrict__ tab, uint64_t &ph, uint64_t step, float2 d,
                                             float &sfm, float &smm) {
    const float mk = tab[(uint32_t)(ph >> 32)];
    sfm = fmaf(d.x, mk, sfm);
    smm = fmaf(d.y * mk, mk, smm);
    ph += step;
}

template <bool kStaged>
__device__ __forceinline__ float2 linear_data(const float2 *__restrict__ s_data, int64_t base,
                                              const float *__restrict__ flux, const float *__restrict__ ivar,
                                              int64_t n) {
    if (kStaged) return s_data[n - base];
    const float wq = ivar[n];
    return make_float2(flux[n] * wq, wq);
}

// The W windows of one lane, all non-null: one pass over the union of their
// points [lo[0], hi[W-1]] in aligned 32-point blocks.  Points inside every
// window ([lo[W-1], hi[0]]) read (w f, w) once for all W windows; the few
// points near the ends test each window's range.
template <int W, bool kStaged>
__device__ __forceinline__ void linear_lane(const float *__restrict__ tab, const float2 *__restrict__ s_data,
                                            int64_t base, const float *__restrict__ flux,
                                            const float *__restrict__ ivar, uint64_t step, const int64_t (&lo)[W],
                                            const int64_t (&hi)[W], uint64_t (&ph)[W], double (&dfm)[W],
                                            double (&dmm)[W]) {
    constexpr int kUnroll = W >= 4 ? 2 : 4;  // keeps four windows per lane within 128 VGPRs
    float sfm[W], smm[W];
#pragma unroll
    for (int w = 0; w < W; ++w) sfm[w] = smm[w] = 0.0f;
    const int64_t n0 = lo[0], n1 = hi[W - 1];
    const int64_t na = lo[W - 1], nb = hi[0];  // [na, nb]: in every window (empty if na > nb)
    for (int64_t b = n0 >> kLinearBlockShift; b <= (n1 >> kLinearBlockShift); ++b) {
        const int64_t s0 = max(n0, b << kLinearBlockShift);
        const int64_t s1 = min(n1, (b << kLinearBlockShift) + (1 << kLinearBlockShift) - 1);
        const int64_t m0 = max(s0, na), m1 = min(s1, nb);
        if (m0 <= m1) {
            for (int64_t n = s0; n < m0; ++n) {  // ramp-in: windows still to start
                const float2 d = linear_data<kStaged>(s_data, base, flux, ivar, n);
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (n >= lo[w] && n <= hi[w]) linear_point(tab, ph[w], step, d, sfm[w], smm[w]);
            }
#pragma unroll kUnroll
            for (int64_t n = m0; n <= m1; ++n) {  // every window
                const float2 d = linear_data<kStaged>(s_data, base, flux, ivar, n);
#pragma unroll
                for (int w = 0; w < W; ++w) linear_point(tab, ph[w], step, d, sfm[w], smm[w]);
            }
            for (int64_t n = m1 + 1; n <= s1; ++n) {  // ramp-out: windows already ended
                const float2 d = linear_data<kStaged>(s_data, base, flux, ivar, n);
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (n >= lo[w] && n <= hi[w]) linear_point(tab, ph[w], step, d, sfm[w], smm[w]);
            }
        } else {
            for (int64_t n = s0; n <= s1; ++n) {
                const float2 d = linear_data<kStaged>(s_data, base, flux, ivar, n);
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (n >= lo[w] && n <= hi[w]) linear_point(tab, ph[w], step, d, sfm[w], smm[w]);
            }
        }
        // fold the block into FP64 for the windows it intersects
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (b >= (lo[w] >> kLinearBlockShift) && b <= (hi[w] >> kLinearBlockShift)) {
                dfm[w] += (double)sfm[w];
                dmm[w] += (double)smm[w];
            }
            sfm[w] = smm[w] = 0.0f;
        }
    }
}

// One workgroup computes reference times i0 .. i0 + 256 W - 1 of one
// duration, W adjacent ones per lane.  The template table and, if
// p.span_cap > 0, the light-curve span of the workgroup's windows as (w f, w)
// pairs are staged in LDS.  Template indices advance in 32.32 fixed point;
// per window S_fm = sum w f m and S_mm = sum w m^2 are FP32 over aligned
// 32-point blocks folded into FP64.  A lane whose W windows are all non-null
// walks their union once; a lane with a null window walks each non-null
// window alone (same blocks, same sums).  Must be called by all lanes of the
// workgroup (it synchronises).
template <int W>
__device__ __forceinline__ void linear_tile(const LinearParams &p, int64_t i0, const float *__restrict__ flux,
                                            const float *__restrict__ ivar, const float *__restrict__ model,
                                            float2 *__restrict__ fold_row, float *__restrict__ depth_row,
                                            float *__restrict__ var_row, float *__restrict__ lr_row, float *lds,
                                            int *s_bounds) {
    const int n_tab = template_table_entries(p.n_model);
    float *s_tab = lds;                                              // [n_tab]
    float2 *s_data = reinterpret_cast<float2 *>(lds + n_tab);        // [span_cap]
    const bool staged = p.span_cap > 0;

    const int64_t ib = i0 + (int64_t)threadIdx.x * W;
    int64_t lo[W], hi[W];
    uint64_t ph[W];
    bool ok[W];
    bool all_ok = true, any_ok = false;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const bool in_range = ib + w < p.n_t0;
        const Window win = make_window(p, in_range ? ib + w : 0);
        ok[w] = win.ok && in_range;
        lo[w] = win.lo;
        hi[w] = win.hi;
        ph[w] = win.phase;
        all_ok = all_ok && ok[w];
        any_ok = any_ok || ok[w];
    }

    for (int k = threadIdx.x; k < n_tab; k += kThreads) s_tab[k] = model[min(k, p.n_model - 1)];
    int64_t base = 0;
    if (staged) {
        if (threadIdx.x == 0) {
            s_bounds[0] = INT_MAX;
            s_bounds[1] = -1;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (ok[w]) {
                atomicMin(&s_bounds[0], (int)lo[w]);
                atomicMax(&s_bounds[1], (int)hi[w]);
            }
        }
        __syncthreads();
        base = s_bounds[0];
        const int64_t count = min((int64_t)s_bounds[1] - (int64_t)s_bounds[0] + 1, (int64_t)p.span_cap);
        for (int64_t q = threadIdx.x; q < count; q += kThreads) {
            const float wq = ivar[base + q];
            s_data[q] = make_float2(flux[base + q] * wq, wq);
        }
    }
    __syncthreads();

    double dfm[W], dmm[W];
#pragma unroll
    for (int w = 0; w < W; ++w) dfm[w] = dmm[w] = 0.0;
    if (all_ok) {
        if (staged)
            linear_lane<W, true>(s_tab, s_data, base, flux, ivar, p.step_fx, lo, hi, ph, dfm, dmm);
        else
            linear_lane<W, false>(s_tab, s_data, base, flux, ivar, p.step_fx, lo, hi, ph, dfm, dmm);
    } else if (any_ok) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (!ok[w]) continue;
            const int64_t l1[1] = {lo[w]}, h1[1] = {hi[w]};
            uint64_t p1[1] = {ph[w]};
            double f1[1] = {0.0}, m1[1] = {0.0};
            if (staged)
                linear_lane<1, true>(s_tab, s_data, base, flux, ivar, p.step_fx, l1, h1, p1, f1, m1);
            else
                linear_lane<1, false>(s_tab, s_data, base, flux, ivar, p.step_fx, l1, h1, p1, f1, m1);
            dfm[w] = f1[0];
            dmm[w] = m1[0];
        }
    }
    __syncthreads();  // LDS may be reused by the caller's next item
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int64_t i = ib + w;
        if (i >= p.n_t0) continue;
        if (ok[w] && dmm[w] > 0.0) {
            fold_row[i] = make_float2((float)dfm[w], (float)dmm[w]);
            if (depth_row) depth_row[i] = (float)(dfm[w] / dmm[w]);
            if (var_row) var_row[i] = (float)(1.0 / dmm[w]);
            if (lr_row) lr_row[i] = (float)(0.5 * dfm[w] * dfm[w] / dmm[w]);
        } else {
            fold_row[i] = make_float2(0.0f, 0.0f);
            if (depth_row) depth_row[i] = __builtin_nanf("");
            if (var_row) var_row[i] = __builtin_inff();
            if (lr_row) lr_row[i] = 0.0f;
        }
    }
}

// ---------------------------------------------------------- periodic search
struct PeriodInfo {
    uint64_t step;   // R = llround(2^32 P/dt); 0 = period not evaluated
    int32_t n_ep;    // I_P = min(I, ceil(R / 2^32))
    int32_t jlo, jhi;
};

// Fixed-point step, epoch count and allowed duration range of a period:
// D_j < P (Sec. 2.3) intersected with [jlo_cap, jhi_cap].  A period shorter
// than the reference-time step (or not finite) is not evaluated, so transit
// offsets advance by >= 1 per transit, which bounds every fold loop.  A
// period of I or more steps has one transit per epoch inside the grid; its
// step is taken as I * 2^32 (the same transits), which keeps R in 64 bits.
__device__ __forceinline__ PeriodInfo period_info(double P, double t0_step, int64_t n_t0, int32_t n_dur,
                                                  const double *durations, int32_t jlo_cap, int32_t jhi_cap) {
    PeriodInfo pi;
    pi.step = 0;
    pi.n_ep = 0;
    pi.jlo = 0;
    pi.jhi = -1;
    if (!isfinite(P) || !(P >= t0_step)) return pi;
    const double x = P / t0_step;
    const uint64_t R = x >= (double)n_t0 ? (uint64_t)n_t0 << 32 : (uint64_t)llround(4294967296.0 * x);
    int64_t ip = (int64_t)((R + 4294967295ull) >> 32);
    if (ip > n_t0) ip = n_t0;
    int lo = max(0, jlo_cap), hi = min(n_dur - 1, jhi_cap);
    while (hi >= lo && !(durations[hi] < P)) --hi;
    pi.step = R;
    pi.n_ep = (int32_t)ip;
    pi.jlo = lo;
    pi.jhi = hi;
    return pi;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, off, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off, 64);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o > v ? o : v;
    }
    return v;
}

// Raw buffer resource over one row: loads at byte offsets >= the row size
// return zero (hardware range check), so the transit loop needs no per-lane
// bounds test and every load can be issued unconditionally.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_resource(const float2 *row, int32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2 *>(row), (short)0, n * 8, 0x00020000);
}

// One float pair at a byte offset (two dword loads; the compiler merges them
// into one 8-byte load, which never straddles the row end because elements
// and the row size are multiples of 8 bytes).
__device__ __forceinline__ float2 load_pair(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, int imm) {
    const float x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off + imm, 0, 0));
    const float y = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off + imm + 4, 0, 0));
    return make_float2(x, y);
}

// Argmax key of a candidate: LR >= 0 makes its FP32 bits monotone; ties go to
// the smallest flat index j I + i.
__device__ __forceinline__ uint64_t fold_key(float lr, uint32_t flat) {
    return ((uint64_t)__float_as_uint(lr) << 32) | (uint64_t)(0xFFFFFFFFu - flat);
}

// 16 bytes (two float pairs) at a byte offset: four dword loads that the
// compiler merges into one 16-byte load.
__device__ __forceinline__ float4 load_quad(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    const float x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
    const float y = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off + 4, 0, 0));
    const float z = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off + 8, 0, 0));
    const float w = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off + 12, 0, 0));
    return make_float4(x, y, z, w);
}

// Ranking value of a fold candidate, LR = A^2 / (2 S), with the hardware
// reciprocal (error of a few FP32 units, below that of the FP32 transit sums
// it is computed from); the winner's LR is recomputed in FP64 afterwards.
__device__ __forceinline__ float fold_rank_lr(float A, float S) {
    return 0.5f * A * (A * __builtin_amdgcn_rcpf(S));
}

// (hi:lo) += (rh:rl) on the scalar unit: one add and one add-with-carry
// (the compiler's own lowering of a wave-uniform 64-bit add whose high word
// is then clamped takes five scalar instructions).
__device__ __forceinline__ void acc_add(uint32_t &lo, uint32_t &hi, uint32_t rl, uint32_t rh) {
    asm("s_add_u32 %0, %0, %2\n\ts_addc_u32 %1, %1, %3" : "+s"(lo), "+s"(hi) : "s"(rl), "s"(rh) : "scc");
}

// One fold unit: B periods (R[b], ipb[b]; ipb = 0 means "skip"), duration row
// `row` (index j), epochs [e_lo, e_hi).  Each wave owns 128 consecutive
// epochs.  kPair = false: lane l takes epochs e_wave + l and e_wave + 64 + l
// (two 8-byte loads per period and step, each wave load 512 contiguous
// bytes); kPair = true: lane l takes the adjacent epochs e_wave + 2l and
// e_wave + 2l + 1 (one 16-byte load, the wave load 1 KB contiguous: half the
// load instructions).  Per transit step and period: four FP32 adds, one
// address add, and three scalar instructions that advance the 32.32
// fixed-point transit offset (its integer part saturates at I, where loads
// read zero).  Offsets and the loop exit are wave-uniform.  The transit
// offset round(m R / 2^32) does not decrease as R grows, so the evaluated
// period with the smallest step is the last to leave the row: its offset
// alone ends the loop.  FP32 chunks of 32 transits fold into FP32 totals
// (error below (31 + n/32) u of the absolute sum); the sums only rank
// candidates -- the epilogue recomputes the winner in FP64.  The per-period
// maxima go to keys[b] by 64-bit atomicMax.
template <int B, bool kPair = false>
__device__ __forceinline__ void fold_unit(const float2 *row, int32_t j, int32_t I, const uint64_t (&R)[B],
                                          const int32_t (&ipb)[B], int32_t e_lo, int32_t e_hi, uint64_t *keys) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const __amdgpu_buffer_rsrc_t rsrc = row_resource(row, I);
    const uint32_t uI = (uint32_t)I;
    // steps split into integer and fraction words (wave-uniform: kept in
    // scalar registers, so the offset updates run on the scalar unit); the
    // slowest period
    uint32_t Rh[B], Rl[B];
    uint64_t r_min = ~0ull;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        Rh[b] = __builtin_amdgcn_readfirstlane((uint32_t)(R[b] >> 32));
        Rl[b] = __builtin_amdgcn_readfirstlane((uint32_t)R[b]);
        r_min = ipb[b] > 0 && R[b] < r_min ? R[b] : r_min;
    }
    if (r_min == ~0ull) return;  // no period of the block is evaluated on this row
    const uint32_t Rh_min = __builtin_amdgcn_readfirstlane((uint32_t)(r_min >> 32));
    const uint32_t Rl_min = __builtin_amdgcn_readfirstlane((uint32_t)r_min);
    uint64_t best[B];
#pragma unroll
    for (int b = 0; b < B; ++b) best[b] = 0;

    for (int32_t e0 = e_lo; e0 < e_hi; e0 += kFoldTileEpochs) {
        const int32_t e_wave = e0 + wave * kFoldWaveEpochs;  // wave-uniform
        if (e_wave >= e_hi) break;
        const int32_t e = e_wave + (kPair ? 2 * lane : lane);  // epochs e and e + kStride
        constexpr int32_t kStride = kPair ? 1 : 64;
        const uint32_t e_bytes = (uint32_t)e * 8u;
        // a transit at offset o is inside the row for some lane iff o < lim
        const uint32_t lim = uI - (uint32_t)e_wave;
        float a0[B], s0[B], a1[B], s1[B], ta0[B], ts0[B], ta1[B], ts1[B];
        uint32_t hi[B], lo[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            a0[b] = s0[b] = a1[b] = s1[b] = 0.0f;
            ta0[b] = ts0[b] = ta1[b] = ts1[b] = 0.0f;
            hi[b] = 0;
            lo[b] = 0x80000000u;  // + 1/2: round half up
        }
        uint32_t h_min = 0, l_min = 0x80000000u;
        {
            // transit 0 sits at offset 0 for every period (and lim > 0):
            // one load serves the whole block
            float2 v0, v1;
            if (kPair) {
                const float4 v = load_quad(rsrc, e_bytes);
                v0 = make_float2(v.x, v.y);
                v1 = make_float2(v.z, v.w);
            } else {
                v0 = load_pair(rsrc, e_bytes, 0);
                v1 = load_pair(rsrc, e_bytes, 64 * 8);
            }
#pragma unroll
            for (int b = 0; b < B; ++b) {
                acc_add(lo[b], hi[b], Rl[b], Rh[b]);
                hi[b] = min(hi[b], uI);
            }
            acc_add(l_min, h_min, Rl_min, Rh_min);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                a0[b] += v0.x;
                s0[b] += v0.y;
                a1[b] += v1.x;
                s1[b] += v1.y;
            }
        }
        int mm0 = 1;  // the first chunk already holds transit 0
        while (h_min < lim) {
            for (int mm = mm0; mm < kFoldChunk && h_min < lim; ++mm) {
                // all 2B loads of the step are issued before the first add
                // consumes one, so a wave keeps 2B loads in flight
                float2 v0[B], v1[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const uint32_t off = e_bytes + hi[b] * 8u;
                    if (kPair) {
                        const float4 v = load_quad(rsrc, off);
                        v0[b] = make_float2(v.x, v.y);
                        v1[b] = make_float2(v.z, v.w);
                    } else {
                        v0[b] = load_pair(rsrc, off, 0);
                        v1[b] = load_pair(rsrc, off, 64 * 8);
                    }
                }
                // next offsets: hi < 2^31 and Rh < 2^31, so no sum wraps
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    acc_add(lo[b], hi[b], Rl[b], Rh[b]);
                    hi[b] = min(hi[b], uI);
                }
                acc_add(l_min, h_min, Rl_min, Rh_min);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    a0[b] += v0[b].x;
                    s0[b] += v0[b].y;
                    a1[b] += v1[b].x;
                    s1[b] += v1[b].y;
                }
            }
            mm0 = 0;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                ta0[b] += a0[b];
                ts0[b] += s0[b];
                ta1[b] += a1[b];
                ts1[b] += s1[b];
                a0[b] = s0[b] = a1[b] = s1[b] = 0.0f;
            }
        }
        if (mm0) {  // a single transit: its sums are still in the chunk partials
#pragma unroll
            for (int b = 0; b < B; ++b) {
                ta0[b] += a0[b];
                ts0[b] += s0[b];
                ta1[b] += a1[b];
                ts1[b] += s1[b];
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int32_t eh = e + kStride * h;
                const float A = h ? ta1[b] : ta0[b];
                const float S = h ? ts1[b] : ts0[b];
                const bool ok = eh < ipb[b] && eh < e_hi && S > 0.0f;
                const uint64_t key = fold_key(fold_rank_lr(A, S), (uint32_t)j * (uint32_t)I + (uint32_t)eh);
                best[b] = ok && key > best[b] ? key : best[b];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const uint64_t m = wave_max_u64(best[b]);
        if (lane == 0 && m != 0) atomicMax((unsigned long long *)&keys[b], (unsigned long long)m);
    }
}

// Fold unit on a coarser epoch grid: epochs e (in units of `s` reference
// times) of duration row j, i.e. fine epochs i = e s, with the transits at
// i + round(m R / 2^32) on the fixed grid as in fold_unit.  Lane l takes
// coarse epochs e_wave + l and e_wave + 64 + l (one 8-byte load each per
// period and step; lanes s elements apart).  ipb[b] counts coarse epochs.
// Offsets, the loop exit, the FP32 chunking and the keys (fine flat index)
// follow fold_unit, so a kept candidate ranks exactly as there.
template <int B>
__device__ __forceinline__ void fold_unit_strided(const float2 *row, int32_t j, int32_t I, int32_t s,
                                                  const uint64_t (&R)[B], const int32_t (&ipb)[B], int32_t e_lo,
                                                  int32_t e_hi, uint64_t *keys) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const __amdgpu_buffer_rsrc_t rsrc = row_resource(row, I);
    const uint32_t uI = (uint32_t)I;
    uint32_t Rh[B], Rl[B];
    uint64_t r_min = ~0ull;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        Rh[b] = __builtin_amdgcn_readfirstlane((uint32_t)(R[b] >> 32));
        Rl[b] = __builtin_amdgcn_readfirstlane((uint32_t)R[b]);
        r_min = ipb[b] > 0 && R[b] < r_min ? R[b] : r_min;
    }
    if (r_min == ~0ull) return;
    const uint32_t Rh_min = __builtin_amdgcn_readfirstlane((uint32_t)(r_min >> 32));
    const uint32_t Rl_min = __builtin_amdgcn_readfirstlane((uint32_t)r_min);
    uint64_t best[B];
#pragma unroll
    for (int b = 0; b < B; ++b) best[b] = 0;

    for (int32_t e0 = e_lo; e0 < e_hi; e0 += kFoldTileEpochs) {
        const int32_t e_wave = e0 + wave * kFoldWaveEpochs;  // wave-uniform
        if (e_wave >= e_hi) break;
        const int32_t e = e_wave + lane;  // coarse epochs e and e + 64
        // fine epochs, saturated at I (past the row every load reads zero and
        // the epoch is not a candidate), so byte offsets stay below 16 I
        const uint32_t f0 = (uint32_t)min((int64_t)e * s, (int64_t)I);
        const uint32_t f1 = (uint32_t)min((int64_t)(e + 64) * s, (int64_t)I);
        const uint32_t b0 = f0 * 8u, b1 = f1 * 8u;
        // e_wave < ceil(I_P / s) gives e_wave s < I_P <= I
        const uint32_t lim = uI - (uint32_t)e_wave * (uint32_t)s;
        float a0[B], s0[B], a1[B], s1[B], ta0[B], ts0[B], ta1[B], ts1[B];
        uint32_t hi[B], lo[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            a0[b] = s0[b] = a1[b] = s1[b] = 0.0f;
            ta0[b] = ts0[b] = ta1[b] = ts1[b] = 0.0f;
            hi[b] = 0;
            lo[b] = 0x80000000u;  // + 1/2: round half up
        }
        uint32_t h_min = 0, l_min = 0x80000000u;
        {
            const float2 v0 = load_pair(rsrc, b0, 0);
            const float2 v1 = load_pair(rsrc, b1, 0);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                acc_add(lo[b], hi[b], Rl[b], Rh[b]);
                hi[b] = min(hi[b], uI);
            }
            acc_add(l_min, h_min, Rl_min, Rh_min);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                a0[b] += v0.x;
                s0[b] += v0.y;
                a1[b] += v1.x;
                s1[b] += v1.y;
            }
        }
        int mm0 = 1;
        while (h_min < lim) {
            for (int mm = mm0; mm < kFoldChunk && h_min < lim; ++mm) {
                float2 v0[B], v1[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    v0[b] = load_pair(rsrc, b0 + hi[b] * 8u, 0);
                    v1[b] = load_pair(rsrc, b1 + hi[b] * 8u, 0);
                }
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    acc_add(lo[b], hi[b], Rl[b], Rh[b]);
                    hi[b] = min(hi[b], uI);
                }
                acc_add(l_min, h_min, Rl_min, Rh_min);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    a0[b] += v0[b].x;
                    s0[b] += v0[b].y;
                    a1[b] += v1[b].x;
                    s1[b] += v1[b].y;
                }
            }
            mm0 = 0;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                ta0[b] += a0[b];
                ts0[b] += s0[b];
                ta1[b] += a1[b];
                ts1[b] += s1[b];
                a0[b] = s0[b] = a1[b] = s1[b] = 0.0f;
            }
        }
        if (mm0) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                ta0[b] += a0[b];
                ts0[b] += s0[b];
                ta1[b] += a1[b];
                ts1[b] += s1[b];
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int32_t eh = e + 64 * h;
                const float A = h ? ta1[b] : ta0[b];
                const float S = h ? ts1[b] : ts0[b];
                const bool ok = eh < ipb[b] && eh < e_hi && S > 0.0f;
                const uint32_t fine = h ? f1 : f0;
                const uint64_t key = fold_key(fold_rank_lr(A, S), (uint32_t)j * (uint32_t)I + fine);
                best[b] = ok && key > best[b] ? key : best[b];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const uint64_t m = wave_max_u64(best[b]);
        if (lane == 0 && m != 0) atomicMax((unsigned long long *)&keys[b], (unsigned long long)m);
    }
}

// FP64 sums of one candidate (epoch i of row `row`, period step R), in
// transit order.
__device__ __forceinline__ void fold_sums(const float2 *row, int64_t I, uint64_t R, int64_t i, double &A, double &S) {
    A = 0.0;
    S = 0.0;
    if (R < 4294967296ull) return;  // not a valid period step (offsets would not advance)
    for (uint64_t acc = 2147483648ull;; acc += R) {
        const int64_t x = i + (int64_t)(acc >> 32);
        if (x >= I) break;
        const float2 v = row[x];
        A += (double)v.x;
        S += (double)v.y;
    }
}

// Decode a period's key into (lr, epoch, dur, depth, depth_var); a zero key
// is the null record.  Returns the LR as written (0 for null).
__device__ __forceinline__ float fold_decode(const float2 *fold, int64_t I, int32_t n_dur, uint64_t R, uint64_t key,
                                             float *lr, int32_t *ep, int32_t *du, float *z, float *zv) {
    const uint32_t flat_ = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
    if (key == 0 || R < 4294967296ull || flat_ / (uint32_t)I >= (uint32_t)n_dur) {
        *lr = 0.0f;
        *ep = -1;
        *du = -1;
        *z = __builtin_nanf("");
        *zv = __builtin_inff();
        return 0.0f;
    }
    const uint32_t flat = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
    const int32_t j = (int32_t)(flat / (uint32_t)I);
    const int32_t i = (int32_t)(flat % (uint32_t)I);
    double A, S;
    fold_sums(fold + (int64_t)j * I, I, R, i, A, S);
    const float l = (float)(0.5 * A * A / S);
    *lr = l;
    *ep = i;
    *du = j;
    *z = (float)(A / S);
    *zv = (float)(1.0 / S);
    return l;
}

}  // namespace dev
}  // namespace cetra
