// Proposal network, after the convolutional trunk: the linear event
// projection, fold pooling (a coarse periodic search of each event channel
// at a few trial periods per period window), a shared MLP head per window,
// the weighted binary cross-entropy, the Adam step, and the top-K window
// selection that restricts the periodic search (Sec. 2.3) to the proposed
// period windows.  VALU kernels (the work here is small next to the
// convolutions).
//
// Shapes: B examples, L bins, E event channels (<= 16), W windows; e is
// [B][L][E] FP32, window features f are [B][W][E + 1] = (best fold score per
// channel, window position), logits z are [B][W].
#include <cmath>

#include "common.h"

namespace {

constexpr int kT = 256;
constexpr int kWidth = 64;
constexpr int kMaxE = 16;
constexpr int kMaxL = 8192;  // bins of an event series (staged in LDS)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// e[b][t][c] = sum_ci P[c][ci] h[b][t][ci] + p[c]
__global__ void project_fwd_kernel(const __bf16 *__restrict__ h, int64_t n_pos, const float *__restrict__ P,
                                   const float *__restrict__ p, int32_t E, float *__restrict__ e) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n_pos) return;
    float hv[kWidth];
#pragma unroll
    for (int ci = 0; ci < kWidth; ++ci) hv[ci] = (float)h[pos * kWidth + ci];
    for (int c = 0; c < E; ++c) {
        float s = p[c];
#pragma unroll
        for (int ci = 0; ci < kWidth; ++ci) s = fmaf(P[c * kWidth + ci], hv[ci], s);
        e[pos * E + c] = s;
    }
}

// dh[pos][ci] = sum_c P[c][ci] ge[pos][c]: a lane per (position, 4
// consecutive channels), so consecutive lanes write consecutive 16 bytes.
__global__ void __launch_bounds__(kT) project_bwd_dh_kernel(const float *__restrict__ ge, int64_t n_pos,
                                                            const float *__restrict__ P, int32_t E,
                                                            float *__restrict__ dh) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_pos * (kWidth / 4)) return;
    const int64_t pos = id / (kWidth / 4);
    const int ci = 4 * (int)(id % (kWidth / 4));
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int c = 0; c < E; ++c) {
        const float g = ge[pos * E + c];
#pragma unroll
        for (int r = 0; r < 4; ++r) s[r] = fmaf(P[c * kWidth + ci + r], g, s[r]);
    }
    *reinterpret_cast<float4 *>(dh + pos * kWidth + ci) = make_float4(s[0], s[1], s[2], s[3]);
}

// dP[c][ci] += sum_pos ge[pos][c] h[pos][ci] and dp[c] += sum_pos ge[pos][c]
// over kProjChunk positions per workgroup: wave w takes a quarter of them in
// order, lane ci holds the E sums of its channel, lanes c < E the bias
// sums.  The four waves' sums meet in LDS and wave 0 adds them with one
// atomic per (c, ci) and workgroup.  (Any E up to kMaxE; E = 8 has its own
// kernel below.)
constexpr int kProjChunk = 1024;
__global__ void __launch_bounds__(kT) project_bwd_dp_kernel(const __bf16 *__restrict__ h,
                                                            const float *__restrict__ ge, int64_t n_pos, int32_t E,
                                                            float *__restrict__ dP, float *__restrict__ dp) {
    constexpr int kWaves = kT / 64;
    __shared__ float s_acc[kWaves][kMaxE][kWidth];
    __shared__ float s_b[kWaves][kMaxE];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t q0 = (int64_t)blockIdx.x * kProjChunk + (int64_t)wave * (kProjChunk / kWaves);
    const int64_t q1 = min(q0 + kProjChunk / kWaves, n_pos);
    float acc[kMaxE];
#pragma unroll
    for (int c = 0; c < kMaxE; ++c) acc[c] = 0.0f;
    float accb = 0.0f;
    for (int64_t pos = q0; pos < q1; ++pos) {
        const float hv = (float)h[pos * kWidth + lane];
        const float *gp = ge + pos * E;
#pragma unroll
        for (int c = 0; c < kMaxE; ++c)
            if (c < E) acc[c] = fmaf(gp[c], hv, acc[c]);
        if (lane < E) accb += gp[lane];
    }
#pragma unroll
    for (int c = 0; c < kMaxE; ++c) s_acc[wave][c][lane] = acc[c];
    if (lane < kMaxE) s_b[wave][lane] = accb;
    __syncthreads();
    if (wave != 0) return;
    for (int c = 0; c < E; ++c) {
        float t = s_acc[0][c][lane];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t += s_acc[w][c][lane];
        atomicAdd(&dP[c * kWidth + lane], t);
    }
    if (lane < E) {
        float t = s_b[0][lane];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t += s_b[w][lane];
        atomicAdd(&dp[lane], t);
    }
}

// The same for E = 8 with wide reads: lane (j, g) = (lane / 8, lane % 8)
// takes channels 8 g .. 8 g + 7 of every eighth position (16 bytes of h, so
// a wave reads eight whole 128-byte rows at once, and the position's 32
// bytes of ge) and keeps 8 x 8 sums plus the 8 bias sums.  The 32 (wave, j)
// partial sums of each output meet in LDS and are added in a fixed order,
// then one atomic per output and workgroup.
constexpr int kProj8Chunk = 1024;
__global__ void __launch_bounds__(kT) project_bwd_dp8_kernel(const __bf16 *__restrict__ h,
                                                             const float *__restrict__ ge, int64_t n_pos,
                                                             float *__restrict__ dP, float *__restrict__ dp) {
    constexpr int kE = 8;
    constexpr int kWaves = kT / 64;
    __shared__ float s_acc[kWaves * 8][kE][kWidth];  // [wave * 8 + j][c][ci]: 64 KB
    __shared__ float s_b[kWaves * 8][kE];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j = lane >> 3, g8 = 8 * (lane & 7);
    const int64_t q0 = (int64_t)blockIdx.x * kProj8Chunk + (int64_t)wave * (kProj8Chunk / kWaves);
    float acc[kE][8], accb[kE];
#pragma unroll
    for (int c = 0; c < kE; ++c) {
        accb[c] = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[c][k] = 0.0f;
    }
#pragma unroll 2
    for (int it = 0; it < kProj8Chunk / kWaves / 8; ++it) {
        const int64_t pos = q0 + 8 * it + j;
        if (pos < n_pos) {
            const bf16x8 hv8 = *reinterpret_cast<const bf16x8 *>(h + pos * kWidth + g8);
            const float4 ga = *reinterpret_cast<const float4 *>(ge + pos * kE);
            const float4 gb = *reinterpret_cast<const float4 *>(ge + pos * kE + 4);
            const float gv[kE] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
#pragma unroll
            for (int c = 0; c < kE; ++c) {
                accb[c] += gv[c];
#pragma unroll
                for (int k = 0; k < 8; ++k) acc[c][k] = fmaf(gv[c], (float)hv8[k], acc[c][k]);
            }
        }
    }
    const int row = wave * 8 + j;
#pragma unroll
    for (int c = 0; c < kE; ++c) {
#pragma unroll
        for (int k = 0; k < 8; ++k) s_acc[row][c][g8 + k] = acc[c][k];
        if (g8 == 0) s_b[row][c] = accb[c];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < kE * kWidth; o += kT) {
        const int c = o / kWidth, ci = o % kWidth;
        float t = 0.0f;
        for (int r = 0; r < kWaves * 8; ++r) t += s_acc[r][c][ci];
        atomicAdd(&dP[o], t);
    }
    if (threadIdx.x < kE) {
        float t = 0.0f;
        for (int r = 0; r < kWaves * 8; ++r) t += s_b[r][threadIdx.x];
        atomicAdd(&dp[threadIdx.x], t);
    }
}

// ---------------------------------------------------------- fold pooling
// Coarse fold of each event series at every window's trial periods.  Trial
// T (bins) has the 32.32 step R = floor(2^32 T + 1/2); phase phi in
// [0, min(L, ceil(R / 2^32))) sums e over the positions phi + ((k R + 2^31)
// >> 32) inside the series; its count n is the number of those positions.
// Per (example, window, channel) the feature is the best score over the
// window's trials and phases, the decision taken on the FP32 score
// fl(S * r(n)), r(n) = fl(1 / sqrt(n)) rounded from FP64 (ties: first trial,
// then smallest phase); f holds that FP32 score and arg keeps
// trial * 65536 + phase.  One workgroup per (channel, example, window group)
// with the series staged in LDS; each wave takes whole windows.  Sums are
// FP32 (exact for the integer-valued inputs of the tests).
// 0 for a trial that is not finite or shorter than one bin (such a trial is
// skipped: its offsets would not advance)
__device__ __forceinline__ uint64_t trial_step(double T) {
    return (T >= 1.0 && T < 1.0e9) ? (uint64_t)floor(4294967296.0 * T + 0.5) : 0ull;
}

__device__ __forceinline__ float inv_sqrt_count(int32_t n) {
    return n > 0 ? (float)(1.0 / sqrt((double)n)) : 0.0f;
}

// Sums over the transit positions of the 64 P phases ph = ph0 + lane + 64 v
// (v < P) of one wave.  The offset of transit k, ((k R + 2^31) >> 32), is the
// same for every phase: it is stepped once per wave in scalar registers.
// While the group's last phase is still inside the series at transit k
// ("full" transits, the bulk) every lane reads without a bounds test, eight
// transits at a time; transit k always adds into partial sum k mod 4.  The
// few transits after that ("tail", while the group's first phase is inside)
// read past the series into the zero padding after it (kFoldPad >= 64 P - 1
// floats), which adds nothing.  Lanes past the trial's phases still read
// inside the staged array; the caller ignores them.
constexpr int kFoldPad = 128;

template <int P>
__device__ __forceinline__ void fold_sum_group(const float *s_e, uint32_t uL, uint64_t step, uint32_t ph0, int lane,
                                               float (&sum)[P]) {
    static_assert(64 * P - 1 <= kFoldPad, "tail reads must stay inside the padding");
    float a[P][4], t[P];
#pragma unroll
    for (int v = 0; v < P; ++v) {
        a[v][0] = a[v][1] = a[v][2] = a[v][3] = 0.0f;
        t[v] = 0.0f;
    }
    const uint32_t base = ph0 + (uint32_t)lane;
    // full transits: offset < uL - (ph0 + 64 P - 1)
    const uint32_t last = ph0 + 64u * P - 1u;
    const uint32_t lim_full = uL > last ? uL - last : 0u;
    uint64_t o = 2147483648ull;
    // (a step of 2^45 or more, a trial of at least kMaxL bins, has one
    // transit in the series; the guard also keeps 7 steps from overflowing).
    // The offsets of a block of eight are o + u step with the multiples
    // precomputed: two scalar adds per transit.
    if (step < (1ull << 45)) {
        uint64_t m[8];
        m[0] = 0;
#pragma unroll
        for (int u = 1; u < 8; ++u) m[u] = m[u - 1] + step;
        const uint64_t m8 = m[7] + step;
        while ((uint32_t)((o + m[7]) >> 32) < lim_full) {
            uint32_t ou[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) ou[u] = (uint32_t)((o + m[u]) >> 32);
            float val[P][8];
#pragma unroll
            for (int v = 0; v < P; ++v)
#pragma unroll
                for (int u = 0; u < 8; ++u) val[v][u] = s_e[base + 64u * v + ou[u]];
#pragma unroll
            for (int v = 0; v < P; ++v)
#pragma unroll
                for (int u = 0; u < 8; ++u) a[v][u & 3] += val[v][u];
            o += m8;
        }
    }
    if ((uint32_t)((o + 3 * step) >> 32) < lim_full) {
        uint32_t ou[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ou[u] = (uint32_t)(o >> 32);
            o += step;
        }
#pragma unroll
        for (int v = 0; v < P; ++v)
#pragma unroll
            for (int u = 0; u < 4; ++u) a[v][u] += s_e[base + 64u * v + ou[u]];
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        if ((uint32_t)(o >> 32) >= lim_full) break;  // wave-uniform
        const uint32_t ou = (uint32_t)(o >> 32);
#pragma unroll
        for (int v = 0; v < P; ++v) a[v][u] += s_e[base + 64u * v + ou];
        o += step;
    }
    // tail: transits while the group's first phase is in the series
    const uint32_t lim0 = uL - ph0;  // ph0 < L
    while ((uint32_t)(o >> 32) < lim0) {
        const uint32_t ou = (uint32_t)(o >> 32);
#pragma unroll
        for (int v = 0; v < P; ++v) t[v] += s_e[base + 64u * v + ou];  // < L + 64 P - 1; 0 past the series
        o += step;
    }
#pragma unroll
    for (int v = 0; v < P; ++v) sum[v] = ((a[v][0] + a[v][1]) + (a[v][2] + a[v][3])) + t[v];
}

// The same sums for a trial of few transits per phase (at most about eight):
// one accumulator per phase, every transit while the group's first phase is
// inside the series, four at a time, reads past the series landing in the
// zero padding.
template <int P>
__device__ __forceinline__ void fold_sum_group_sparse(const float *s_e, uint32_t uL, uint64_t step, uint32_t ph0,
                                                      int lane, float (&sum)[P]) {
    static_assert(64 * P - 1 <= kFoldPad, "reads past the series must stay inside the padding");
#pragma unroll
    for (int v = 0; v < P; ++v) sum[v] = 0.0f;
    const uint32_t base = ph0 + (uint32_t)lane;
    const uint32_t lim0 = uL - ph0;  // ph0 < L
    uint64_t o = 2147483648ull;
    while ((uint32_t)((o + 3 * step) >> 32) < lim0) {
        uint32_t ou[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ou[u] = (uint32_t)((o + u * step) >> 32);
        float val[P][4];
#pragma unroll
        for (int v = 0; v < P; ++v)
#pragma unroll
            for (int u = 0; u < 4; ++u) val[v][u] = s_e[base + 64u * v + ou[u]];
#pragma unroll
        for (int v = 0; v < P; ++v) sum[v] += (val[v][0] + val[v][1]) + (val[v][2] + val[v][3]);
        o += 4 * step;
    }
    while ((uint32_t)(o >> 32) < lim0) {
        const uint32_t ou = (uint32_t)(o >> 32);
#pragma unroll
        for (int v = 0; v < P; ++v) sum[v] += s_e[base + 64u * v + ou];
        o += step;
    }
}

// One trial's phases of a wave, P per lane: scores, and the lane's best
// (score, index) updated in increasing index order (so a strict comparison
// keeps the first of equal scores).  Phase 0 has n0 = ceil((2^32 L - 2^31)
// / R) transit positions in the series, the number of k with
// (k R + 2^31) >> 32 < L.  The phases span fewer bins than the gap between
// two transits, so only transit n0 - 1 can leave the series across them: a
// phase has n0 positions below ph_split = L - ((( n0 - 1) R + 2^31) >> 32)
// and n0 - 1 from there on.
template <int P>
__device__ __forceinline__ void fold_trial(const float *s_e, uint32_t uL, uint64_t step, int32_t n_ph, int32_t q,
                                           int32_t n_ph_max, int lane, float &best, int32_t &bj) {
    const uint64_t num = ((uint64_t)uL << 32) - 2147483649ull;  // 2^32 L - 2^31 - 1 >= 2^31 - 1
    const int32_t n0 = (int32_t)(num / step) + 1;
    const int32_t ph_split = (int32_t)uL - (int32_t)(((uint64_t)(n0 - 1) * step + 2147483648ull) >> 32);
    const float r0 = inv_sqrt_count(n0), r1 = inv_sqrt_count(n0 - 1);
    const bool sparse = step >= ((uint64_t)uL << 29);  // at most about 8 transits per phase
    for (int32_t ph0 = 0; ph0 < n_ph; ph0 += 64 * P) {
        float sum[P];
        if (sparse)
            fold_sum_group_sparse<P>(s_e, uL, step, (uint32_t)ph0, lane, sum);
        else
            fold_sum_group<P>(s_e, uL, step, (uint32_t)ph0, lane, sum);
#pragma unroll
        for (int v = 0; v < P; ++v) {
            const int32_t ph = ph0 + lane + 64 * v;
            const float sc = sum[v] * (ph < ph_split ? r0 : r1);
            if (ph < n_ph && sc > best) {
                best = sc;
                bj = q * n_ph_max + ph;
            }
        }
    }
}

// Grid (channel, example, window group); each workgroup of eight waves
// stages its event series in LDS (33 KB, so four workgroups, eight waves per
// SIMD, share a CU and hide each other's LDS and scalar latencies), and each
// wave takes whole windows (wave index = group * 8 + wave, striding by
// 8 n_groups), so a window's maximum is a wave reduction.  Trials with more
// than 64 phases take two phases per lane, so each scalar offset step serves
// 128 phases.
constexpr int kFoldThreads = 512;
__global__ void __launch_bounds__(kFoldThreads) foldpool_fwd_kernel(const float *__restrict__ e, int32_t L, int32_t E,
                                                          const double *__restrict__ trials, int32_t W, int32_t S,
                                                          const float *__restrict__ win_q, float *__restrict__ f,
                                                          int32_t *__restrict__ arg) {
    __shared__ float s_e[kMaxL + kFoldPad];
    const int32_t c = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int32_t nf = E + 1;
    const int lane = threadIdx.x & 63;
    const int32_t wave_id = blockIdx.z * (kFoldThreads / 64) + (threadIdx.x >> 6);
    const int32_t n_waves = gridDim.z * (kFoldThreads / 64);
    const uint32_t uL = (uint32_t)L;
    for (int t = threadIdx.x; t < L + kFoldPad; t += kFoldThreads) s_e[t] = t < L ? e[(b * L + t) * E + c] : 0.0f;
    __syncthreads();
    for (int32_t w = wave_id; w < W; w += n_waves) {
        int32_t n_ph_max = 0;
        for (int32_t q = 0; q < S; ++q) {
            const uint64_t R = trial_step(trials[w * S + q]);
            n_ph_max = max(n_ph_max, (int32_t)min<uint64_t>((uint64_t)L, (R + 4294967295ull) >> 32));
        }
        float best = -INFINITY;
        int32_t bj = INT_MAX;
        for (int32_t q = 0; q < S; ++q) {
            const uint64_t R = trial_step(trials[w * S + q]);
            const uint32_t Rh = __builtin_amdgcn_readfirstlane((uint32_t)(R >> 32));
            const uint32_t Rl = __builtin_amdgcn_readfirstlane((uint32_t)R);
            const uint64_t step = ((uint64_t)Rh << 32) | Rl;
            if (step == 0) continue;
            const int32_t n_ph = (int32_t)min<uint64_t>((uint64_t)L, (step + 4294967295ull) >> 32);
            if (n_ph > 64)
                fold_trial<2>(s_e, uL, step, n_ph, q, n_ph_max, lane, best, bj);
            else
                fold_trial<1>(s_e, uL, step, n_ph, q, n_ph_max, lane, best, bj);
        }
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(best, off, 64);
            const int32_t oj = __shfl_xor(bj, off, 64);
            if (ov > best || (ov == best && oj < bj)) {
                best = ov;
                bj = oj;
            }
        }
        if (lane == 0) {
            const bool none = bj == INT_MAX;  // no valid trial, or no finite score
            f[(b * W + w) * nf + c] = none ? 0.0f : best;
            arg[(b * W + w) * E + c] = none ? -1 : (bj / n_ph_max) * 65536 + bj % n_ph_max;
            if (c == 0) f[(b * W + w) * nf + E] = win_q[w];
        }
    }
}

// ge[b][t][c] (overwritten) = sum over windows of gf[b][w][c] / sqrt(n) at
// every transit position of the window's winning (trial, phase).
__global__ void __launch_bounds__(kT) foldpool_bwd_kernel(const float *__restrict__ gf, const int32_t *__restrict__ arg,
                                                          const double *__restrict__ trials, int32_t L, int32_t E,
                                                          int32_t W, int32_t S, float *__restrict__ ge) {
    __shared__ float s_g[kMaxL];
    const int32_t c = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int32_t nf = E + 1;
    for (int t = threadIdx.x; t < L; t += kT) s_g[t] = 0.0f;
    __syncthreads();
    for (int32_t w = threadIdx.x; w < W; w += kT) {
        const int32_t a = arg[(b * W + w) * E + c];
        const int32_t q = a >> 16, ph = a & 0xFFFF;
        if (q < 0 || q >= S) continue;
        const uint64_t R = trial_step(trials[w * S + q]);
        if (R == 0) continue;
        int32_t n = 0;
        for (uint64_t o = 2147483648ull;; o += R) {
            if ((uint64_t)ph + (o >> 32) >= (uint64_t)L) break;
            ++n;
        }
        if (n == 0) continue;
        const float gg = gf[(b * W + w) * nf + c] / sqrtf((float)n);
        for (uint64_t o = 2147483648ull;; o += R) {
            const uint64_t x = (uint64_t)ph + (o >> 32);
            if (x >= (uint64_t)L) break;
            atomicAdd(&s_g[x], gg);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < L; t += kT) ge[(b * L + t) * E + c] = s_g[t];
}

// z[b][w] = v . relu(U f + u) + v0 (hidden width <= 128)
constexpr int kMaxHidden = 128;
__global__ void head_fwd_kernel(const float *__restrict__ f, int64_t n_bw, int32_t nf, const float *__restrict__ U,
                                const float *__restrict__ u, const float *__restrict__ v, const float *__restrict__ v0,
                                int32_t H, float *__restrict__ z) {
    const int64_t bw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bw >= n_bw) return;
    float s = v0[0];
    for (int hh = 0; hh < H; ++hh) {
        float r = u[hh];
        for (int k = 0; k < nf; ++k) r = fmaf(U[hh * nf + k], f[bw * nf + k], r);
        s = fmaf(v[hh], fmaxf(r, 0.0f), s);
    }
    z[bw] = s;
}

// Weighted BCE with logits, mean over (b, w): loss (atomic sum) and dz.
__global__ void bce_kernel(const float *__restrict__ z, const float *__restrict__ y, int64_t n, float pos_weight,
                           float *__restrict__ gz, float *__restrict__ loss) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < n) {
        const float zz = z[i], yy = y[i];
        const float wt = yy > 0.5f ? pos_weight : 1.0f;
        l = wt * (fmaxf(zz, 0.0f) - zz * yy + log1pf(expf(-fabsf(zz)))) / (float)n;
        gz[i] = wt * (1.0f / (1.0f + expf(-zz)) - yy) / (float)n;
    }
    l = wave_sum(l);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

// Head backward: the window-feature gradients gf[b][w][k] per row, and the
// parameter gradients summed over the workgroup's kHeadRows rows in LDS
// (per-row terms staged there; one thread per parameter sums them), so each
// workgroup adds one FP32 atomic per parameter.  The rows' features are
// staged in LDS first; then wave q takes hidden units q, q + 4, ... of every
// row (lane = row), so the weights it reads are wave-uniform, and the four
// waves' partial feature gradients are added in order.  Loops over the
// features are unrolled to their maximum with a guard, which keeps the
// per-row arrays in registers.
constexpr int kHeadRows = 64;
constexpr int kHeadMaxF = 2 * kMaxE + 1;
__global__ void __launch_bounds__(kT) head_bwd_kernel(const float *__restrict__ f, int64_t n_bw, int32_t nf,
                                                      const float *__restrict__ U, const float *__restrict__ u,
                                                      const float *__restrict__ v, int32_t H,
                                                      const float *__restrict__ gz, float *__restrict__ gU,
                                                      float *__restrict__ gu, float *__restrict__ gv,
                                                      float *__restrict__ gv0, float *__restrict__ gf) {
    constexpr int kWaves = kT / 64;
    static_assert(kHeadRows == 64, "one lane per row");
    __shared__ float s_gp[kHeadRows][kMaxHidden + 1];   // dL/d(pre-activation) of the hidden units
    __shared__ float s_grr[kHeadRows][kMaxHidden + 1];  // gz times the hidden activation
    __shared__ float s_f[kHeadRows][kHeadMaxF];
    __shared__ float s_gfp[kWaves][kHeadRows][kHeadMaxF];  // partial feature gradients per wave
    __shared__ float s_g[kHeadRows];
    const int64_t row0 = (int64_t)blockIdx.x * kHeadRows;
    const int64_t n_rows = min((int64_t)kHeadRows, n_bw - row0);
    for (int i = threadIdx.x; i < kHeadRows * nf; i += kT) {
        const int r = i / nf, k = i % nf;
        s_f[r][k] = r < n_rows ? f[(row0 + r) * nf + k] : 0.0f;
    }
    for (int r = threadIdx.x; r < kHeadRows; r += kT) s_g[r] = r < n_rows ? gz[row0 + r] : 0.0f;
    __syncthreads();
    {
        const int r = threadIdx.x & 63;
        const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const float g = s_g[r];
        float fv[kHeadMaxF], gfv[kHeadMaxF];
#pragma unroll
        for (int k = 0; k < kHeadMaxF; ++k) {
            fv[k] = k < nf ? s_f[r][k] : 0.0f;
            gfv[k] = 0.0f;
        }
        for (int hh = q; hh < H; hh += kWaves) {
            const float *Uh = U + hh * nf;
            float pre = u[hh];
#pragma unroll
            for (int k = 0; k < kHeadMaxF; ++k)
                if (k < nf) pre = fmaf(Uh[k], fv[k], pre);
            const float gp = pre > 0.0f ? g * v[hh] : 0.0f;
            s_gp[r][hh] = gp;
            s_grr[r][hh] = g * fmaxf(pre, 0.0f);
#pragma unroll
            for (int k = 0; k < kHeadMaxF; ++k)
                if (k < nf) gfv[k] = fmaf(Uh[k], gp, gfv[k]);
        }
#pragma unroll
        for (int k = 0; k < kHeadMaxF; ++k)
            if (k < nf) s_gfp[q][r][k] = gfv[k];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHeadRows * nf; i += kT) {
        const int r = i / nf, k = i % nf;
        if (r >= n_rows) continue;
        float t = s_gfp[0][r][k];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t += s_gfp[w][r][k];
        gf[(row0 + r) * nf + k] = t;
    }
    __syncthreads();
    // parameters: gU[hh][k] (H nf), gu[hh] (H), gv[hh] (H), gv0 (1)
    const int n_par = H * nf + 2 * H + 1;
    for (int p = threadIdx.x; p < n_par; p += blockDim.x) {
        float acc = 0.0f;
        if (p < H * nf) {
            const int hh = p / nf, k = p % nf;
            for (int r = 0; r < kHeadRows; ++r) acc = fmaf(s_gp[r][hh], s_f[r][k], acc);
            atomicAdd(&gU[p], acc);
        } else if (p < H * nf + H) {
            const int hh = p - H * nf;
            for (int r = 0; r < kHeadRows; ++r) acc += s_gp[r][hh];
            atomicAdd(&gu[hh], acc);
        } else if (p < H * nf + 2 * H) {
            const int hh = p - H * nf - H;
            for (int r = 0; r < kHeadRows; ++r) acc += s_grr[r][hh];
            atomicAdd(&gv[hh], acc);
        } else {
            for (int r = 0; r < kHeadRows; ++r) acc += s_g[r];
            atomicAdd(gv0, acc);
        }
    }
}

// Adam on FP32 master parameters.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                            float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 copy of FP32 conv weights [co][k32] (k = tap * cin + ci), padding
// columns k >= 9 cin forced to zero.
__global__ void pack_conv_w_kernel(const float *__restrict__ w, int32_t cin, int32_t k32, __bf16 *__restrict__ out) {
    const int32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= kWidth * k32) return;
    const int32_t k = id % k32;
    out[id] = k < 9 * cin ? (__bf16)w[id] : (__bf16)0.0f;
}

// Top-K windows per example by score (bitonic sort of W <= 1024 in LDS;
// ties to the smaller window index); out[b][r] = window of rank r.
__global__ void __launch_bounds__(1024) topk_kernel(const float *__restrict__ z, int32_t W, int32_t K,
                                                    int32_t *__restrict__ out) {
    __shared__ float s_v[1024];
    __shared__ int32_t s_i[1024];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    s_v[tid] = tid < W ? z[b * W + tid] : -INFINITY;
    s_i[tid] = tid < W ? tid : 0x7fffffff;
    __syncthreads();
    // descending by value, ascending index on ties
    for (int size = 2; size <= 1024; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int partner = tid ^ stride;
            if (partner > tid) {
                const bool desc = (tid & size) == 0;
                const float va = s_v[tid], vb = s_v[partner];
                const int32_t ia = s_i[tid], ib = s_i[partner];
                const bool a_first = va > vb || (va == vb && ia < ib);
                if (a_first != desc) {
                    s_v[tid] = vb;
                    s_v[partner] = va;
                    s_i[tid] = ib;
                    s_i[partner] = ia;
                }
            }
            __syncthreads();
        }
    }
    if (tid < K) out[b * K + tid] = s_i[tid];
}

// Period subset of the selected windows: periods (ascending) whose value lies
// in [edges[w], edges[w+1]) for a selected window w, as ascending indices.
// One workgroup; returns the count in *n_out.
__global__ void __launch_bounds__(1024) windows_to_periods_kernel(const double *__restrict__ periods, int64_t K,
                                                                  const double *__restrict__ edges, int32_t W,
                                                                  const int32_t *__restrict__ sel, int32_t n_sel,
                                                                  int64_t *__restrict__ subset,
                                                                  int64_t *__restrict__ n_out) {
    __shared__ uint8_t s_on[4096];
    __shared__ int64_t s_base;
    __shared__ int32_t s_cnt[1024];
    for (int i = threadIdx.x; i < W; i += blockDim.x) s_on[i] = 0;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n_sel; i += blockDim.x)
        if (sel[i] >= 0 && sel[i] < W) s_on[sel[i]] = 1;
    __syncthreads();
    for (int64_t k0 = 0; k0 < K; k0 += blockDim.x) {
        const int64_t k = k0 + threadIdx.x;
        int32_t on = 0;
        if (k < K) {
            const double P = periods[k];
            int lo = 0, hi = W;  // window w with edges[w] <= P < edges[w+1]
            if (P >= edges[0] && P < edges[W]) {
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (edges[mid] <= P)
                        lo = mid;
                    else
                        hi = mid;
                }
                on = s_on[lo];
            }
        }
        s_cnt[threadIdx.x] = on;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {  // inclusive scan
            const int32_t add = threadIdx.x >= (unsigned)off ? s_cnt[threadIdx.x - off] : 0;
            __syncthreads();
            s_cnt[threadIdx.x] += add;
            __syncthreads();
        }
        if (on) subset[s_base + s_cnt[threadIdx.x] - 1] = k;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) s_base += s_cnt[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_out = s_base;
}

}  // namespace

using namespace cetra;

extern "C" int cetra_net_project_fwd(void *stream, const void *h, int64_t n_pos, const float *P, const float *p,
                                     int32_t E, float *e) {
    clear_error();
    CETRA_REQUIRE(h && P && p && e, "net_project_fwd: NULL pointer");
    CETRA_REQUIRE(E >= 1 && E <= kMaxE && n_pos >= 0, "net_project_fwd: bad sizes");
    hipLaunchKernelGGL(project_fwd_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n_pos, 1), kT)), dim3(kT), 0,
                       as_stream(stream), (const __bf16 *)h, n_pos, P, p, E, e);
    return check_launch("net_project_fwd");
}

extern "C" int cetra_net_project_bwd(void *stream, const void *h, const float *ge, int64_t n_pos, const float *P,
                                     int32_t E, float *dh, float *dP, float *dp) {
    clear_error();
    CETRA_REQUIRE(h && ge && P && dh && dP && dp, "net_project_bwd: NULL pointer");
    CETRA_REQUIRE(E >= 1 && E <= kMaxE && n_pos >= 0 && n_pos <= ((int64_t)1 << 31), "net_project_bwd: bad sizes");
    CETRA_REQUIRE(((uintptr_t)dh & 15) == 0, "net_project_bwd: dh must be 16-byte aligned");
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(project_bwd_dh_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n_pos * (kWidth / 4), 1), kT)),
                       dim3(kT), 0, st, ge, n_pos, P, E, dh);
    int rc = check_launch("net_project_bwd/dh");
    if (rc) return rc;
    const bool wide = E == 8 && (((uintptr_t)h | (uintptr_t)ge) & 15) == 0;
    if (wide)
        hipLaunchKernelGGL(project_bwd_dp8_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n_pos, 1), kProj8Chunk)),
                           dim3(kT), 0, st, (const __bf16 *)h, ge, n_pos, dP, dp);
    else
        hipLaunchKernelGGL(project_bwd_dp_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n_pos, 1), kProjChunk)),
                           dim3(kT), 0, st, (const __bf16 *)h, ge, n_pos, E, dP, dp);
    return check_launch("net_project_bwd");
}

static int foldpool_args_ok(int32_t B, int32_t L, int32_t E, int32_t W, int32_t S) {
    CETRA_REQUIRE(B >= 1 && B <= 65535 && L >= 1 && L <= kMaxL && E >= 1 && E <= kMaxE,
                  "net_foldpool: need 1 <= B <= 65535, 1 <= L <= 8192, 1 <= E <= 16");
    CETRA_REQUIRE(W >= 1 && S >= 1 && S <= 32, "net_foldpool: need W >= 1 and 1 <= S <= 32");
    return CETRA_OK;
}

extern "C" int cetra_net_foldpool_fwd(void *stream, const float *e, int32_t B, int32_t L, int32_t E,
                                      const double *trials, int32_t W, int32_t S, const float *win_q, float *f,
                                      int32_t *arg) {
    clear_error();
    CETRA_REQUIRE(e && trials && win_q && f && arg, "net_foldpool_fwd: NULL pointer");
    int rc = foldpool_args_ok(B, L, E, W, S);
    if (rc) return rc;
    // window groups: enough workgroups to fill the chip even for one example
    const int64_t want = (int64_t)4 * device_cu_count();
    const int32_t groups = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(ceil_div(W, kFoldThreads / 64), ceil_div(want, (int64_t)E * B)));
    hipLaunchKernelGGL(foldpool_fwd_kernel, dim3((unsigned)E, (unsigned)B, (unsigned)groups), dim3(kFoldThreads), 0,
                       as_stream(stream), e, L, E, trials, W, S, win_q, f, arg);
    return check_launch("net_foldpool_fwd");
}

extern "C" int cetra_net_foldpool_bwd(void *stream, const float *gf, const int32_t *arg, const double *trials,
                                      int32_t B, int32_t L, int32_t E, int32_t W, int32_t S, float *ge) {
    clear_error();
    CETRA_REQUIRE(gf && arg && trials && ge, "net_foldpool_bwd: NULL pointer");
    int rc = foldpool_args_ok(B, L, E, W, S);
    if (rc) return rc;
    hipLaunchKernelGGL(foldpool_bwd_kernel, dim3((unsigned)E, (unsigned)B), dim3(kT), 0, as_stream(stream), gf, arg,
                       trials, L, E, W, S, ge);
    return check_launch("net_foldpool_bwd");
}

extern "C" int cetra_net_head_fwd(void *stream, const float *f, int64_t n_bw, int32_t nf, const float *U,
                                  const float *u, const float *v, const float *v0, int32_t H, float *z) {
    clear_error();
    CETRA_REQUIRE(f && U && u && v && v0 && z, "net_head_fwd: NULL pointer");
    CETRA_REQUIRE(nf >= 1 && nf <= 2 * kMaxE + 1 && H >= 1 && H <= kMaxHidden, "net_head_fwd: bad sizes");
    hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n_bw, 1), kT)), dim3(kT), 0,
                       as_stream(stream), f, n_bw, nf, U, u, v, v0, H, z);
    return check_launch("net_head_fwd");
}

extern "C" int cetra_net_bce(void *stream, const float *z, const float *y, int64_t n, float pos_weight, float *gz,
                             float *loss) {
    clear_error();
    CETRA_REQUIRE(z && y && gz && loss, "net_bce: NULL pointer");
    hipLaunchKernelGGL(bce_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n, 1), kT)), dim3(kT), 0,
                       as_stream(stream), z, y, n, pos_weight, gz, loss);
    return check_launch("net_bce");
}

extern "C" int cetra_net_head_bwd(void *stream, const float *f, int64_t n_bw, int32_t nf, const float *U,
                                  const float *u, const float *v, int32_t H, const float *gz, float *gU, float *gu,
                                  float *gv, float *gv0, float *gf) {
    clear_error();
    CETRA_REQUIRE(f && U && u && v && gz && gU && gu && gv && gv0 && gf, "net_head_bwd: NULL pointer");
    CETRA_REQUIRE(nf >= 1 && nf <= 2 * kMaxE + 1 && H >= 1 && H <= kMaxHidden, "net_head_bwd: bad sizes");
    hipLaunchKernelGGL(head_bwd_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n_bw, 1), kHeadRows)), dim3(kT), 0,
                       as_stream(stream), f, n_bw, nf, U, u, v, H, gz, gU, gu, gv, gv0, gf);
    return check_launch("net_head_bwd");
}

extern "C" int cetra_adam_step(void *stream, float *p, const float *g, float *m, float *v, int64_t n, float lr,
                               float beta1, float beta2, float eps, int64_t step) {
    clear_error();
    CETRA_REQUIRE(p && g && m && v && n >= 0 && step >= 1, "adam_step: bad arguments");
    const float bc1 = 1.0f - powf(beta1, (float)step), bc2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)ceil_div(std::max<int64_t>(n, 1), kT)), dim3(kT), 0,
                       as_stream(stream), p, g, m, v, n, lr, beta1, beta2, eps, bc1, bc2);
    return check_launch("adam_step");
}

extern "C" int cetra_net_pack_conv_w(void *stream, const float *w, int32_t cin, int32_t k32, void *out) {
    clear_error();
    CETRA_REQUIRE(w && out && (cin == 16 || cin == 64) && k32 == (9 * cin + 31) / 32 * 32,
                  "net_pack_conv_w: cin must be 16 or 64 and k32 = 9 cin rounded up to 32");
    hipLaunchKernelGGL(pack_conv_w_kernel, dim3((unsigned)ceil_div(kWidth * k32, kT)), dim3(kT), 0,
                       as_stream(stream), w, cin, k32, (__bf16 *)out);
    return check_launch("net_pack_conv_w");
}

extern "C" int cetra_topk_windows(void *stream, const float *scores, int32_t B, int32_t W, int32_t K,
                                  int32_t *out) {
    clear_error();
    CETRA_REQUIRE(scores && out, "topk_windows: NULL pointer");
    CETRA_REQUIRE(W >= 1 && W <= 1024 && K >= 1 && K <= W && B >= 1, "topk_windows: need 1 <= K <= W <= 1024");
    hipLaunchKernelGGL(topk_kernel, dim3(B), dim3(1024), 0, as_stream(stream), scores, W, K, out);
    return check_launch("topk_windows");
}

extern "C" int cetra_windows_to_periods(void *stream, const double *periods, int64_t K, const double *edges,
                                        int32_t W, const int32_t *sel, int32_t n_sel, int64_t *subset,
                                        int64_t *n_out) {
    clear_error();
    CETRA_REQUIRE(periods && edges && sel && subset && n_out, "windows_to_periods: NULL pointer");
    CETRA_REQUIRE(W >= 1 && W <= 4096 && n_sel >= 0 && K >= 0, "windows_to_periods: bad sizes");
    hipLaunchKernelGGL(windows_to_periods_kernel, dim3(1), dim3(1024), 0, as_stream(stream), periods, K, edges, W, sel,
                       n_sel, subset, n_out);
    return check_launch("windows_to_periods");
}
