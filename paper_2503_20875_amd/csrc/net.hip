// Period-window proposal network (not part of the paper: it ranks period
// windows from the linear search's single-event likelihood ratios so the
// periodic search of Sec. 2.3 folds only the best-ranked windows).
//
// Layouts (channel-last, so an MFMA operand fragment of 8 consecutive
// channels is one 16-byte load):
//   activations  X[b][t][c]  BF16 (inputs of a conv), Y[b][t][64] BF16
//   conv weights W[co][k]    BF16, k = tap * C_in + ci, padded with zeros to
//                            a multiple of 32 (K32)
//   gradients    FP32 in the same layouts
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (FP32
// accumulation):
//   forward      Y[t][co]   = relu(b[co] + sum_k W[co][k] X[t + tap - 4][ci])
//   backward-x   dX[t][ci]  = sum_{tap,co} WT[ci][tap*64 + co] G[t - tap + 4][co]
//   backward-w   dW[co][k]  = sum_{b,t} G[t][co] X[t + tap - 4][ci]
// with G = dY * (Y > 0) in BF16 and WT the per-step transpose of W.
#include <cmath>

#include "common.h"

namespace {

constexpr int kT = 256;
constexpr int kWidth = 64;  // channels of every conv output
constexpr int kTaps = 9;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 load8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

// ---------------------------------------------------------------- probe
// C[16][16] = A[16][32] B[32][16] with one MFMA, A row-major, B row-major
// (used by the tests to pin the operand layout).
__global__ void mfma_probe_kernel(const __bf16 *A, const __bf16 *B, float *C) {
    const int l = threadIdx.x;
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = A[(l % 16) * 32 + 8 * (l / 16) + i];
        b[i] = B[(8 * (l / 16) + i) * 16 + (l % 16)];
    }
    f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
    c = mfma16(a, b, c);
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(4 * (l / 16) + r) * 16 + (l % 16)] = c[r];
}

// ------------------------------------------------------------ downsample
// x[b][bin][j] = min(sqrt(2 LR), 30) / 8 with LR = max over the reference
// times of the bin of S_fm^2 / (2 S_mm) (single-event |SNR|, max-pooled).
__global__ void downsample_kernel(const float2 *__restrict__ fold, int32_t J, int64_t I, int32_t L,
                                  __bf16 *__restrict__ x) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)J * L) return;
    const int32_t bin = (int32_t)(id / J), j = (int32_t)(id % J);
    const int64_t i0 = (int64_t)bin * I / L, i1 = (int64_t)(bin + 1) * I / L;
    float best = 0.0f;
    for (int64_t i = i0; i < i1; ++i) {
        const float2 v = fold[(int64_t)j * I + i];
        if (v.y > 0.0f) best = fmaxf(best, v.x * (v.x / v.y));  // 2 LR = S_fm^2 / S_mm
    }
    x[id] = (__bf16)(fminf(sqrtf(best), 30.0f) * 0.125f);
}

// x[b][bin][j] = clamp(z, -30, 30) / 8 with z = max over the reference times
// of the bin of S_fm / sqrt(S_mm) (signed single-event SNR, max-pooled: a
// dimming gives S_fm > 0); a bin with only null elements gives 0.
__global__ void downsample_signed_kernel(const float2 *__restrict__ fold, int32_t J, int64_t I, int32_t L,
                                         __bf16 *__restrict__ x) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)J * L) return;
    const int32_t bin = (int32_t)(id / J), j = (int32_t)(id % J);
    const int64_t i0 = (int64_t)bin * I / L, i1 = (int64_t)(bin + 1) * I / L;
    float best = -INFINITY;
    for (int64_t i = i0; i < i1; ++i) {
        const float2 v = fold[(int64_t)j * I + i];
        if (v.y > 0.0f) best = fmaxf(best, v.x / sqrtf(v.y));
    }
    x[id] = (__bf16)(best == -INFINITY ? 0.0f : fminf(fmaxf(best, -30.0f), 30.0f) * 0.125f);
}

// ------------------------------------------------------------ conv forward
// Implicit GEMM with a 64 x 64 register tile per wave.  Workgroup: 512
// positions x 64 output channels of one example (8 waves); wave w owns
// positions [64 w, 64 w + 64) (4 MFMA column tiles) and all 16 MT rows
// (MT row tiles).  Both operands are staged in LDS once per workgroup, so the
// reduction loop reads no global memory:
//   A (weights) in fragment order -- the 16-byte fragment of k-step s, row
//     tile m and lane l at ((s MT + m) 64 + l) 16 bytes, so a wave's fragment
//     read is 1 KB contiguous;
//   B (inputs) as the 520 source positions [base - 4, base + 516) of the
//     tile, channel-last with rows padded to c + 8 channels (16 lanes on 16
//     consecutive positions then hit distinct banks); positions outside
//     [0, L) are zero.
// Each k-step's 4 weight and 4 input fragments feed 16 MFMAs, and the next
// k-step's fragments are read while this one's MFMAs issue.  Reduction
// indices past 9 c read zero.
constexpr int kConvWaves = 8;
constexpr int kConvThreads = 64 * kConvWaves;
constexpr int kConvPos = 64 * kConvWaves;  // positions per workgroup
constexpr int kConvHalo = 4;
constexpr int kConvRows = kConvPos + 2 * kConvHalo;
constexpr int kConvMaxK = kTaps * kWidth;  // 576
constexpr int kConvLdsA = kWidth * kConvMaxK * 2;              // bytes: 64 rows x 576, bf16
constexpr int kConvLdsB = kConvRows * (kWidth + 8) * 2;        // bytes: 520 rows x 72, bf16
static_assert(kConvLdsA % 16 == 0 && kConvLdsB % 16 == 0, "16-byte LDS fragments");
static_assert(kConvLdsA == 16 * 4 * (kConvMaxK / 32) * 64, "A holds 4 row tiles x 18 k-steps x 64 fragments");
static_assert(kConvLdsA + kConvLdsB <= 160 * 1024, "one workgroup's LDS");
// 16-byte staging chunks per thread, enough for the largest operands
constexpr int kConvStageIters = 9;
static_assert(kConvStageIters * kConvThreads * 16 >= kConvLdsA, "A chunks per thread");
static_assert(kConvStageIters * kConvThreads >= kConvRows * kWidth / 8, "B chunks per thread");

template <int MT>
struct ConvFrags {
    bf16x8 a[MT];
    bf16x8 b[4];
};

// Stage A rows [0, 16 MT) x [0, KP) of `a_mat` (row stride a_ld) and the
// source rows of `src` (C channels, channel-last) around `base` into LDS.
// Every load of a thread is issued before its first store (from a clamped,
// always valid address; out-of-range chunks are zeroed afterwards), so
// staging waits for memory about once instead of once per chunk.
template <int MT, int C, int KP>
__device__ __forceinline__ void conv_stage(bf16x8 *sA, __bf16 *sB, const __bf16 *__restrict__ a_mat, int32_t a_ld,
                                           const __bf16 *__restrict__ src, int32_t L, int32_t base) {
    constexpr int32_t n_kk = KP / 8, n_a = 16 * MT * n_kk;
    constexpr int32_t n_cc = C / 8, stride = C + 8, n_b = kConvRows * n_cc;
    static_assert(n_a <= kConvStageIters * kConvThreads && n_b <= kConvStageIters * kConvThreads, "chunks");
    bf16x8 va[kConvStageIters], vb[kConvStageIters];
#pragma unroll
    for (int u = 0; u < kConvStageIters; ++u) {
        const int32_t id = min((int32_t)threadIdx.x + u * kConvThreads, n_a - 1);
        va[u] = load8(a_mat + (int64_t)(id / n_kk) * a_ld + 8 * (id % n_kk));
    }
#pragma unroll
    for (int u = 0; u < kConvStageIters; ++u) {
        const int32_t id = min((int32_t)threadIdx.x + u * kConvThreads, n_b - 1);
        const int32_t pos = min(max(base - kConvHalo + id / n_cc, 0), L - 1);
        vb[u] = load8(src + (int64_t)pos * C + 8 * (id % n_cc));
    }
#pragma unroll
    for (int u = 0; u < kConvStageIters; ++u) {
        const int32_t id = threadIdx.x + u * kConvThreads;
        if (id < n_a) {
            const int32_t r = id / n_kk, kk = id % n_kk;
            sA[((kk / 4 * MT + r / 16) * 64) + (r % 16) + 16 * (kk % 4)] = va[u];
        }
    }
#pragma unroll
    for (int u = 0; u < kConvStageIters; ++u) {
        const int32_t id = threadIdx.x + u * kConvThreads;
        const int32_t pos = base - kConvHalo + id / n_cc;
        if (id < n_b)
            *reinterpret_cast<bf16x8 *>(sB + (id / n_cc) * stride + 8 * (id % n_cc)) =
                pos >= 0 && pos < L ? vb[u] : zero8();
    }
}

// Fragments of k-step k0 from LDS: B at source position t + sign (tap - 4)
// (sign +1 forward, -1 for the input gradient), t = tb + 16 n, tb the lane's
// position relative to the staged origin base - 4.
template <int MT, int C>
__device__ __forceinline__ void conv_read(ConvFrags<MT> &f, const bf16x8 *sA, const __bf16 *sB, int32_t k_valid,
                                          int32_t tb, int sign, int32_t k0, int l) {
    const int32_t k = k0 + 8 * (l / 16);
    const int32_t tap = k / C, ci = k % C;
    constexpr int32_t stride = C + 8;
#pragma unroll
    for (int m = 0; m < MT; ++m) f.a[m] = sA[((k0 / 32) * MT + m) * 64 + l];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int32_t rr = tb + 16 * n + sign * (tap - 4);
        f.b[n] = k < k_valid ? *reinterpret_cast<const bf16x8 *>(sB + rr * stride + ci) : zero8();
    }
}

template <int MT>
__device__ __forceinline__ void conv_mfma(f32x4 (&acc)[MT][4], const ConvFrags<MT> &f) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = mfma16(f.a[m], f.b[n], acc[m][n]);
}

// acc[m][n] = sum over the k-steps of A rows x B columns, from the staged
// operands (ping-pong over two fragment sets).
template <int MT, int C, int KP>
__device__ __forceinline__ void conv_gemm(f32x4 (&acc)[MT][4], const bf16x8 *sA, const __bf16 *sB, int32_t k_valid,
                                          int32_t tb, int sign, int l) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    ConvFrags<MT> f0, f1;
    conv_read<MT, C>(f0, sA, sB, k_valid, tb, sign, 0, l);
    for (int32_t k0 = 0; k0 < KP; k0 += 64) {
        const bool more = k0 + 32 < KP;
        if (more) conv_read<MT, C>(f1, sA, sB, k_valid, tb, sign, k0 + 32, l);
        conv_mfma<MT>(acc, f0);
        if (!more) break;
        if (k0 + 64 < KP) conv_read<MT, C>(f0, sA, sB, k_valid, tb, sign, k0 + 64, l);
        conv_mfma<MT>(acc, f1);
    }
}

template <int CIN>
__global__ void __launch_bounds__(kConvThreads) __attribute__((amdgpu_waves_per_eu(2)))
conv_fwd_kernel(const __bf16 *__restrict__ x, int32_t L, const __bf16 *__restrict__ w,
                const float *__restrict__ bias, __bf16 *__restrict__ y) {
    constexpr int32_t k32 = (kTaps * CIN + 31) / 32 * 32;
    __shared__ bf16x8 s_a[kConvLdsA / 16];
    __shared__ bf16x8 s_b[kConvLdsB / 16];
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.y;
    const int32_t base = blockIdx.x * kConvPos;
    conv_stage<4, CIN, k32>(s_a, reinterpret_cast<__bf16 *>(s_b), w, k32, x + b * (int64_t)L * CIN, L, base);
    __syncthreads();
    const int32_t tb = kConvHalo + wave * 64 + (l % 16);  // staged row of this lane's column of tile 0
    f32x4 acc[4][4];
    conv_gemm<4, CIN, k32>(acc, s_a, reinterpret_cast<const __bf16 *>(s_b), kTaps * CIN, tb, +1, l);
    const int32_t t0 = base + wave * 64 + (l % 16);  // this lane's column of tile n: t0 + 16 n
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int32_t t = t0 + 16 * n;
        if (t >= L) continue;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = 16 * m + 4 * (l / 16) + r;
                y[(b * L + t) * kWidth + co] = (__bf16)fmaxf(acc[m][n][r] + bias[co], 0.0f);
            }
    }
}

// G = dY * (Y > 0) in BF16, and the bias gradient is left to bwd-weight.
__global__ void relu_mask_kernel(const float *__restrict__ dy, const __bf16 *__restrict__ y, int64_t n,
                                 __bf16 *__restrict__ g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    g[i] = (float)y[i] > 0.0f ? (__bf16)dy[i] : (__bf16)0.0f;
}

// The same, eight elements per thread (n a multiple of 8; dy 32-byte, y and
// g 16-byte aligned): two 16-byte loads of dY, one of Y, one 16-byte store.
__global__ void relu_mask8_kernel(const float *__restrict__ dy, const __bf16 *__restrict__ y, int64_t n8,
                                  __bf16 *__restrict__ g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const float4 d0 = reinterpret_cast<const float4 *>(dy)[2 * i];
    const float4 d1 = reinterpret_cast<const float4 *>(dy)[2 * i + 1];
    const bf16x8 yy = reinterpret_cast<const bf16x8 *>(y)[i];
    const float d[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    bf16x8 out;
#pragma unroll
    for (int j = 0; j < 8; ++j) out[j] = (float)yy[j] > 0.0f ? (__bf16)d[j] : (__bf16)0.0f;
    reinterpret_cast<bf16x8 *>(g)[i] = out;
}

// WT[ci][tap * 64 + co] = W[co][tap * cin + ci]
__global__ void conv_transpose_w_kernel(const __bf16 *__restrict__ w, int32_t cin, int32_t k32,
                                        __bf16 *__restrict__ wt) {
    const int32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= kWidth * kTaps * cin) return;
    const int32_t ci = id / (kTaps * kWidth), rem = id % (kTaps * kWidth);
    const int32_t tap = rem / kWidth, co = rem % kWidth;
    wt[id] = w[co * k32 + tap * cin + ci];
}

// ------------------------------------------------------- conv backward-x
// dX[b][t][ci] (FP32) = sum over tap, co of WT[ci][tap*64 + co] G[b][t - tap + 4][co],
// the same LDS-staged implicit GEMM as the forward pass with cin / 16 row
// tiles (cin in {16, 64}); workgroup: 512 positions of one example.
template <int MT>
__global__ void __launch_bounds__(kConvThreads) __attribute__((amdgpu_waves_per_eu(2)))
conv_bwd_x_kernel(const __bf16 *__restrict__ g, int32_t L, const __bf16 *__restrict__ wt, float *__restrict__ dx) {
    __shared__ bf16x8 s_a[kConvLdsA / 16];
    __shared__ bf16x8 s_b[kConvLdsB / 16];
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.y;
    const int32_t base = blockIdx.x * kConvPos;
    constexpr int32_t kK = kTaps * kWidth;  // 576, a multiple of 32
    constexpr int cin = 16 * MT;
    conv_stage<MT, kWidth, kK>(s_a, reinterpret_cast<__bf16 *>(s_b), wt, kK, g + b * (int64_t)L * kWidth, L, base);
    __syncthreads();
    const int32_t tb = kConvHalo + wave * 64 + (l % 16);
    f32x4 acc[MT][4];
    conv_gemm<MT, kWidth, kK>(acc, s_a, reinterpret_cast<const __bf16 *>(s_b), kK, tb, -1, l);
    const int32_t t0 = base + wave * 64 + (l % 16);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int32_t t = t0 + 16 * n;
        if (t >= L) continue;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) dx[(b * L + t) * cin + 16 * m + 4 * (l / 16) + r] = acc[m][n][r];
    }
}

// ------------------------------------------------------ conv backward-w
// dW[co][tap * cin + ci] += sum over positions t of G[t][co] X[t + tap - 4][ci]
// and db[co] += sum over t of G[t][co]: a GEMM whose reduction runs over
// positions, so both operands are staged in LDS position-fastest (one chunk
// of 256 positions at a time; X with a 4-position halo on each side).
// Workgroup: chunks_per_wg chunks of one example (8 with atomics, fewer with
// partial sums so that every CU gets a workgroup), eight waves; wave w owns
// output channels [16 (w mod 4), +16) and half of the (ci tile, tap) column
// tiles (w < 4 the first half), so a CU keeps twice as many MFMA streams
// busy as with one wave per channel tile, for the same FP32 atomics.  Per
// 32-position step a lane reads its G fragment (8 positions) and, per ci
// tile, 16 consecutive positions of X (two aligned 16-byte reads); the nine
// taps' fragments are the 8-position windows of those 16 values starting at
// the tap (a register selection for even taps, one byte-align per dword for
// odd taps).  The bias gradient is one more MFMA against a fragment of ones.
// The workgroup's sums go to dW and db by FP32 atomics (kPartial = false),
// or (kPartial = true) to the workgroup's own slab of a partial-sum array,
// [workgroup][64 k32 + 64] FP32, by plain stores; conv_bwd_w_reduce_kernel
// then adds the slabs into dW and db in a fixed order.
constexpr int kPosChunk = 256;
constexpr int kChunksPerWg = 8;
constexpr int kHalo = 4;
constexpr int kBwdWaves = 8;
constexpr int kBwdThreads = 64 * kBwdWaves;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Window of 8 bf16 starting at element s (0..8) of the 16 held in lo, hi.
template <int S>
__device__ __forceinline__ bf16x8 window8(const u32x4 &lo, const u32x4 &hi) {
    const uint32_t v[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    u32x4 w;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        constexpr int q = S / 2;
        if (S % 2 == 0)
            w[d] = v[q + d];
        else  // high half of v[q + d] and low half of v[q + d + 1]
            w[d] = __builtin_amdgcn_alignbyte(v[q + d + 1], v[q + d], 2);
    }
    return __builtin_bit_cast(bf16x8, w);
}

// The same for a tap known after unrolling (the switch folds away).
__device__ __forceinline__ bf16x8 window8_at(int s, const u32x4 &lo, const u32x4 &hi) {
    switch (s) {
    case 0: return window8<0>(lo, hi);
    case 1: return window8<1>(lo, hi);
    case 2: return window8<2>(lo, hi);
    case 3: return window8<3>(lo, hi);
    case 4: return window8<4>(lo, hi);
    case 5: return window8<5>(lo, hi);
    case 6: return window8<6>(lo, hi);
    case 7: return window8<7>(lo, hi);
    default: return window8<8>(lo, hi);
    }
}

// (ci tile, tap) column tiles p = 9 c + tap of half H: [H NH, min(NP, (H + 1) NH)).
template <int CT>
struct BwdPairs {
    static constexpr int NP = CT * kTaps;
    static constexpr int NH = (NP + 1) / 2;
};

// One 32-position step of half H: the G fragment against every column tile
// of the half (and the bias for half 0).
template <int CT, int H, int kRow>
__device__ __forceinline__ void bwd_w_step(const bf16x8 &afrag, const __bf16 (*s_x)[kRow], int q, int l,
                                           f32x4 (&acc)[BwdPairs<CT>::NH]) {
    constexpr int NP = BwdPairs<CT>::NP, NH = BwdPairs<CT>::NH;
    constexpr int P0 = H * NH, P1 = (P0 + NH < NP) ? P0 + NH : NP;
    constexpr int C0 = P0 / kTaps, C1 = (P1 - 1) / kTaps;
    u32x4 lo[C1 - C0 + 1], hi[C1 - C0 + 1];
#pragma unroll
    for (int c = C0; c <= C1; ++c) {
        // X[p0 + q + tap - 4 + i] = s_x[ci][q + tap + i], i < 8, tap < 9
        const __bf16 *row = &s_x[16 * c + (l % 16)][q];
        lo[c - C0] = *reinterpret_cast<const u32x4 *>(row);
        hi[c - C0] = *reinterpret_cast<const u32x4 *>(row + 8);
    }
#pragma unroll
    for (int p = P0; p < P1; ++p)
        acc[p - P0] = mfma16(afrag, window8_at(p % kTaps, lo[p / kTaps - C0], hi[p / kTaps - C0]), acc[p - P0]);
}

template <int CT, bool kPartial>
__global__ void __launch_bounds__(kBwdThreads) __attribute__((amdgpu_waves_per_eu(2))) conv_bwd_w_kernel(
    const __bf16 *__restrict__ g, const __bf16 *__restrict__ x, int32_t L, int32_t k32, int32_t chunks_per_wg,
    float *__restrict__ dw, float *__restrict__ db, float *__restrict__ part) {
    constexpr int cin = 16 * CT;
    constexpr int NH = BwdPairs<CT>::NH, NP = BwdPairs<CT>::NP;
    // rows of 264 elements (528 bytes, 16 bytes past a multiple of 256): the
    // 16 rows one MFMA fragment read touches start on distinct bank groups
    constexpr int kRow = kPosChunk + 2 * kHalo;
    static_assert(kRow % 8 == 0 && kPosChunk % 8 == 0, "8-position blocks");
    __shared__ __attribute__((aligned(16))) __bf16 s_g[kWidth][kRow];  // 33 KB
    __shared__ __attribute__((aligned(16))) __bf16 s_x[cin][kRow];     // <= 33 KB
    const int l = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int half = wave >> 2;  // wave-uniform
    const int64_t b = blockIdx.y;
    const __bf16 *gb = g + b * (int64_t)L * kWidth;
    const __bf16 *xb = x + b * (int64_t)L * cin;
    f32x4 acc[NH];
#pragma unroll
    for (int p = 0; p < NH; ++p) acc[p] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 acc_b = {0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones[i] = (__bf16)1.0f;
    const int co = 16 * (wave & 3) + (l % 16);
    for (int32_t ch = 0; ch < chunks_per_wg; ++ch) {
        const int32_t p0 = (blockIdx.x * chunks_per_wg + ch) * kPosChunk;
        if (p0 >= L) break;  // uniform over the workgroup
        __syncthreads();     // the previous chunk's reads are done
        // transposing copies in 8 x 8 blocks: a thread loads 8 consecutive
        // positions of 8 channels (eight 16-byte loads, from clamped and
        // always valid positions, zeroed afterwards when outside [0, L)),
        // transposes them in registers and writes 8 channel rows of 8
        // positions with 16-byte LDS stores
        for (int i = threadIdx.x; i < (kWidth / 8) * (kPosChunk / 8); i += kBwdThreads) {
            const int c8 = 8 * (i / (kPosChunk / 8)), pg = 8 * (i % (kPosChunk / 8));
            bf16x8 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = load8(gb + (int64_t)min(p0 + pg + q, L - 1) * kWidth + c8);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (p0 + pg + q >= L) v[q] = zero8();
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                bf16x8 r;
#pragma unroll
                for (int q = 0; q < 8; ++q) r[q] = v[q][j];
                *reinterpret_cast<bf16x8 *>(&s_g[c8 + j][pg]) = r;
            }
        }
        // s_x[ci][pp] = X[p0 + pp - kHalo], pp < kRow (= 33 blocks of 8)
        for (int i = threadIdx.x; i < (cin / 8) * (kRow / 8); i += kBwdThreads) {
            const int c8 = 8 * (i / (kRow / 8)), pg = 8 * (i % (kRow / 8));
            bf16x8 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[q] = load8(xb + (int64_t)min(max(p0 + pg + q - kHalo, 0), L - 1) * cin + c8);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int32_t src = p0 + pg + q - kHalo;
                if (src < 0 || src >= L) v[q] = zero8();
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                bf16x8 r;
#pragma unroll
                for (int q = 0; q < 8; ++q) r[q] = v[q][j];
                *reinterpret_cast<bf16x8 *>(&s_x[c8 + j][pg]) = r;
            }
        }
        __syncthreads();
        for (int32_t q0 = 0; q0 < kPosChunk; q0 += 32) {
            const int q = q0 + 8 * (l / 16);  // this lane's 8 positions
            const bf16x8 afrag = *reinterpret_cast<const bf16x8 *>(&s_g[co][q]);
            if (half == 0) {
                acc_b = mfma16(afrag, ones, acc_b);
                bwd_w_step<CT, 0, kRow>(afrag, s_x, q, l, acc);
            } else {
                bwd_w_step<CT, 1, kRow>(afrag, s_x, q, l, acc);
            }
        }
    }
    // C layout: lane holds rows 4 (l / 16) + r of the tile, column l % 16
    const int p_base = half * NH;
    float *slab = kPartial ? part + (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * (kWidth * k32 + kWidth)
                           : nullptr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * (wave & 3) + 4 * (l / 16) + r;
        if (half == 0 && l % 16 == 0) {
            if (kPartial)
                slab[kWidth * k32 + row] = acc_b[r];
            else
                atomicAdd(&db[row], acc_b[r]);
        }
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const int p = p_base + k;
            if (p >= NP) continue;
            const int32_t o = row * k32 + (p % kTaps) * cin + 16 * (p / kTaps) + (l % 16);
            if (kPartial)
                slab[o] = acc[k][r];
            else
                atomicAdd(&dw[o], acc[k][r]);
        }
    }
}

// dW[o] += sum over slabs of part[s][o] for the columns below n_col = 9 cin
// (a slab's padding columns are never written) and db[co] += sum of
// part[s][64 k32 + co].  A workgroup takes 256 consecutive outputs, four per
// lane (16-byte loads); wave w sums slabs w, w + 8, w + 16, ... in order and
// wave 0 adds the eight wave sums in order, so the result does not depend
// on timing.
constexpr int kRedWaves = 8;

__global__ void __launch_bounds__(64 * kRedWaves) conv_bwd_w_reduce_kernel(const float *__restrict__ part,
                                                                            int32_t n_slabs, int32_t k32,
                                                                            int32_t n_col, float *__restrict__ dw,
                                                                            float *__restrict__ db) {
    __shared__ float s_sum[kRedWaves][4][64];
    const int32_t slab = kWidth * k32 + kWidth;  // a multiple of 4
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t o4 = (blockIdx.x * 64 + lane) * 4;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (o4 < slab) {
#pragma unroll 8
        for (int32_t i = wave; i < n_slabs; i += kRedWaves) {
            const float4 v = *reinterpret_cast<const float4 *>(part + (int64_t)i * slab + o4);
            a0 += v.x;
            a1 += v.y;
            a2 += v.z;
            a3 += v.w;
        }
    }
    s_sum[wave][0][lane] = a0;
    s_sum[wave][1][lane] = a1;
    s_sum[wave][2][lane] = a2;
    s_sum[wave][3][lane] = a3;
    __syncthreads();
    if (wave != 0 || o4 >= slab) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float t = s_sum[0][j][lane];
#pragma unroll
        for (int w = 1; w < kRedWaves; ++w) t += s_sum[w][j][lane];
        const int32_t o = o4 + j;
        if (o < kWidth * k32) {
            if (o % k32 < n_col) dw[o] += t;
        } else {
            db[o - kWidth * k32] += t;
        }
    }
}

// Chunks of 256 positions per weight-gradient workgroup.  With partial
// slabs: the most (8, 4, 2 or 1) that still give one workgroup per CU of
// the 256; with atomics: 8 (each workgroup adds its sums once).
int bwd_chunks_per_wg(int32_t L, int32_t batch, bool partial) {
    if (!partial) return kChunksPerWg;
    for (int c = kChunksPerWg; c > 1; c /= 2)
        if (cetra::ceil_div(L, kPosChunk * c) * (int64_t)batch >= 256) return c;
    return 1;
}

int64_t bwd_partial_floats(int32_t cin, int32_t L, int32_t batch) {
    const int64_t k32 = ((kTaps * cin + 31) / 32) * 32;
    const int64_t n_wg = cetra::ceil_div(L, kPosChunk * bwd_chunks_per_wg(L, batch, true)) * (int64_t)batch;
    return n_wg * (kWidth * k32 + kWidth);
}

}  // namespace

using namespace cetra;

extern "C" int cetra_net_mfma_probe(void *stream, const void *a, const void *b, float *c) {
    clear_error();
    CETRA_REQUIRE(a && b && c, "net_mfma_probe: NULL pointer");
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, as_stream(stream), (const __bf16 *)a,
                       (const __bf16 *)b, c);
    return check_launch("net_mfma_probe");
}

extern "C" int cetra_net_downsample(void *stream, const float *fold, int32_t n_dur, int64_t n_t0, int32_t n_bins,
                                    void *x) {
    clear_error();
    CETRA_REQUIRE(fold && x, "net_downsample: NULL pointer");
    CETRA_REQUIRE(n_dur >= 1 && n_t0 >= 1 && n_bins >= 1 && n_bins <= n_t0, "net_downsample: bad sizes");
    const int64_t n = (int64_t)n_dur * n_bins;
    hipLaunchKernelGGL(downsample_kernel, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, as_stream(stream),
                       reinterpret_cast<const float2 *>(fold), n_dur, n_t0, n_bins, (__bf16 *)x);
    return check_launch("net_downsample");
}

extern "C" int cetra_net_downsample_signed(void *stream, const float *fold, int32_t n_dur, int64_t n_t0,
                                           int32_t n_bins, void *x) {
    clear_error();
    CETRA_REQUIRE(fold && x, "net_downsample_signed: NULL pointer");
    CETRA_REQUIRE(n_dur >= 1 && n_t0 >= 1 && n_bins >= 1 && n_bins <= n_t0, "net_downsample_signed: bad sizes");
    const int64_t n = (int64_t)n_dur * n_bins;
    hipLaunchKernelGGL(downsample_signed_kernel, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, as_stream(stream),
                       reinterpret_cast<const float2 *>(fold), n_dur, n_t0, n_bins, (__bf16 *)x);
    return check_launch("net_downsample_signed");
}

static int conv_args_ok(int32_t cin, int32_t L, int32_t batch, int32_t k32) {
    CETRA_REQUIRE(cin == 16 || cin == 64, "conv: cin must be 16 or 64");
    CETRA_REQUIRE(L >= 1 && batch >= 1, "conv: bad sizes");
    CETRA_REQUIRE(k32 == ((kTaps * cin + 31) / 32) * 32, "conv: k32 must be 9*cin rounded up to 32");
    return CETRA_OK;
}

extern "C" int cetra_conv1d_fwd(void *stream, const void *x, int32_t cin, int32_t L, int32_t batch, const void *w,
                                int32_t k32, const float *bias, void *y) {
    clear_error();
    CETRA_REQUIRE(x && w && bias && y, "conv1d_fwd: NULL pointer");
    int rc = conv_args_ok(cin, L, batch, k32);
    if (rc) return rc;
    const dim3 gf((unsigned)ceil_div(L, kConvPos), (unsigned)batch);
    if (cin == 16)
        hipLaunchKernelGGL(conv_fwd_kernel<16>, gf, dim3(kConvThreads), 0, as_stream(stream), (const __bf16 *)x, L,
                           (const __bf16 *)w, bias, (__bf16 *)y);
    else
        hipLaunchKernelGGL(conv_fwd_kernel<64>, gf, dim3(kConvThreads), 0, as_stream(stream), (const __bf16 *)x, L,
                           (const __bf16 *)w, bias, (__bf16 *)y);
    return check_launch("conv1d_fwd");
}

extern "C" int64_t cetra_conv1d_bwd_partial_floats(int32_t cin, int32_t L, int32_t batch) {
    clear_error();
    if ((cin != 16 && cin != 64) || L < 1 || batch < 1) return -1;
    return bwd_partial_floats(cin, L, batch);
}

extern "C" int cetra_conv1d_bwd(void *stream, const float *dy, const void *y, const void *x, int32_t cin, int32_t L,
                                int32_t batch, const void *w, int32_t k32, void *g_scratch, void *wt_scratch,
                                float *dw_partial, int64_t dw_partial_floats, float *dx, float *dw, float *db) {
    clear_error();
    CETRA_REQUIRE(dy && y && x && w && g_scratch && wt_scratch && dw && db, "conv1d_bwd: NULL pointer");
    int rc = conv_args_ok(cin, L, batch, k32);
    if (rc) return rc;
    CETRA_REQUIRE(((uintptr_t)dw_partial & 15) == 0, "conv1d_bwd: dw_partial must be 16-byte aligned");
    CETRA_REQUIRE(!dw_partial || dw_partial_floats >= bwd_partial_floats(cin, L, batch),
                  "conv1d_bwd: dw_partial smaller than cetra_conv1d_bwd_partial_floats");
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)batch * L * kWidth;  // a multiple of 64
    if ((((uintptr_t)dy & 31) | ((uintptr_t)y & 15) | ((uintptr_t)g_scratch & 15)) == 0)
        hipLaunchKernelGGL(relu_mask8_kernel, dim3((unsigned)ceil_div(n / 8, kT)), dim3(kT), 0, s, dy,
                           (const __bf16 *)y, n / 8, (__bf16 *)g_scratch);
    else
        hipLaunchKernelGGL(relu_mask_kernel, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, dy, (const __bf16 *)y,
                           n, (__bf16 *)g_scratch);
    if ((rc = check_launch("conv1d_bwd/mask"))) return rc;
    const bool partial = dw_partial != nullptr;
    const int cpw = bwd_chunks_per_wg(L, batch, partial);
    const dim3 gw((unsigned)ceil_div(L, kPosChunk * cpw), (unsigned)batch);
    const __bf16 *gs = (const __bf16 *)g_scratch, *xs = (const __bf16 *)x;
    if (cin == 16 && partial)
        hipLaunchKernelGGL((conv_bwd_w_kernel<1, true>), gw, dim3(kBwdThreads), 0, s, gs, xs, L, k32, cpw, dw, db,
                           dw_partial);
    else if (cin == 16)
        hipLaunchKernelGGL((conv_bwd_w_kernel<1, false>), gw, dim3(kBwdThreads), 0, s, gs, xs, L, k32, cpw, dw, db,
                           nullptr);
    else if (partial)
        hipLaunchKernelGGL((conv_bwd_w_kernel<4, true>), gw, dim3(kBwdThreads), 0, s, gs, xs, L, k32, cpw, dw, db,
                           dw_partial);
    else
        hipLaunchKernelGGL((conv_bwd_w_kernel<4, false>), gw, dim3(kBwdThreads), 0, s, gs, xs, L, k32, cpw, dw, db,
                           nullptr);
    if ((rc = check_launch("conv1d_bwd/w"))) return rc;
    if (partial) {
        const int32_t slab = kWidth * k32 + kWidth;
        hipLaunchKernelGGL(conv_bwd_w_reduce_kernel, dim3((unsigned)ceil_div(slab, 256)), dim3(64 * kRedWaves), 0, s,
                           dw_partial, (int32_t)(gw.x * gw.y), k32, kTaps * cin, dw, db);
        if ((rc = check_launch("conv1d_bwd/w_reduce"))) return rc;
    }
    if (!dx) return CETRA_OK;
    hipLaunchKernelGGL(conv_transpose_w_kernel, dim3((unsigned)ceil_div(kWidth * kTaps * cin, kT)), dim3(kT), 0, s,
                       (const __bf16 *)w, cin, k32, (__bf16 *)wt_scratch);
    if ((rc = check_launch("conv1d_bwd/transpose"))) return rc;
    const dim3 gx((unsigned)ceil_div(L, kConvPos), (unsigned)batch);
    if (cin == 16)
        hipLaunchKernelGGL(conv_bwd_x_kernel<1>, gx, dim3(kConvThreads), 0, s, (const __bf16 *)g_scratch, L,
                           (const __bf16 *)wt_scratch, dx);
    else
        hipLaunchKernelGGL(conv_bwd_x_kernel<4>, gx, dim3(kConvThreads), 0, s, (const __bf16 *)g_scratch, L,
                           (const __bf16 *)wt_scratch, dx);
    return check_launch("conv1d_bwd/x");
}
