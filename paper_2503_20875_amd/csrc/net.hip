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

// ------------------------------------------------------------ conv forward
// Workgroup: 64 positions x 64 output channels of one example; wave w owns
// positions [16 w, 16 w + 16) and all 64 channels (4 MFMA row tiles).
__global__ void __launch_bounds__(kT) conv_fwd_kernel(const __bf16 *__restrict__ x, int32_t cin, int32_t L,
                                                      const __bf16 *__restrict__ w, int32_t k32,
                                                      const float *__restrict__ bias, __bf16 *__restrict__ y) {
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.y;
    const int32_t t = blockIdx.x * 64 + wave * 16 + (l % 16);  // output position of this lane's B column
    const __bf16 *xb = x + b * (int64_t)L * cin;
    f32x4 acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int32_t k0 = 0; k0 < k32; k0 += 32) {
        const int32_t k = k0 + 8 * (l / 16);  // first of this lane's 8 reduction indices
        const int32_t tap = k / cin, ci = k % cin;
        const int32_t src = t + tap - 4;
        const bf16x8 bfrag = (tap < kTaps && src >= 0 && src < L && t < L) ? load8(xb + (int64_t)src * cin + ci)
                                                                            : zero8();
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const bf16x8 afrag = load8(w + (int64_t)(16 * m + (l % 16)) * k32 + k);
            acc[m] = mfma16(afrag, bfrag, acc[m]);
        }
    }
    if (t >= L) return;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = 16 * m + 4 * (l / 16) + r;
            const float v = fmaxf(acc[m][r] + bias[co], 0.0f);
            y[(b * L + t) * kWidth + co] = (__bf16)v;
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
// dX[b][t][ci] (FP32) = sum over tap, co of WT[ci][tap*64 + co] G[b][t - tap + 4][co].
// Workgroup: 64 positions of one example; wave w owns 16 positions and all
// cin input channels (cin / 16 MFMA row tiles, cin in {16, 64}).
__global__ void __launch_bounds__(kT) conv_bwd_x_kernel(const __bf16 *__restrict__ g, int32_t L,
                                                        const __bf16 *__restrict__ wt, int32_t cin,
                                                        float *__restrict__ dx) {
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.y;
    const int32_t t = blockIdx.x * 64 + wave * 16 + (l % 16);
    const __bf16 *gb = g + b * (int64_t)L * kWidth;
    const int mt = cin / 16;
    f32x4 acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    constexpr int32_t kK = kTaps * kWidth;  // 576, a multiple of 32
    for (int32_t k0 = 0; k0 < kK; k0 += 32) {
        const int32_t k = k0 + 8 * (l / 16);
        const int32_t tap = k / kWidth, co = k % kWidth;
        const int32_t src = t - tap + 4;
        const bf16x8 bfrag = (src >= 0 && src < L && t < L) ? load8(gb + (int64_t)src * kWidth + co) : zero8();
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m >= mt) break;
            const bf16x8 afrag = load8(wt + (int64_t)(16 * m + (l % 16)) * kK + k);
            acc[m] = mfma16(afrag, bfrag, acc[m]);
        }
    }
    if (t >= L) return;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (m >= mt) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) dx[(b * L + t) * cin + 16 * m + 4 * (l / 16) + r] = acc[m][r];
    }
}

// ------------------------------------------------------ conv backward-w
// dW[co][k] += sum over 256 positions of one example of G[t][co] X[t+tap-4][ci]
// (k = tap * cin + ci).  Workgroup: (8 chunks of 256 positions, example,
// block of 64 reduction columns k); each chunk of G and of X (with a
// 4-position halo) is staged in LDS transposed to position-fastest order so
// every MFMA fragment is one 16-byte LDS read.  The workgroup's partial sums
// over its 2048 positions are added to dW (FP32 atomics); db[co] gets the
// column sums of G.
constexpr int kPosChunk = 256;
constexpr int kChunksPerWg = 8;
__global__ void __launch_bounds__(kT) conv_bwd_w_kernel(const __bf16 *__restrict__ g, const __bf16 *__restrict__ x,
                                                        int32_t cin, int32_t L, int32_t k32,
                                                        float *__restrict__ dw, float *__restrict__ db) {
    __shared__ __attribute__((aligned(16))) __bf16 s_g[kWidth][kPosChunk];            // 32 KB
    __shared__ __attribute__((aligned(16))) __bf16 s_x[kWidth][kPosChunk + 16];       // 34 KB (cin <= 64)
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.y;
    const int32_t kb = blockIdx.z * 64;  // this workgroup's 64 reduction columns
    const __bf16 *gb = g + b * (int64_t)L * kWidth;
    const __bf16 *xb = x + b * (int64_t)L * cin;
    // wave w: output rows co in [16 w, 16 w + 16), columns k in [kb, kb + 64)
    // (4 tiles), accumulated over kChunksPerWg position chunks before the
    // atomics
    f32x4 acc[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bias_acc = 0.0f;
    const int co = 16 * wave + (l % 16);
    for (int32_t ch = 0; ch < kChunksPerWg; ++ch) {
        const int32_t p0 = (blockIdx.x * kChunksPerWg + ch) * kPosChunk;
        if (p0 >= L) break;  // uniform over the workgroup
        __syncthreads();     // the previous chunk's reads are done
        for (int i = threadIdx.x; i < kWidth * kPosChunk; i += kT) {
            const int p = i / kWidth, c = i % kWidth;
            s_g[c][p] = (p0 + p < L) ? gb[(int64_t)(p0 + p) * kWidth + c] : (__bf16)0.0f;
        }
        for (int i = threadIdx.x; i < cin * (kPosChunk + 16); i += kT) {
            const int p = i / cin, ci = i % cin;
            const int32_t src = p0 + p - 4;
            s_x[ci][p] = (src >= 0 && src < L) ? xb[(int64_t)src * cin + ci] : (__bf16)0.0f;
        }
        __syncthreads();
        if (blockIdx.z == 0 && wave == 0)  // bias gradient: column sums of G
            for (int p = 0; p < kPosChunk; ++p) bias_acc += (float)s_g[l][p];
        for (int32_t q0 = 0; q0 < kPosChunk; q0 += 32) {
            const int q = q0 + 8 * (l / 16);
            const bf16x8 afrag = *reinterpret_cast<const bf16x8 *>(&s_g[co][q]);
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int32_t k = kb + 16 * n + (l % 16);
                const int32_t tap = k / cin, ci = k % cin;
                bf16x8 bfrag;
                if (k < kTaps * cin) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) bfrag[i] = s_x[ci][q + i + tap];
                } else {
                    bfrag = zero8();
                }
                acc[n] = mfma16(afrag, bfrag, acc[n]);
            }
        }
    }
    if (blockIdx.z == 0 && wave == 0) atomicAdd(&db[l], bias_acc);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * wave + 4 * (l / 16) + r;
            const int32_t k = kb + 16 * n + (l % 16);
            if (k < k32) atomicAdd(&dw[row * k32 + k], acc[n][r]);
        }
    }
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
    hipLaunchKernelGGL(conv_fwd_kernel, dim3((unsigned)ceil_div(L, 64), (unsigned)batch), dim3(kT), 0,
                       as_stream(stream), (const __bf16 *)x, cin, L, (const __bf16 *)w, k32, bias, (__bf16 *)y);
    return check_launch("conv1d_fwd");
}

extern "C" int cetra_conv1d_bwd(void *stream, const float *dy, const void *y, const void *x, int32_t cin, int32_t L,
                                int32_t batch, const void *w, int32_t k32, void *g_scratch, void *wt_scratch,
                                float *dx, float *dw, float *db) {
    clear_error();
    CETRA_REQUIRE(dy && y && x && w && g_scratch && wt_scratch && dw && db, "conv1d_bwd: NULL pointer");
    int rc = conv_args_ok(cin, L, batch, k32);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)batch * L * kWidth;
    hipLaunchKernelGGL(relu_mask_kernel, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, dy, (const __bf16 *)y, n,
                       (__bf16 *)g_scratch);
    if ((rc = check_launch("conv1d_bwd/mask"))) return rc;
    hipLaunchKernelGGL(conv_bwd_w_kernel, dim3((unsigned)ceil_div(L, kPosChunk * kChunksPerWg), (unsigned)batch,
                                               (unsigned)ceil_div(kTaps * cin, 64)),
                       dim3(kT), 0, s, (const __bf16 *)g_scratch, (const __bf16 *)x, cin, L, k32, dw, db);
    if ((rc = check_launch("conv1d_bwd/w"))) return rc;
    if (!dx) return CETRA_OK;
    hipLaunchKernelGGL(conv_transpose_w_kernel, dim3((unsigned)ceil_div(kWidth * kTaps * cin, kT)), dim3(kT), 0, s,
                       (const __bf16 *)w, cin, k32, (__bf16 *)wt_scratch);
    if ((rc = check_launch("conv1d_bwd/transpose"))) return rc;
    hipLaunchKernelGGL(conv_bwd_x_kernel, dim3((unsigned)ceil_div(L, 64), (unsigned)batch), dim3(kT), 0, s,
                       (const __bf16 *)g_scratch, L, (const __bf16 *)wt_scratch, cin, dx);
    return check_launch("conv1d_bwd/x");
}
