// mlp.hip -- the learned warm start (not in the paper): a 3-layer perceptron
// theta -> relu(W1 theta + b1) -> relu(W2 h1 + b2) -> W3 h2 + b3 whose output is
// the starting point (x0, y0) and log omega0 of a solve.  Weights and GEMM
// operands are BF16; products accumulate in FP32 on the matrix cores
// (v_mfma_f32_32x32x16_bf16); master weights, biases, activations before
// rounding, the loss and the Adam moments are FP32.
//
// GEMM: C[M x N] = op(A) op(B) (+ bias[n]) (relu), A and B BF16, C FP32 and/or
// BF16.  op(A)(m, k) = a[m lda + k] (ta = 0) or a[k lda + m] (ta = 1); op(B)(k, n)
// = b[k ldb + n] (tb = 0) or b[n ldb + k] (tb = 1).  A workgroup of 4 wavefronts
// owns a 128 x 128 tile of C, each wavefront a 64 x 64 quarter (2 x 2 blocks of
// 32 x 32 on the matrix cores); K advances through LDS, where each row of A and
// each column of B keeps its k-values contiguous so a lane reads its 8
// operands in one 16-byte access.  When both operands are read along k with
// aligned rows (the forward pass), K advances by 64 and the next slab's global
// loads overlap the current slab's MFMAs (gemm_bf16_pipe_kernel); the other
// transpose combinations advance by 32, staging and computing in turn.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "device_common.hpp"
#include <algorithm>

namespace pdcs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}
// round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

constexpr int kTile = 128, kKStep = 32, kLdsK = 40;   // LDS row: 32 k-values + 8 padding

// Stages op(X)[r0 .. r0+127][k0 .. k0+31] into S[r][k] (zero outside), where X
// is read along k (KCONT: x[r ld + k], 16-byte vectors when VEC) or along r
// (x[k ld + r]).
template <bool KCONT, bool VEC>
__device__ __forceinline__ void stage(uint16_t (*S)[kLdsK], const uint16_t *__restrict__ x,
                                      int64_t ld, int64_t R, int64_t K, int64_t r0, int64_t k0) {
    const int t = threadIdx.x;
    if (KCONT && VEC) {
        for (int e = t; e < kTile * (kKStep / 8); e += 256) {
            const int r = e / (kKStep / 8), c = (e % (kKStep / 8)) * 8;
            const int64_t gr = r0 + r, gk = k0 + c;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gr < R && gk + 7 < K) {
                v = *reinterpret_cast<const uint4 *>(x + gr * ld + gk);
            } else if (gr < R) {   // the ragged end of k
                uint32_t q[4];
                for (int j = 0; j < 4; ++j) {
                    const uint32_t lo = gk + 2 * j < K ? x[gr * ld + gk + 2 * j] : 0;
                    const uint32_t hi = gk + 2 * j + 1 < K ? x[gr * ld + gk + 2 * j + 1] : 0;
                    q[j] = lo | (hi << 16);
                }
                v = make_uint4(q[0], q[1], q[2], q[3]);
            }
            *reinterpret_cast<uint4 *>(&S[r][c]) = v;
        }
    } else {
        for (int e = t; e < kTile * kKStep; e += 256) {
            int r, kk;
            if (KCONT) r = e / kKStep, kk = e % kKStep;   // consecutive threads walk k
            else kk = e / kTile, r = e % kTile;           // consecutive threads walk r
            const int64_t gr = r0 + r, gk = k0 + kk;
            uint16_t v = 0;
            if (gr < R && gk < K) v = KCONT ? x[gr * ld + gk] : x[gk * ld + gr];
            S[r][kk] = v;
        }
    }
}

template <int TA, int TB, bool VA, bool VB>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int64_t M, int64_t N, int64_t K,
                                                        const uint16_t *__restrict__ a, int64_t lda,
                                                        const uint16_t *__restrict__ b, int64_t ldb,
                                                        const float *__restrict__ bias, int relu,
                                                        float *__restrict__ c32,
                                                        uint16_t *__restrict__ c16, int64_t ldc) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kTile][kLdsK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTile][kLdsK];
    const int t = threadIdx.x, lane = t % 64, w = t / 64;
    const int wm = w / 2, wn = w % 2;                 // each wavefront: 64 x 64 of the tile
    const int64_t m0 = (int64_t)blockIdx.y * kTile, n0 = (int64_t)blockIdx.x * kTile;
    f32x16 acc[2][2] = {};
    const int half = lane / 32, idx = lane % 32;
    for (int64_t k0 = 0; k0 < K; k0 += kKStep) {
        stage<TA == 0, VA>(As, a, lda, M, K, m0, k0);
        stage<TB == 1, VB>(Bs, b, ldb, N, K, n0, k0);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKStep; kk += 16) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 64 + i * 32 + idx][kk + 8 * half]);
                bv[i] = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 64 + i * 32 + idx][kk + 8 * half]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // acc[i][j][r]: row 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32 of block (i, j)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int64_t gn = n0 + wn * 64 + j * 32 + idx;
        if (gn >= N) continue;
        const float bn = bias ? bias[gn] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t gm = m0 + wm * 64 + i * 32 + 8 * (r / 4) + 4 * half + (r % 4);
                if (gm >= M) continue;
                float v = acc[i][j][r] + bn;
                if (relu && v < 0.0f) v = 0.0f;
                if (c32) c32[gm * ldc + gn] = v;
                if (c16) c16[gm * ldc + gn] = f32_to_bf16(v);
            }
    }
}

// The common case of the network (both operands read along k with 16-byte
// vectors: the forward pass and dH = dZ W), pipelined: the global loads of the
// next 64-wide k-slab go to registers while the matrix cores work on the
// current one in LDS, so the load latency overlaps the MFMAs instead of
// preceding them.  Same tile and MFMA layout as gemm_bf16_kernel.
constexpr int kKStepP = 64, kLdsKP = 72;   // LDS row: 64 k-values + 8 padding
// split K (gemm_bf16_split): only for products of at most kSplitMaxTiles output
// tiles over at least kSplitMinK (too few workgroups for a long k loop), in
// chunks of about kSplitChunk
constexpr int64_t kSplitMaxTiles = 64, kSplitMinK = 4096, kSplitChunk = 1024;

// op(X)[r0 .. r0+127][k0 .. k0+63] (X read along k, 8-aligned rows) into four
// 16-byte registers per thread, zero outside.
__device__ __forceinline__ void fetch_k64(uint4 (&r)[4], const uint16_t *__restrict__ x, int64_t ld,
                                          int64_t R, int64_t K, int64_t r0, int64_t k0) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = t + u * 256, rr = e / 8, c = (e % 8) * 8;
        const int64_t gr = r0 + rr, gk = k0 + c;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gr < R && gk + 7 < K) {
            v = *reinterpret_cast<const uint4 *>(x + gr * ld + gk);
        } else if (gr < R && gk < K) {   // the ragged end of k
            uint32_t q[4];
            for (int j = 0; j < 4; ++j) {
                const uint32_t lo = gk + 2 * j < K ? x[gr * ld + gk + 2 * j] : 0;
                const uint32_t hi = gk + 2 * j + 1 < K ? x[gr * ld + gk + 2 * j + 1] : 0;
                q[j] = lo | (hi << 16);
            }
            v = make_uint4(q[0], q[1], q[2], q[3]);
        }
        r[u] = v;
    }
}

__device__ __forceinline__ void put_k64(uint16_t (*S)[kLdsKP], const uint4 (&r)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = t + u * 256, rr = e / 8, c = (e % 8) * 8;
        *reinterpret_cast<uint4 *>(&S[rr][c]) = r[u];
    }
}

// kchunk > 0 (split K): workgroup z takes k in [z kchunk, (z + 1) kchunk) and
// writes its raw partial product to the M x N block z of c32 (no bias, ReLU
// or BF16 copy: splitk_sum_kernel adds the blocks and applies them).
__global__ __launch_bounds__(256) void gemm_bf16_pipe_kernel(int64_t M, int64_t N, int64_t K,
                                                             const uint16_t *__restrict__ a, int64_t lda,
                                                             const uint16_t *__restrict__ b, int64_t ldb,
                                                             const float *__restrict__ bias, int relu,
                                                             float *__restrict__ c32,
                                                             uint16_t *__restrict__ c16, int64_t ldc,
                                                             int64_t kchunk) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kTile][kLdsKP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTile][kLdsKP];
    if (kchunk > 0) {
        const int64_t k0 = (int64_t)blockIdx.z * kchunk;
        a += k0, b += k0;
        K = K - k0 < kchunk ? K - k0 : kchunk;
        c32 += (int64_t)blockIdx.z * M * ldc;
    }
    const int t = threadIdx.x, lane = t % 64, w = t / 64;
    const int wm = w / 2, wn = w % 2;
    const int64_t m0 = (int64_t)blockIdx.y * kTile, n0 = (int64_t)blockIdx.x * kTile;
    f32x16 acc[2][2] = {};
    const int half = lane / 32, idx = lane % 32;
    uint4 ra[4], rb[4];
    fetch_k64(ra, a, lda, M, K, m0, 0);
    fetch_k64(rb, b, ldb, N, K, n0, 0);
    for (int64_t k0 = 0; k0 < K; k0 += kKStepP) {
        put_k64(As, ra);
        put_k64(Bs, rb);
        __syncthreads();
        if (k0 + kKStepP < K) {   // the next slab's loads fly during this slab's MFMAs
            fetch_k64(ra, a, lda, M, K, m0, k0 + kKStepP);
            fetch_k64(rb, b, ldb, N, K, n0, k0 + kKStepP);
        }
#pragma unroll
        for (int kk = 0; kk < kKStepP; kk += 16) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 64 + i * 32 + idx][kk + 8 * half]);
                bv[i] = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 64 + i * 32 + idx][kk + 8 * half]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int64_t gn = n0 + wn * 64 + j * 32 + idx;
        if (gn >= N) continue;
        const float bn = bias ? bias[gn] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t gm = m0 + wm * 64 + i * 32 + 8 * (r / 4) + 4 * half + (r % 4);
                if (gm >= M) continue;
                float v = acc[i][j][r] + bn;
                if (relu && v < 0.0f) v = 0.0f;
                if (c32) c32[gm * ldc + gn] = v;
                if (c16) c16[gm * ldc + gn] = f32_to_bf16(v);
            }
    }
}

void gemm_bf16(int ta, int tb, int64_t M, int64_t N, int64_t K, const uint16_t *a, int64_t lda,
               const uint16_t *b, int64_t ldb, const float *bias, int relu, float *c32,
               uint16_t *c16, int64_t ldc, hipStream_t s) {
    if (M == 0 || N == 0) return;
    const dim3 grid((unsigned)((N + kTile - 1) / kTile), (unsigned)((M + kTile - 1) / kTile));
    // 16-byte loads along k need 8-aligned rows and a 16-byte aligned base
    const bool va = ta == 0 && lda % 8 == 0 && ((uintptr_t)a % 16) == 0;
    const bool vb = tb == 1 && ldb % 8 == 0 && ((uintptr_t)b % 16) == 0;
#define PDCS_GEMM(TA, TB, VA, VB)                                                                \
    hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, VA, VB>), grid, dim3(256), 0, s, M, N, K, a, lda, \
                       b, ldb, bias, relu, c32, c16, ldc)
    if (ta == 0 && tb == 1) {
        if (va && vb)
            hipLaunchKernelGGL(gemm_bf16_pipe_kernel, grid, dim3(256), 0, s, M, N, K, a, lda, b, ldb,
                               bias, relu, c32, c16, ldc, (int64_t)0);
        else if (va) PDCS_GEMM(0, 1, true, false);
        else if (vb) PDCS_GEMM(0, 1, false, true);
        else PDCS_GEMM(0, 1, false, false);
    } else if (ta == 0) {
        if (va) PDCS_GEMM(0, 0, true, false);
        else PDCS_GEMM(0, 0, false, false);
    } else if (tb == 1) {
        if (vb) PDCS_GEMM(1, 1, false, true);
        else PDCS_GEMM(1, 1, false, false);
    } else {
        PDCS_GEMM(1, 0, false, false);
    }
#undef PDCS_GEMM
    PDCS_HIP(hipGetLastError());
}

// The split-K blocks of gemm_bf16_split added in block order (so the result
// does not depend on scheduling), then bias, ReLU and the FP32 / BF16 stores.
__global__ void splitk_sum_kernel(const float *__restrict__ ws, int64_t S, int64_t M, int64_t N,
                                  const float *__restrict__ bias, int relu, float *__restrict__ c32,
                                  uint16_t *__restrict__ c16, int64_t ldc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    const int64_t m = i / N, n = i % N;
    float v = 0.0f;
    for (int64_t z = 0; z < S; ++z) v += ws[z * M * N + i];
    if (bias) v += bias[n];
    if (relu && v < 0.0f) v = 0.0f;
    if (c32) c32[m * ldc + n] = v;
    if (c16) c16[m * ldc + n] = f32_to_bf16(v);
}

bool gemm_bf16_split(int64_t M, int64_t N, int64_t K, const uint16_t *a, int64_t lda,
                     const uint16_t *b, int64_t ldb, const float *bias, int relu, float *c32,
                     uint16_t *c16, int64_t ldc, float *ws, int64_t ws_elems, hipStream_t s) {
    const int64_t tiles = ((M + kTile - 1) / kTile) * ((N + kTile - 1) / kTile);
    const bool vec = lda % 8 == 0 && ldb % 8 == 0 && ((uintptr_t)a % 16) == 0 && ((uintptr_t)b % 16) == 0;
    if (!ws || !vec || M < 1 || N < 1 || tiles > kSplitMaxTiles || K < kSplitMinK) return false;
    // chunks of whole 64-wide k-steps, about kSplitChunk each, as many as ws holds
    int64_t S = std::min<int64_t>((K + kSplitChunk - 1) / kSplitChunk, ws_elems / (M * N));
    if (S < 2) return false;
    const int64_t kchunk = ((K + S - 1) / S + kKStepP - 1) / kKStepP * kKStepP;
    S = (K + kchunk - 1) / kchunk;
    const dim3 grid((unsigned)((N + kTile - 1) / kTile), (unsigned)((M + kTile - 1) / kTile), (unsigned)S);
    hipLaunchKernelGGL(gemm_bf16_pipe_kernel, grid, dim3(256), 0, s, M, N, K, a, lda, b, ldb,
                       (const float *)nullptr, 0, ws, (uint16_t *)nullptr, N, kchunk);
    PDCS_HIP(hipGetLastError());
    hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, s, ws, S,
                       M, N, bias, relu, c32, c16, ldc);
    PDCS_HIP(hipGetLastError());
    return true;
}

// ------------------------------------------------ fused hidden layers
// The network's two hidden layers for a block of 32 rows (samples) in one
// launch: h1 = relu(W1 theta + b1) for all hid units of those rows (theta
// rounded to BF16 on the way in, h1 kept in LDS as BF16), then h2 = relu(W2 h1
// + b2) for 128 of the hid units, one 32 x 32 block of the matrix cores per
// wavefront.  Workgroup (x, y) takes rows 32 y .. and units 128 x ..; for the
// backward pass the workgroups with x = 0 also write theta's BF16 copy, and
// each workgroup of a row block writes its share of h1 (FP32 and BF16), so
// that no workgroup carries all of those stores.  The weights (B operands) are read straight from
// global memory with the lane layout of gemm_bf16_kernel; the products
// accumulate over k in ascending steps of 16 as in that kernel, so the
// results are the same bits as the three separate launches.
constexpr int kHidRows = 32, kHidMaxIn = 256, kHidMaxHid = 1024;
__global__ __launch_bounds__(256) void mlp_hidden_kernel(int64_t B, int in, int hid,
                                                         const float *__restrict__ theta,
                                                         const uint16_t *__restrict__ w1,
                                                         const float *__restrict__ b1,
                                                         const uint16_t *__restrict__ w2,
                                                         const float *__restrict__ b2,
                                                         uint16_t *__restrict__ xb,
                                                         float *__restrict__ h1, uint16_t *__restrict__ h1b,
                                                         float *__restrict__ h2, uint16_t *__restrict__ h2b) {
    __shared__ __attribute__((aligned(16))) uint16_t ts[kHidRows][kHidMaxIn + 8];
    __shared__ __attribute__((aligned(16))) uint16_t hs[kHidRows][kHidMaxHid + 8];
    const int t = threadIdx.x, lane = t % 64, w = t / 64;
    const int half = lane / 32, idx = lane % 32;
    const int64_t r0 = (int64_t)blockIdx.y * kHidRows;
    const bool first = blockIdx.x == 0;
    for (int e = t; e < kHidRows * in; e += 256) {   // theta rows in BF16
        const int r = e / in, k = e % in;
        const uint16_t v = r0 + r < B ? f32_to_bf16(theta[(r0 + r) * in + k]) : 0;
        ts[r][k] = v;
        if (first && r0 + r < B) xb[(r0 + r) * in + k] = v;
    }
    __syncthreads();
    // layer 1: every 32-unit block of h1, block jb on wavefront jb mod 4
    for (int jb = w; jb * 32 < hid; jb += 4) {
        f32x16 acc = {};
        const uint16_t *wr = w1 + (int64_t)(jb * 32 + idx) * in + 8 * half;
        for (int kk = 0; kk < in; kk += 16) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&ts[idx][kk + 8 * half]);
            const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(wr + kk);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        const int col = jb * 32 + idx;
        const float bn = b1[col];
        // h1 for the backward pass: each 32-unit block written by one of the
        // workgroups of this row block (block jb by workgroup jb mod gridDim.x)
        const bool mine = jb % (int)gridDim.x == (int)blockIdx.x;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r / 4) + 4 * half + (r % 4);
            float v = acc[r] + bn;
            if (v < 0.0f) v = 0.0f;
            const uint16_t v16 = f32_to_bf16(v);
            hs[row][col] = v16;
            if (mine && r0 + row < B) {
                h1[(r0 + row) * hid + col] = v;
                h1b[(r0 + row) * hid + col] = v16;
            }
        }
    }
    __syncthreads();
    // layer 2: units [128 x + 32 w, +32) of h2, eight k-steps of weights in flight
    const int cb = blockIdx.x * 4 + w;
    if (cb * 32 >= hid) return;
    f32x16 acc = {};
    const uint16_t *wr = w2 + (int64_t)(cb * 32 + idx) * hid + 8 * half;
    for (int k0 = 0; k0 < hid; k0 += 128) {
        bf16x8 bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            bv[u] = k0 + 16 * u < hid ? *reinterpret_cast<const bf16x8 *>(wr + k0 + 16 * u) : bf16x8{};
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (k0 + 16 * u >= hid) break;
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&hs[idx][k0 + 16 * u + 8 * half]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[u], acc, 0, 0, 0);
        }
    }
    const int col = cb * 32 + idx;
    const float bn = b2[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + 4 * half + (r % 4);
        if (r0 + row >= B) continue;
        float v = acc[r] + bn;
        if (v < 0.0f) v = 0.0f;
        h2[(r0 + row) * hid + col] = v;
        h2b[(r0 + row) * hid + col] = f32_to_bf16(v);
    }
}

bool mlp_hidden(int64_t B, int64_t in, int64_t hid, const float *theta, const uint16_t *w1,
                const float *b1, const uint16_t *w2, const float *b2, uint16_t *xb, float *h1,
                uint16_t *h1b, float *h2, uint16_t *h2b, hipStream_t s) {
    // shapes the fused kernel covers: whole 16-wide k-steps, 128-unit blocks of
    // h2, the LDS tiles' sizes, and 16-byte aligned weight rows
    if (B < 1 || in % 16 || in > kHidMaxIn || hid % 128 || hid > kHidMaxHid) return false;
    if ((uintptr_t)w1 % 16 || (uintptr_t)w2 % 16) return false;
    const dim3 grid((unsigned)(hid / 128), (unsigned)((B + kHidRows - 1) / kHidRows));
    hipLaunchKernelGGL(mlp_hidden_kernel, grid, dim3(256), 0, s, B, (int)in, (int)hid, theta, w1, b1,
                       w2, b2, xb, h1, h1b, h2, h2b);
    PDCS_HIP(hipGetLastError());
    return true;
}

// ------------------------------------------------------------- elementwise
__global__ void to_bf16_kernel(const float *in, uint16_t *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = f32_to_bf16(in[i]);
}
void to_bf16(const float *in, uint16_t *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
    PDCS_HIP(hipGetLastError());
}

// out[c ldo + r] = in[r ldi + c] for a rows x cols BF16 matrix, through a
// 32 x 32 LDS tile so reads and writes are both along rows
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const uint16_t *in, int64_t rows,
                                                             int64_t cols, int64_t ldi,
                                                             uint16_t *out, int64_t ldo) {
    __shared__ uint16_t tile[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        tile[k][tx] = (r < rows && c < cols) ? in[r * ldi + c] : 0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (c < cols && r < rows) out[c * ldo + r] = tile[tx][k];
    }
}
void transpose_bf16(const uint16_t *in, int64_t rows, int64_t cols, int64_t ldi, uint16_t *out,
                    int64_t ldo, hipStream_t s) {
    if (rows == 0 || cols == 0) return;
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(transpose_bf16_kernel, grid, dim3(256), 0, s, in, rows, cols, ldi, out, ldo);
    PDCS_HIP(hipGetLastError());
}

// d = (out - target) / (rows cols) for a rows x cols batch (d32 dense, d16 with
// leading dimension ld16); loss partial sums of (out - target)^2 per block
__global__ void mse_kernel(const float *out, const float *target, int64_t n, int64_t cols,
                           int64_t ld16, float inv, float *d32, uint16_t *d16, double *part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc[1] = {0.0};
    if (i < n) {
        const float r = out[i] - target[i];
        const float g = r * inv;
        d32[i] = g;
        d16[(i / cols) * ld16 + i % cols] = f32_to_bf16(g);
        acc[0] = (double)r * (double)r;
    }
    block_sum_all<1>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// dz = dh where z > 0 (the relu derivative), FP32 and BF16 copies
__global__ void relu_back_kernel(const float *dh, const float *z, int64_t n, float *dz32,
                                 uint16_t *dz16) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = z[i] > 0.0f ? dh[i] : 0.0f;
    dz32[i] = g;
    dz16[i] = f32_to_bf16(g);
}

// db[j] = sum over rows of d[r, j], rows in order
// Column sums, rows added in order; a thread issues 16 rows' loads before
// adding them, so a short, wide sum waits on few memory latencies.
__global__ void colsum_kernel(const float *d, int64_t rows, int64_t cols, float *db) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= cols) return;
    constexpr int U = 16;
    float acc = 0.0f;
    int64_t r = 0;
    for (; r + U <= rows; r += U) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = d[(r + u) * cols + j];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    for (; r < rows; ++r) acc += d[r * cols + j];
    db[j] = acc;
}

// Adam (Kingma and Ba) on FP32 master parameters, BF16 copy refreshed
__global__ void adam_kernel(float *p, const float *g, float *m1, float *m2, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2, uint16_t *p16) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a, m2[i] = v;
    const float q = p[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[i] = q;
    if (p16) p16[i] = f32_to_bf16(q);
}

void mse_grad(const float *out, const float *target, int64_t n, int64_t cols, int64_t ld16,
              float inv, float *d32, uint16_t *d16, double *part, hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, target,
                       n, cols, ld16, inv, d32, d16, part);
    PDCS_HIP(hipGetLastError());
}
void relu_back(const float *dh, const float *z, int64_t n, float *dz32, uint16_t *dz16, hipStream_t s) {
    hipLaunchKernelGGL(relu_back_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dh, z,
                       n, dz32, dz16);
    PDCS_HIP(hipGetLastError());
}
void colsum(const float *d, int64_t rows, int64_t cols, float *db, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, d, rows,
                       cols, db);
    PDCS_HIP(hipGetLastError());
}
void adam(float *p, const float *g, float *m1, float *m2, int64_t n, float lr, float b1, float b2,
          float eps, float c1, float c2, uint16_t *p16, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m1, m2,
                       n, lr, b1, b2, eps, c1, c2, p16);
    PDCS_HIP(hipGetLastError());
}

}  // namespace pdcs
