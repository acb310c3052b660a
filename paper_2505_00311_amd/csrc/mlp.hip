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
// owns a 64 x 64 tile of C, each wavefront a 32 x 32 block; K advances by 16
// through LDS, where each row of A and each column of B keeps its 16 k-values
// contiguous so a lane reads its 8 operands in one 16-byte access.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "device_common.hpp"

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

constexpr int kTile = 64, kKStep = 16, kLdsK = 24;   // LDS row: 16 k-values + 8 padding

template <int TA, int TB>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int64_t M, int64_t N, int64_t K,
                                                        const uint16_t *__restrict__ a, int64_t lda,
                                                        const uint16_t *__restrict__ b, int64_t ldb,
                                                        const float *__restrict__ bias, int relu,
                                                        float *__restrict__ c32,
                                                        uint16_t *__restrict__ c16, int64_t ldc) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kTile][kLdsK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTile][kLdsK];
    const int t = threadIdx.x, lane = t % 64, w = t / 64;
    const int wm = w / 2, wn = w % 2;
    const int64_t m0 = (int64_t)blockIdx.y * kTile, n0 = (int64_t)blockIdx.x * kTile;
    f32x16 acc = {};
    for (int64_t k0 = 0; k0 < K; k0 += kKStep) {
        // stage op(A)[m0 .. m0+63][k0 .. k0+15] and op(B)[k0 ..][n0 .. n0+63], zero outside
        for (int e = t; e < kTile * kKStep; e += 256) {
            int r, kk;
            if (TA == 0) r = e / kKStep, kk = e % kKStep;   // consecutive threads walk k
            else kk = e / kTile, r = e % kTile;             // consecutive threads walk m
            const int64_t gm = m0 + r, gk = k0 + kk;
            uint16_t v = 0;
            if (gm < M && gk < K) v = TA == 0 ? a[gm * lda + gk] : a[gk * lda + gm];
            As[r][kk] = v;
        }
        for (int e = t; e < kTile * kKStep; e += 256) {
            int cidx, kk;
            if (TB == 1) cidx = e / kKStep, kk = e % kKStep;
            else kk = e / kTile, cidx = e % kTile;
            const int64_t gn = n0 + cidx, gk = k0 + kk;
            uint16_t v = 0;
            if (gn < N && gk < K) v = TB == 1 ? b[gn * ldb + gk] : b[gk * ldb + gn];
            Bs[cidx][kk] = v;
        }
        __syncthreads();
        const int half = lane / 32, idx = lane % 32;
        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + idx][8 * half]);
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 32 + idx][8 * half]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        __syncthreads();
    }
    // acc[r]: row 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32 of the block
    const int64_t gn = n0 + wn * 32 + lane % 32;
    if (gn >= N) return;
    const float bn = bias ? bias[gn] : 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t gm = m0 + wm * 32 + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        if (gm >= M) continue;
        float v = acc[r] + bn;
        if (relu && v < 0.0f) v = 0.0f;
        if (c32) c32[gm * ldc + gn] = v;
        if (c16) c16[gm * ldc + gn] = f32_to_bf16(v);
    }
}

void gemm_bf16(int ta, int tb, int64_t M, int64_t N, int64_t K, const uint16_t *a, int64_t lda,
               const uint16_t *b, int64_t ldb, const float *bias, int relu, float *c32,
               uint16_t *c16, int64_t ldc, hipStream_t s) {
    if (M == 0 || N == 0) return;
    const dim3 grid((unsigned)((N + kTile - 1) / kTile), (unsigned)((M + kTile - 1) / kTile));
#define PDCS_GEMM(TA, TB)                                                                        \
    hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB>), grid, dim3(256), 0, s, M, N, K, a, lda, b, ldb, \
                       bias, relu, c32, c16, ldc)
    if (ta == 0 && tb == 0) PDCS_GEMM(0, 0);
    else if (ta == 0) PDCS_GEMM(0, 1);
    else if (tb == 0) PDCS_GEMM(1, 0);
    else PDCS_GEMM(1, 1);
#undef PDCS_GEMM
    PDCS_HIP(hipGetLastError());
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

// d = (out - target) / (rows cols); loss partial sums of (out - target)^2 per block
__global__ void mse_kernel(const float *out, const float *target, int64_t n, float inv,
                           float *d32, uint16_t *d16, double *part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc[1] = {0.0};
    if (i < n) {
        const float r = out[i] - target[i];
        const float g = r * inv;
        d32[i] = g;
        d16[i] = f32_to_bf16(g);
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
__global__ void colsum_kernel(const float *d, int64_t rows, int64_t cols, float *db) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= cols) return;
    float acc = 0.0f;
    for (int64_t r = 0; r < rows; ++r) acc += d[r * cols + j];
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

void mse_grad(const float *out, const float *target, int64_t n, float inv, float *d32, uint16_t *d16,
              double *part, hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, target,
                       n, inv, d32, d16, part);
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
