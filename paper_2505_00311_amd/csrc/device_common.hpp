// device_common.hpp -- reductions for 64-lane wavefronts and 256-thread
// workgroups.  Butterfly (xor) exchanges leave the same bits in every lane,
// since each step adds the same two operands in either order, so decisions
// taken on a reduced value are uniform across the wavefront.
#pragma once
#include "internal.hpp"

namespace pdcs {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// Sum of K values over the workgroup; every thread receives the same result.
template <int K>
__device__ __forceinline__ void block_sum_all(double (&v)[K]) {
    __shared__ double red[kBlock / kWave][K];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[w][k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = red[0][k];
#pragma unroll
        for (int i = 1; i < kBlock / kWave; ++i) s += red[i][k];
        v[k] = s;
    }
    __syncthreads();
}

// Accumulators of a pass: 3 sums and 3 maxima per thread.
struct Acc {
    double s[3] = {0.0, 0.0, 0.0};
    double mx[3] = {0.0, 0.0, 0.0};
};

// Reduces Acc over the workgroup in a fixed order; thread 0 writes
// partials[tile * kPartials + {0..5}].
__device__ __forceinline__ void write_partials(Acc &a, double *partials, int64_t tile) {
    __shared__ double red[kBlock / kWave][kPartials];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double v[kPartials];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = wave_sum(a.s[k]);
        v[3 + k] = wave_max(a.mx[k]);
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kPartials; ++k) red[w][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kPartials; ++k) {
            double r = red[0][k];
#pragma unroll
            for (int i = 1; i < kBlock / kWave; ++i) r = k < 3 ? r + red[i][k] : fmax(r, red[i][k]);
            partials[tile * kPartials + k] = r;
        }
    }
}

}  // namespace pdcs
