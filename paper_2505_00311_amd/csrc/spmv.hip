// spmv.hip -- y = A x for a CSR matrix in FP64, the products G x and G^T y of
// eq. (5).  Row-split CSR: a group of L lanes (a power of two dividing the
// 64-lane wavefront) owns one short row and streams its val/col entries with
// unit stride across the group, then reduces with xor exchanges; matrices whose
// rows average fewer than 12 entries (G^T here) use a CSR-stream kernel that
// streams whole row ranges through LDS instead, so no lane idles on a short
// row.  Rows longer
// than the plan's threshold (power-law column degrees make G^T rows up to
// ~1e5 long) are cut into chunks of kLongChunk entries, one workgroup per
// chunk, and each row's chunk sums are added in chunk order, so every row's
// sum is formed in a fixed order on every run.
#include "device_common.hpp"

namespace pdcs {

// One chunk of a long row: its sum goes to chunk_part[c]; a second kernel adds
// each row's chunk sums in chunk order (a kernel boundary orders the writes).
__device__ __forceinline__ void long_chunk(int64_t c, const int64_t *__restrict__ rp,
                                           const int32_t *__restrict__ ci,
                                           const double *__restrict__ v,
                                           const double *__restrict__ x, const SpmvPlan &p) {
    const int64_t row = p.long_rows[p.chunk_row[c]];
    const int64_t b = p.chunk_begin[c];
    const int64_t e = min(b + kLongChunk, rp[row + 1]);
    double acc[1] = {0.0};
    for (int64_t k = b + threadIdx.x; k < e; k += kBlock) acc[0] += v[k] * x[ci[k]];
    block_sum_all<1>(acc);
    if (threadIdx.x == 0) p.chunk_part[c] = acc[0];
}

__global__ void spmv_chunks_finish(SpmvPlan p, double *__restrict__ y, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_long) return;
    double s = 0.0;
    for (int64_t c = p.long_chunk_ptr[i]; c < p.long_chunk_ptr[i + 1]; ++c) s += p.chunk_part[c];
    y[p.long_rows[i]] = s;
}

// Workgroups [0, n_chunks) take the long-row chunks, the rest the short rows:
// a group of L lanes per row.
template <int L>
__global__ __launch_bounds__(kBlock) void spmv_rows_kernel(int64_t rows, const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const double *__restrict__ v,
                                                           const double *__restrict__ x,
                                                           double *__restrict__ y, SpmvPlan p,
                                                           const int *__restrict__ skip) {
    if (skip && *skip) return;
    if ((int64_t)blockIdx.x < p.n_chunks) {
        long_chunk(blockIdx.x, rp, ci, v, x, p);
        return;
    }
    const int64_t gid = ((int64_t)blockIdx.x - p.n_chunks) * kBlock + threadIdx.x;
    const int64_t row = gid / L;
    const int lane = (int)(gid % L);
    if (row >= rows) return;           // uniform within the L-lane group
    const int64_t s = rp[row], e = rp[row + 1];
    if (e - s > p.long_thr) return;    // long rows: chunks above
    double acc = 0.0;
    for (int64_t k = s + lane; k < e; k += L) acc += v[k] * x[ci[k]];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) y[row] = acc;
}

// CSR-stream: after the chunk workgroups, workgroup b owns the rows
// [sb[2b], sb[2b+1]) whose entries (at most kStreamNnz, long rows excluded by the
// plan) it streams with unit stride into LDS as products, then one thread per
// row adds its segment in order.
__global__ __launch_bounds__(kBlock) void spmv_stream_kernel(const int64_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const double *__restrict__ v,
                                                             const double *__restrict__ x,
                                                             double *__restrict__ y, SpmvPlan p,
                                                             const int *__restrict__ skip) {
    if (skip && *skip) return;
    if ((int64_t)blockIdx.x < p.n_chunks) {
        long_chunk(blockIdx.x, rp, ci, v, x, p);
        return;
    }
    __shared__ double prod[kStreamNnz];
    const int64_t bb = (int64_t)blockIdx.x - p.n_chunks;
    const int64_t r0 = p.sblock[2 * bb], r1 = p.sblock[2 * bb + 1];
    const int64_t k0 = rp[r0];
    const int cnt = (int)(rp[r1] - k0);
    for (int i = threadIdx.x; i < cnt; i += kBlock) prod[i] = v[k0 + i] * x[ci[k0 + i]];
    __syncthreads();
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        const int a = (int)(rp[r] - k0), b = (int)(rp[r + 1] - k0);
        double acc = 0.0;
        for (int i = a; i < b; ++i) acc += prod[i];
        y[r] = acc;
    }
}

// smallest power of two >= half the mean row length, within [2, 64]
int choose_lanes(double avg) {
    int L = 2;
    while (L < 64 && 2.0 * L < avg) L <<= 1;
    return L;
}

template <int L>
static void launch_rows(const Csr &A, const SpmvPlan &p, const double *x, double *y,
                        const int *skip, hipStream_t s) {
    const int64_t blocks = (A.rows * L + kBlock - 1) / kBlock + p.n_chunks;
    hipLaunchKernelGGL(spmv_rows_kernel<L>, dim3((unsigned)blocks), dim3(kBlock), 0, s, A.rows,
                       A.rp, A.ci, A.v, x, y, p, skip);
}

void spmv(const Csr &A, const SpmvPlan &p, const double *x, double *y, const int *skip,
          hipStream_t s) {
    if (A.rows == 0) return;
    if (p.stream) {
        const int64_t blocks = p.n_sblocks + p.n_chunks;
        if (blocks > 0)
            hipLaunchKernelGGL(spmv_stream_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, A.rp,
                               A.ci, A.v, x, y, p, skip);
    } else {
        switch (p.lanes) {
        case 2: launch_rows<2>(A, p, x, y, skip, s); break;
        case 4: launch_rows<4>(A, p, x, y, skip, s); break;
        case 8: launch_rows<8>(A, p, x, y, skip, s); break;
        case 16: launch_rows<16>(A, p, x, y, skip, s); break;
        case 32: launch_rows<32>(A, p, x, y, skip, s); break;
        default: launch_rows<64>(A, p, x, y, skip, s); break;
        }
    }
    if (p.n_long > 0)
        hipLaunchKernelGGL(spmv_chunks_finish, dim3((unsigned)((p.n_long + 255) / 256)), dim3(256),
                           0, s, p, y, skip);
    PDCS_HIP(hipGetLastError());
}

}  // namespace pdcs
