// spmv.hip -- y = A x for a CSR matrix in FP64, the products G x and G^T y of
// eq. (5).  Row-split CSR: a group of L lanes (a power of two dividing the
// 64-lane wavefront) owns one short row and streams its val/col entries with
// unit stride across the group, then reduces with xor exchanges.  Rows longer
// than the plan's threshold (power-law column degrees make G^T rows up to
// ~1e5 long) are cut into chunks of kLongChunk entries, one workgroup per
// chunk, and each row's chunk sums are added in chunk order, so every row's
// sum is formed in a fixed order on every run.
#include "device_common.hpp"

namespace pdcs {

template <int L>
__global__ __launch_bounds__(kBlock) void spmv_rows_kernel(int64_t rows, const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const double *__restrict__ v,
                                                           const double *__restrict__ x,
                                                           double *__restrict__ y, int64_t long_thr,
                                                           const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t row = gid / L;
    const int lane = (int)(gid % L);
    if (row >= rows) return;           // uniform within the L-lane group
    const int64_t s = rp[row], e = rp[row + 1];
    if (e - s > long_thr) return;      // long rows: chunked path
    double acc = 0.0;
    for (int64_t k = s + lane; k < e; k += L) acc += v[k] * x[ci[k]];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) y[row] = acc;
}

__global__ __launch_bounds__(kBlock) void spmv_chunks_kernel(const int64_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const double *__restrict__ v,
                                                             const double *__restrict__ x,
                                                             const int32_t *__restrict__ long_rows,
                                                             const int32_t *__restrict__ chunk_row,
                                                             const int64_t *__restrict__ chunk_begin,
                                                             double *__restrict__ part,
                                                             const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t c = blockIdx.x;
    const int64_t row = long_rows[chunk_row[c]];
    const int64_t b = chunk_begin[c];
    const int64_t e = min(b + kLongChunk, rp[row + 1]);
    double acc[1] = {0.0};
    for (int64_t k = b + threadIdx.x; k < e; k += kBlock) acc[0] += v[k] * x[ci[k]];
    block_sum_all<1>(acc);
    if (threadIdx.x == 0) part[c] = acc[0];
}

__global__ void spmv_chunks_finish(int64_t n_long, const int32_t *__restrict__ long_rows,
                                   const int64_t *__restrict__ chunk_ptr,
                                   const double *__restrict__ part, double *__restrict__ y,
                                   const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_long) return;
    double s = 0.0;
    for (int64_t c = chunk_ptr[i]; c < chunk_ptr[i + 1]; ++c) s += part[c];
    y[long_rows[i]] = s;
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
    const int64_t threads = A.rows * L;
    const int64_t blocks = (threads + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(spmv_rows_kernel<L>, dim3((unsigned)blocks), dim3(kBlock), 0, s, A.rows,
                       A.rp, A.ci, A.v, x, y, p.long_thr, skip);
}

void spmv(const Csr &A, const SpmvPlan &p, const double *x, double *y, const int *skip,
          hipStream_t s) {
    if (A.rows == 0) return;
    switch (p.lanes) {
    case 2: launch_rows<2>(A, p, x, y, skip, s); break;
    case 4: launch_rows<4>(A, p, x, y, skip, s); break;
    case 8: launch_rows<8>(A, p, x, y, skip, s); break;
    case 16: launch_rows<16>(A, p, x, y, skip, s); break;
    case 32: launch_rows<32>(A, p, x, y, skip, s); break;
    default: launch_rows<64>(A, p, x, y, skip, s); break;
    }
    PDCS_HIP(hipGetLastError());
    if (p.n_long > 0) {
        hipLaunchKernelGGL(spmv_chunks_kernel, dim3((unsigned)p.n_chunks), dim3(kBlock), 0, s, A.rp,
                           A.ci, A.v, x, p.long_rows, p.chunk_row, p.chunk_begin, p.chunk_part,
                           skip);
        hipLaunchKernelGGL(spmv_chunks_finish, dim3((unsigned)((p.n_long + 255) / 256)), dim3(256),
                           0, s, p.n_long, p.long_rows, p.long_chunk_ptr, p.chunk_part, y, skip);
        PDCS_HIP(hipGetLastError());
    }
}

}  // namespace pdcs
