// spmv.hip -- y = A x for a CSR matrix, the products G x and G^T y of eq. (5).
// Values and the gathered x are FP64, or FP32 in the mixed-precision form;
// products and sums are always formed in FP64 (a product of two FP32 numbers
// is exact in FP64), so the FP32 form's only error is the rounding of its
// inputs.  Row-split CSR: a group of L lanes (a power of two dividing the
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

// Whether the instance of `row` has the skip flag set (see SpmvSkip).
__device__ __forceinline__ bool row_skipped(const SpmvSkip &k, int64_t row) {
    if (k.flag == SkipNone) return false;
    const DevState &s = k.st[inst_of(k.row_inst, row)];
    return k.flag == SkipHalt ? s.halt != 0 : s.skip_update != 0;
}

// One chunk of a long row: its sum goes to chunk_part[c]; a second kernel adds
// each row's chunk sums in chunk order (a kernel boundary orders the writes).
template <class T>
__device__ __forceinline__ void long_chunk(int64_t c, const int64_t *__restrict__ rp,
                                           const int32_t *__restrict__ ci,
                                           const T *__restrict__ v,
                                           const T *__restrict__ x, const SpmvPlan &p) {
    const int64_t row = p.long_rows[p.chunk_row[c]];
    const int64_t b = p.chunk_begin[c];
    const int64_t e = min(b + kLongChunk, rp[row + 1]);
    double acc[1] = {0.0};
    for (int64_t k = b + threadIdx.x; k < e; k += kBlock) acc[0] += (double)v[k] * (double)x[ci[k]];
    block_sum_all<1>(acc);
    if (threadIdx.x == 0) p.chunk_part[c] = acc[0];
}

__global__ void spmv_chunks_finish(SpmvPlan p, double *__restrict__ y, SpmvSkip skip) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_long || row_skipped(skip, p.long_rows[i])) return;
    double s = 0.0;
    for (int64_t c = p.long_chunk_ptr[i]; c < p.long_chunk_ptr[i + 1]; ++c) s += p.chunk_part[c];
    y[p.long_rows[i]] = s;
}

// Workgroups [0, n_chunks) take the long-row chunks, the rest the short rows:
// a group of L lanes per row.
template <int L, class T>
__global__ __launch_bounds__(kBlock) void spmv_rows_kernel(int64_t rows, const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const T *__restrict__ v,
                                                           const T *__restrict__ x,
                                                           double *__restrict__ y, SpmvPlan p,
                                                           SpmvSkip skip) {
    if (!skip.row_inst && row_skipped(skip, 0)) return;   // one problem: one flag
    if ((int64_t)blockIdx.x < p.n_chunks) {
        if (!row_skipped(skip, p.long_rows[p.chunk_row[blockIdx.x]]))
            long_chunk(blockIdx.x, rp, ci, v, x, p);
        return;
    }
    const int64_t gid = ((int64_t)blockIdx.x - p.n_chunks) * kBlock + threadIdx.x;
    const int64_t row = gid / L;
    const int lane = (int)(gid % L);
    if (row >= rows) return;           // uniform within the L-lane group
    if (skip.row_inst && row_skipped(skip, row)) return;
    const int64_t s = rp[row], e = rp[row + 1];
    if (e - s > p.long_thr) return;    // long rows: chunks above
    double acc = 0.0;
    for (int64_t k = s + lane; k < e; k += L) acc += (double)v[k] * (double)x[ci[k]];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) y[row] = acc;
}

// CSR-stream: after the chunk workgroups, workgroup b owns the rows
// [sb[2b], sb[2b+1]) whose entries (at most kStreamNnz, long rows excluded by the
// plan) it streams with unit stride into LDS as products, then one thread per
// row adds its segment in order.
template <class T>
__global__ __launch_bounds__(kBlock) void spmv_stream_kernel(const int64_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const T *__restrict__ v,
                                                             const T *__restrict__ x,
                                                             double *__restrict__ y, SpmvPlan p,
                                                             SpmvSkip skip) {
    if (!skip.row_inst && row_skipped(skip, 0)) return;   // one problem: one flag
    if ((int64_t)blockIdx.x < p.n_chunks) {
        if (!row_skipped(skip, p.long_rows[p.chunk_row[blockIdx.x]]))
            long_chunk(blockIdx.x, rp, ci, v, x, p);
        return;
    }
    __shared__ double prod[kStreamNnz];
    const int64_t bb = (int64_t)blockIdx.x - p.n_chunks;
    const int64_t r0 = p.sblock[2 * bb], r1 = p.sblock[2 * bb + 1];
    // a batch: skip the workgroup when all its rows belong to one flagged
    // instance (rows of a flagged instance are otherwise computed and unused)
    if (skip.row_inst && inst_of(skip.row_inst, r0) == inst_of(skip.row_inst, r1 - 1) &&
        row_skipped(skip, r0))
        return;
    const int64_t k0 = rp[r0];
    const int cnt = (int)(rp[r1] - k0);
    for (int i = threadIdx.x; i < cnt; i += kBlock) prod[i] = (double)v[k0 + i] * (double)x[ci[k0 + i]];
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

template <int L, class T>
static void launch_rows(const Csr &A, const SpmvPlan &p, const T *v, const T *x, double *y,
                        const SpmvSkip &skip, hipStream_t s) {
    const int64_t blocks = (A.rows * L + kBlock - 1) / kBlock + p.n_chunks;
    hipLaunchKernelGGL((spmv_rows_kernel<L, T>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A.rows,
                       A.rp, A.ci, v, x, y, p, skip);
}

template <class T>
static void spmv_impl(const Csr &A, const SpmvPlan &p, const T *v, const T *x, double *y,
                      const SpmvSkip &skip, hipStream_t s) {
    if (A.rows == 0) return;
    if (p.stream) {
        const int64_t blocks = p.n_sblocks + p.n_chunks;
        if (blocks > 0)
            hipLaunchKernelGGL((spmv_stream_kernel<T>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                               A.rp, A.ci, v, x, y, p, skip);
    } else {
        switch (p.lanes) {
        case 2: launch_rows<2>(A, p, v, x, y, skip, s); break;
        case 4: launch_rows<4>(A, p, v, x, y, skip, s); break;
        case 8: launch_rows<8>(A, p, v, x, y, skip, s); break;
        case 16: launch_rows<16>(A, p, v, x, y, skip, s); break;
        case 32: launch_rows<32>(A, p, v, x, y, skip, s); break;
        default: launch_rows<64>(A, p, v, x, y, skip, s); break;
        }
    }
    if (p.n_long > 0)
        hipLaunchKernelGGL(spmv_chunks_finish, dim3((unsigned)((p.n_long + 255) / 256)), dim3(256),
                           0, s, p, y, skip);
    PDCS_HIP(hipGetLastError());
}

void spmv(const Csr &A, const SpmvPlan &p, const double *x, double *y, const SpmvSkip &skip,
          hipStream_t s) {
    spmv_impl<double>(A, p, A.v, x, y, skip, s);
}

void spmv32(const Csr &A, const SpmvPlan &p, const float *x, double *y, const SpmvSkip &skip,
            hipStream_t s) {
    if (A.rows > 0 && !A.v32) throw_hip(hipErrorInvalidValue, "spmv32 without FP32 values", __FILE__, __LINE__);
    spmv_impl<float>(A, p, A.v32, x, y, skip, s);
}

}  // namespace pdcs
