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
//
// Column-slab form: gathers of x with power-law column popularity miss each
// XCD's L2 on almost every entry once x outgrows it.  The plan cuts the
// columns into S slabs of equal entry counts; workgroup i runs on XCD i mod 8
// and the plan orders the workgroups so that each XCD takes the blocks of one
// slab only, whose slice of x (|x|/S) then stays in that XCD's L2.  When the
// first (hottest) columns hold a large share of the entries they form a hot
// slab of their own, whose few columns every block stages in LDS and whose
// blocks go to every XCD; a narrow hot slab cut like the others would leave
// its XCDs idle while the others gather from L2.  Each
// workgroup streams a row range of its slab like the CSR-stream kernel and
// writes the slab's row sums; a second kernel adds a row's S slab sums in slab
// order (a fixed order, so results repeat bit for bit from run to run).
#include "decide_device.hpp"

namespace pdcs {

// Whether the instance of `row` has the skip flag set (see SpmvSkip).
__device__ __forceinline__ bool row_skipped(const SpmvSkip &k, int64_t row) {
    if (k.flag == SkipNone) return false;
    const DevState &s = k.st[inst_of(k.row_inst, row)];
    return k.flag == SkipHalt ? s.halt != 0 : s.skip_update != 0;
}

// Workgroups [0, dec.nblk) of a product launch take the step decision (one
// per instance, the rest idle); returns true for them, else shifts bid to the
// product's own numbering.
__device__ __forceinline__ bool decide_blocks(const DecideArgs &dec, int64_t &bid) {
    if (bid >= dec.nblk) {
        bid -= dec.nblk;
        return false;
    }
    if (bid < dec.B) decide_instance(dec.st, bid, dec.px, dec.tx, dec.ntx, dec.py, dec.ty, dec.nty);
    return true;
}

// Whether chunk c's row is skipped; a single problem's one flag was checked at
// the kernel's start, so only a batch looks the row up.
__device__ __forceinline__ bool chunk_skipped(const SpmvSkip &k, const SpmvPlan &p, int64_t c) {
    return k.row_inst && row_skipped(k, p.long_rows[p.chunk_row[c]]);
}

// The workgroup's sum of v[k] x[ci[k]] over k in [b, e) (a chunk of a long
// row), identical in every thread: each thread takes its entries
// kChunkRound at a time with all loads issued first and adds them in entry
// order, then the workgroup sum is formed in a fixed order.  A second kernel
// (or the product's consumer) adds each row's chunk sums in chunk order.
constexpr int kChunkRound = 8;
template <class T>
__device__ __forceinline__ double chunk_sum(int64_t b, int64_t e, const int32_t *__restrict__ ci,
                                            const T *__restrict__ v, const T *__restrict__ x) {
    constexpr int U = kChunkRound;
    double acc[1] = {0.0};
    for (int64_t k0 = b + threadIdx.x; k0 < e; k0 += U * kBlock) {
        int32_t cc[U];
        T w[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {   // streamed once: kept out of the way of x in L2
            const int64_t k = min(k0 + (int64_t)u * kBlock, e - 1);
            cc[u] = __builtin_nontemporal_load(&ci[k]);
            w[u] = __builtin_nontemporal_load(&v[k]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[cc[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + (int64_t)u * kBlock < e) acc[0] += (double)w[u] * (double)xv[u];
    }
    block_sum_all<1>(acc);
    return acc[0];
}

// Chunk c of a long row of the CSR matrix itself (the layouts without slabs).
template <class T>
__device__ __forceinline__ void long_chunk(int64_t c, const int64_t *__restrict__,
                                           const int32_t *__restrict__ ci,
                                           const T *__restrict__ v,
                                           const T *__restrict__ x, const SpmvPlan &p) {
    const double sum = chunk_sum(p.chunk_begin[c], p.chunk_end[c], ci, v, x);
    if (threadIdx.x == 0) p.chunk_part[c] = sum;
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
                                                           SpmvSkip skip, DecideArgs dec) {
    int64_t bid = blockIdx.x;
    if (decide_blocks(dec, bid)) return;
    if (!skip.row_inst && row_skipped(skip, 0)) return;   // one problem: one flag
    if (bid < p.n_chunks) {
        if (!chunk_skipped(skip, p, bid)) long_chunk(bid, rp, ci, v, x, p);
        return;
    }
    const int64_t gid = (bid - p.n_chunks) * kBlock + threadIdx.x;
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

// One streamed block: rows [0, nrows) of a row range whose entries are
// [k0, k0 + cnt) (cnt <= kStreamNnz, nrows <= kStreamRows); rp points at the
// range's first row pointer, ci, v and out are offset to the range.  Every
// thread first issues all of its loads (row pointers into LDS, then its
// kStreamNnz / kBlock column indices and values, then the gathers of x), so a
// block waits on two memory latencies rather than one per entry; the products
// go to LDS and one thread per row adds its segment in entry order.
template <class T, class RP>
__device__ __forceinline__ void stream_block(int nrows, const RP *__restrict__ rp, RP k0, int cnt,
                                             const int32_t *__restrict__ ci,
                                             const T *__restrict__ v, const T *__restrict__ x,
                                             double *__restrict__ out, int lds_cols = 0) {
    __shared__ double prod[kStreamNnz];
    __shared__ int32_t seg[kStreamRows + 1];
    constexpr int U = kStreamNnz / kBlock;
    constexpr int UR = (kStreamRows + kBlock) / kBlock;   // covers nrows + 1 <= kStreamRows + 1
    const int t = threadIdx.x;
    // loads at clamped indices, unconditional, so none waits behind a branch
    int32_t sg[UR];
#pragma unroll
    for (int u = 0; u < UR; ++u) sg[u] = (int32_t)(rp[min(t + u * kBlock, nrows)] - k0);
    if (cnt > 0) {
        int32_t c[U];
        T w[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {   // streamed once: kept out of the way of x in L2
            const int i = min(t + u * kBlock, cnt - 1);
            c[u] = __builtin_nontemporal_load(&ci[i]);
            w[u] = __builtin_nontemporal_load(&v[i]);
        }
        if (lds_cols > 0) {   // a hot slab: its columns x[0, lds_cols) are staged in LDS first
            for (int j = t; j < lds_cols; j += kBlock) prod[j] = (double)x[j];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = (T)prod[c[u]];
            __syncthreads();
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t + u * kBlock < cnt) prod[t + u * kBlock] = (double)w[u] * (double)xv[u];
    }
#pragma unroll
    for (int u = 0; u < UR; ++u)
        if (t + u * kBlock <= nrows) seg[t + u * kBlock] = sg[u];
    __syncthreads();
    for (int r = t; r < nrows; r += kBlock) {
        int i = seg[r];
        const int e = seg[r + 1];
        double acc = 0.0;
        for (; i + 4 <= e; i += 4) {   // four reads in flight, added in entry order
            const double a0 = prod[i], a1 = prod[i + 1], a2 = prod[i + 2], a3 = prod[i + 3];
            acc += a0;
            acc += a1;
            acc += a2;
            acc += a3;
        }
        for (; i < e; ++i) acc += prod[i];
        out[r] = acc;
    }
}

// CSR-stream: after the chunk workgroups, workgroup b owns the rows
// [sb[2b], sb[2b+1]) (long rows excluded by the plan), streamed as above.
template <class T>
__global__ __launch_bounds__(kBlock) void spmv_stream_kernel(const int64_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const T *__restrict__ v,
                                                             const T *__restrict__ x,
                                                             double *__restrict__ y, SpmvPlan p,
                                                             SpmvSkip skip, DecideArgs dec) {
    int64_t bid = blockIdx.x;
    if (decide_blocks(dec, bid)) return;
    if (!skip.row_inst && row_skipped(skip, 0)) return;   // one problem: one flag
    if (bid < p.n_chunks) {
        if (!chunk_skipped(skip, p, bid)) long_chunk(bid, rp, ci, v, x, p);
        return;
    }
    const int64_t bb = bid - p.n_chunks;
    const int64_t r0 = p.sblock[2 * bb], r1 = p.sblock[2 * bb + 1];
    // a batch: skip the workgroup when all its rows belong to one flagged
    // instance (rows of a flagged instance are otherwise computed and unused)
    if (skip.row_inst && inst_of(skip.row_inst, r0) == inst_of(skip.row_inst, r1 - 1) &&
        row_skipped(skip, r0))
        return;
    const int64_t k0 = rp[r0];
    stream_block<T, int64_t>((int)(r1 - r0), rp + r0, k0, (int)(rp[r1] - k0), ci + k0, v + k0, x,
                             y + r0);
}

// smallest power of two >= half the mean row length, within [2, 64]
int choose_lanes(double avg) {
    int L = 2;
    while (L < 64 && 2.0 * L < avg) L <<= 1;
    return L;
}

int64_t spmv_blocks(const Csr &A, const SpmvPlan &p) {
    if (A.rows == 0) return 0;
    if (p.n_slabs > 0) return p.n_slab_blocks;
    if (p.stream) return p.n_sblocks + p.n_chunks;
    return (A.rows * p.lanes + kBlock - 1) / kBlock + p.n_chunks;
}

template <int L, class T>
static void launch_rows(const Csr &A, const SpmvPlan &p, const T *v, const T *x, double *y,
                        const SpmvSkip &skip, const DecideArgs &dec, hipStream_t s) {
    const int64_t blocks = dec.nblk + (A.rows * L + kBlock - 1) / kBlock + p.n_chunks;
    hipLaunchKernelGGL((spmv_rows_kernel<L, T>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A.rows,
                       A.rp, A.ci, v, x, y, p, skip, dec);
}

// Column-slab blocks (after the decision's): a streamed block of a slab's
// short rows [r0, r1) writes their slab sums (0 for an empty segment); a
// chunk block (r0 < 0) writes the sum of a piece of a long row's entries in
// that slab.
template <class T>
__global__ __launch_bounds__(kBlock) void spmv_slab_kernel(int64_t rows,
                                                           const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const T *__restrict__ v,
                                                           const T *__restrict__ sv,
                                                           const T *__restrict__ x, SpmvPlan p,
                                                           SpmvSkip skip, DecideArgs dec) {
    int64_t bid = blockIdx.x;
    if (decide_blocks(dec, bid)) return;
    if (!skip.row_inst && row_skipped(skip, 0)) return;   // one problem: one flag
    const SlabBlock d = p.slab_blk[bid];
    if (d.r0 < 0) {   // a chunk of a long row, on its slab's XCDs
        const int64_t c = -1 - (int64_t)d.r0;
        if (chunk_skipped(skip, p, c)) return;
        const double sum = chunk_sum(d.k0, (int64_t)d.k0 + (d.cs & 0xffff), p.slab_ci, sv, x);
        if (threadIdx.x == 0) p.chunk_part[c] = sum;
        return;
    }
    if (d.r1 <= d.r0) return;   // padding that keeps the slab-to-XCD assignment
    if (skip.row_inst && inst_of(skip.row_inst, d.r0) == inst_of(skip.row_inst, d.r1 - 1) &&
        row_skipped(skip, d.r0))
        return;
    const int cnt = d.cs & 0xffff, slab = d.cs >> 16;
    const int32_t *__restrict__ lrp = p.slab_rp + (int64_t)slab * (rows + 1) + d.r0;
    stream_block<T, int32_t>(d.r1 - d.r0, lrp, d.k0, cnt, p.slab_ci + d.k0, sv + d.k0, x,
                             p.slab_part + (int64_t)slab * rows + d.r0,
                             slab == 0 ? p.hot_cols : 0);
}

// y[i] = sum over slabs s = 0..S-1 of slab_part[s][i], in slab order.  Long
// rows have no slab entries (their 0 is overwritten by spmv_chunks_finish).
template <int S>
__global__ __launch_bounds__(kBlock) void spmv_slab_sum(int64_t rows, const double *__restrict__ part,
                                                        double *__restrict__ y, SpmvSkip skip) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= rows || row_skipped(skip, i)) return;
    double t[S];
#pragma unroll
    for (int k = 0; k < S; ++k) t[k] = part[k * rows + i];
    double acc = t[0];
#pragma unroll
    for (int k = 1; k < S; ++k) acc += t[k];
    y[i] = acc;
}

template <class T>
__global__ void slab_values_kernel(const T *__restrict__ v, const int32_t *__restrict__ perm,
                                   T *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v[perm[i]];
}

void slab_values(const Csr &A, const SpmvPlan &p, hipStream_t s) {
    const int64_t n = p.slab_base[p.n_slabs];
    if (p.n_slabs == 0 || n == 0) return;
    if (!A.sv) throw_hip(hipErrorInvalidValue, "slab values not allocated", __FILE__, __LINE__);
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL((slab_values_kernel<double>), dim3(g), dim3(256), 0, s, A.v, p.slab_perm, A.sv, n);
    if (A.v32 && A.sv32)
        hipLaunchKernelGGL((slab_values_kernel<float>), dim3(g), dim3(256), 0, s, A.v32, p.slab_perm,
                           A.sv32, n);
    PDCS_HIP(hipGetLastError());
}

// finish = false: the first kernel only (see ProductTail).  dec_in.st set:
// the launch also takes the step decision.
template <class T>
static void spmv_impl(const Csr &A, const SpmvPlan &p, const T *v, const T *sv, const T *x,
                      double *y, const SpmvSkip &skip, hipStream_t s, bool finish,
                      const DecideArgs &dec_in = DecideArgs{}) {
    DecideArgs dec = dec_in;
    dec.nblk = dec.st ? (dec.B + kXcds - 1) / kXcds * kXcds : 0;
    if (spmv_blocks(A, p) + dec.nblk > kMaxLaunchBlocks)
        throw_hip(hipErrorInvalidConfiguration, "product plan needs more workgroups than one launch holds",
                  __FILE__, __LINE__);
    if (A.rows == 0) {   // no product: the decision still runs
        if (dec.nblk > 0)
            hipLaunchKernelGGL((spmv_stream_kernel<T>), dim3((unsigned)dec.nblk), dim3(kBlock), 0, s,
                               A.rp, A.ci, v, x, y, p, skip, dec);
        PDCS_HIP(hipGetLastError());
        return;
    }
    if (p.n_slabs > 0) {
        if (!sv) throw_hip(hipErrorInvalidValue, "column-slab plan without slab values", __FILE__, __LINE__);
        const int64_t blocks = dec.nblk + p.n_slab_blocks;   // chunks are slab blocks here
        if (blocks > 0)
            hipLaunchKernelGGL((spmv_slab_kernel<T>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                               A.rows, A.rp, A.ci, v, sv, x, p, skip, dec);
        if (!finish) {
            PDCS_HIP(hipGetLastError());
            return;
        }
        const dim3 g((unsigned)((A.rows + kBlock - 1) / kBlock));
        switch (p.n_slabs) {   // 1, 2, 4 or 8 slabs, plus one when there is a hot slab
        case 1: hipLaunchKernelGGL(spmv_slab_sum<1>, g, dim3(kBlock), 0, s, A.rows, p.slab_part, y, skip); break;
        case 2: hipLaunchKernelGGL(spmv_slab_sum<2>, g, dim3(kBlock), 0, s, A.rows, p.slab_part, y, skip); break;
        case 3: hipLaunchKernelGGL(spmv_slab_sum<3>, g, dim3(kBlock), 0, s, A.rows, p.slab_part, y, skip); break;
        case 4: hipLaunchKernelGGL(spmv_slab_sum<4>, g, dim3(kBlock), 0, s, A.rows, p.slab_part, y, skip); break;
        case 5: hipLaunchKernelGGL(spmv_slab_sum<5>, g, dim3(kBlock), 0, s, A.rows, p.slab_part, y, skip); break;
        case 8: hipLaunchKernelGGL(spmv_slab_sum<8>, g, dim3(kBlock), 0, s, A.rows, p.slab_part, y, skip); break;
        default: hipLaunchKernelGGL(spmv_slab_sum<9>, g, dim3(kBlock), 0, s, A.rows, p.slab_part, y, skip); break;
        }
    } else if (p.stream) {
        const int64_t blocks = dec.nblk + p.n_sblocks + p.n_chunks;
        if (blocks > 0)
            hipLaunchKernelGGL((spmv_stream_kernel<T>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                               A.rp, A.ci, v, x, y, p, skip, dec);
    } else {
        switch (p.lanes) {
        case 2: launch_rows<2>(A, p, v, x, y, skip, dec, s); break;
        case 4: launch_rows<4>(A, p, v, x, y, skip, dec, s); break;
        case 8: launch_rows<8>(A, p, v, x, y, skip, dec, s); break;
        case 16: launch_rows<16>(A, p, v, x, y, skip, dec, s); break;
        case 32: launch_rows<32>(A, p, v, x, y, skip, dec, s); break;
        default: launch_rows<64>(A, p, v, x, y, skip, dec, s); break;
        }
    }
    if (p.n_long > 0 && finish)
        hipLaunchKernelGGL(spmv_chunks_finish, dim3((unsigned)((p.n_long + 255) / 256)), dim3(256),
                           0, s, p, y, skip);
    PDCS_HIP(hipGetLastError());
}

void spmv(const Csr &A, const SpmvPlan &p, const double *x, double *y, const SpmvSkip &skip,
          hipStream_t s) {
    spmv_impl<double>(A, p, A.v, A.sv, x, y, skip, s, true);
}

void spmv_head(const Csr &A, const SpmvPlan &p, const double *x, double *y, const SpmvSkip &skip,
               hipStream_t s, const DecideArgs &dec) {
    spmv_impl<double>(A, p, A.v, A.sv, x, y, skip, s, false, dec);
}

void spmv32(const Csr &A, const SpmvPlan &p, const float *x, double *y, const SpmvSkip &skip,
            hipStream_t s) {
    if (A.rows > 0 && !A.v32) throw_hip(hipErrorInvalidValue, "spmv32 without FP32 values", __FILE__, __LINE__);
    spmv_impl<float>(A, p, A.v32, A.sv32, x, y, skip, s, true);
}

void spmv32_head(const Csr &A, const SpmvPlan &p, const float *x, double *y, const SpmvSkip &skip,
                 hipStream_t s, const DecideArgs &dec) {
    if (A.rows > 0 && !A.v32) throw_hip(hipErrorInvalidValue, "spmv32 without FP32 values", __FILE__, __LINE__);
    spmv_impl<float>(A, p, A.v32, A.sv32, x, y, skip, s, false, dec);
}

}  // namespace pdcs
