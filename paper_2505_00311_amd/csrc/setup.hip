// setup.hip -- once-per-problem work on the device: the CSR of G^T, the
// diagonal rescaling of Section 3 (reading: Ruiz infinity-norm passes, then one
// Pock-Chambolle pass with alpha = 1), the scaled problem vectors, input
// validation and small deterministic reductions.
#include <algorithm>
#include <cmath>

#include <rocprim/device/device_radix_sort.hpp>

#include "device_common.hpp"

namespace pdcs {

static unsigned grid_for(int64_t n, int block = kBlock) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

// Grid of the grid-stride kernels over a matrix's entries: a batch may hold
// more entries than one launch has work-items (2^32), so these kernels loop.
constexpr int64_t kStrideBlocks = (int64_t)1 << 20;
static unsigned grid_stride(int64_t n) {
    const int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g < kStrideBlocks ? g : kStrideBlocks);
}

// ------------------------------------------------------------- transpose
__global__ void iota_kernel(int32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

// Rows [c0, c0 + cols] of the transpose's row pointers from the block's sorted
// column keys (global columns in [c0, c0 + cols)): rp[j] = k0 + the first
// position whose key is >= j.
__global__ void rowptr_from_sorted(const int32_t *__restrict__ keys, int64_t nnz, int64_t c0,
                                   int64_t cols, int64_t k0, int64_t *__restrict__ rp) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nnz) return;
    const int64_t prev = k == 0 ? c0 - 1 : (int64_t)keys[k - 1];
    const int64_t cur = k == nnz ? c0 + cols : (int64_t)keys[k];
    for (int64_t j = prev + 1; j <= cur; ++j) rp[j] = k0 + k;
}

// Entry k0 + p of the transposed block is entry k0 + perm[p] of the block;
// its column in G^T is that entry's row, found among rows [r0, r0 + rows].
__global__ void gather_transpose(const int64_t *__restrict__ rp, int64_t r0, int64_t rows,
                                 const double *__restrict__ v, const int32_t *__restrict__ perm,
                                 int64_t k0, int64_t nnz, int32_t *__restrict__ tci,
                                 double *__restrict__ tv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int64_t k = k0 + perm[p];
    int64_t lo = r0, hi = r0 + rows;  // largest row i with rp[i] <= k
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (rp[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    tci[k0 + p] = (int32_t)lo;
    tv[k0 + p] = v[k];
}

// The transpose of a block-diagonal A, block by block (a single problem is
// one block): each block's entries are sorted by column with a stable radix
// sort of 32-bit positions, so a block needs fewer than 2^31 entries while
// the whole matrix may hold more.  Block b of A (rows [r0, r0 + rows),
// columns [c0, c0 + cols), entries [k0, k0 + nnz)) becomes rows [c0, c0 +
// cols) and the same entries of At.
void transpose_csr(const Csr &A, Csr &At, const TBlock *blocks, int64_t nblocks, hipStream_t s) {
    int64_t big = 0;
    for (int64_t b = 0; b < nblocks; ++b) big = std::max(big, blocks[b].nnz);
    if (big >= ((int64_t)1 << 31))
        throw_hip(hipErrorInvalidValue, "transpose block of 2^31 or more entries", __FILE__, __LINE__);
    int32_t *keys_out = nullptr, *perm_in = nullptr, *perm_out = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    unsigned bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < A.cols) ++bits;
    if (big > 0) {
        PDCS_HIP(hipMallocAsync((void **)&keys_out, sizeof(int32_t) * big, s));
        PDCS_HIP(hipMallocAsync((void **)&perm_in, sizeof(int32_t) * big, s));
        PDCS_HIP(hipMallocAsync((void **)&perm_out, sizeof(int32_t) * big, s));
        PDCS_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, A.ci, keys_out, perm_in, perm_out,
                                           (size_t)big, 0, bits, s));
        PDCS_HIP(hipMallocAsync(&tmp, tmp_bytes, s));
    }
    for (int64_t b = 0; b < nblocks; ++b) {
        const TBlock &B = blocks[b];
        if (B.nnz == 0) {
            hipLaunchKernelGGL(rowptr_from_sorted, dim3(1), dim3(1), 0, s, (const int32_t *)nullptr,
                               (int64_t)0, B.c0, B.cols, B.k0, At.rp);
            continue;
        }
        hipLaunchKernelGGL(iota_kernel, dim3(grid_for(B.nnz)), dim3(kBlock), 0, s, perm_in, B.nnz);
        size_t need = 0;
        PDCS_HIP(rocprim::radix_sort_pairs(nullptr, need, A.ci + B.k0, keys_out, perm_in, perm_out,
                                           (size_t)B.nnz, 0, bits, s));
        // LSD radix sort is stable: entries of a column keep increasing row order
        PDCS_HIP(rocprim::radix_sort_pairs(tmp, need, A.ci + B.k0, keys_out, perm_in, perm_out,
                                           (size_t)B.nnz, 0, bits, s));
        hipLaunchKernelGGL(rowptr_from_sorted, dim3(grid_for(B.nnz + 1)), dim3(kBlock), 0, s, keys_out,
                           B.nnz, B.c0, B.cols, B.k0, At.rp);
        hipLaunchKernelGGL(gather_transpose, dim3(grid_for(B.nnz)), dim3(kBlock), 0, s, A.rp, B.r0,
                           B.rows, A.v, perm_out, B.k0, B.nnz, At.ci, At.v);
    }
    PDCS_HIP(hipGetLastError());
    if (big > 0) {
        PDCS_HIP(hipFreeAsync(tmp, s));
        PDCS_HIP(hipFreeAsync(keys_out, s));
        PDCS_HIP(hipFreeAsync(perm_in, s));
        PDCS_HIP(hipFreeAsync(perm_out, s));
    }
}

// ------------------------------------------------------------- rescaling
// One wavefront per row.  For G (row_first) the entry is (e_i a_ij) f_j; for
// G^T, whose rows are G's columns, the same product (e_i a_ij) f_j is formed.
template <bool MAX>
__global__ __launch_bounds__(kBlock) void rows_reduce_scaled(int64_t rows, const int64_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const double *__restrict__ v,
                                                             const double *__restrict__ srow,
                                                             const double *__restrict__ scol,
                                                             int row_first, double *__restrict__ out) {
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    if (row >= rows) return;
    double acc = 0.0;
    const double sr = srow[row];
    for (int64_t k = rp[row] + lane; k < rp[row + 1]; k += kWave) {
        const double a = row_first ? fabs(sr * v[k] * scol[ci[k]]) : fabs(scol[ci[k]] * v[k] * sr);
        acc = MAX ? fmax(acc, a) : acc + a;
    }
    acc = MAX ? wave_max(acc) : wave_sum(acc);
    if (lane == 0) out[row] = acc;
}

// er scales this matrix's rows and ec its columns; row_first says whether er
// is G's row scale E (A = G) or its column scale F (A = G^T).
void rows_absmax_scaled(const Csr &A, const double *er, const double *ec, bool row_first,
                        double *out, hipStream_t s) {
    if (A.rows == 0) return;
    hipLaunchKernelGGL(rows_reduce_scaled<true>, dim3(grid_for(A.rows * kWave)), dim3(kBlock), 0,
                       s, A.rows, A.rp, A.ci, A.v, er, ec, row_first ? 1 : 0, out);
    PDCS_HIP(hipGetLastError());
}

void rows_abssum_scaled(const Csr &A, const double *er, const double *ec, bool row_first,
                        double *out, hipStream_t s) {
    if (A.rows == 0) return;
    hipLaunchKernelGGL(rows_reduce_scaled<false>, dim3(grid_for(A.rows * kWave)), dim3(kBlock), 0,
                       s, A.rows, A.rp, A.ci, A.v, er, ec, row_first ? 1 : 0, out);
    PDCS_HIP(hipGetLastError());
}

__global__ void divide_by_sqrt_kernel(double *e, const double *r, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && r[i] > 0.0) e[i] /= sqrt(r[i]);
}

void divide_by_sqrt(double *e, const double *r, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(divide_by_sqrt_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, e, r, n);
    PDCS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kBlock) void scale_values_kernel(int64_t rows, const int64_t *__restrict__ rp,
                                                              const int32_t *__restrict__ ci,
                                                              const double *__restrict__ v,
                                                              const double *__restrict__ srow,
                                                              const double *__restrict__ scol,
                                                              int row_first,
                                                              double *__restrict__ out) {
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    if (row >= rows) return;
    const double sr = srow[row];
    for (int64_t k = rp[row] + lane; k < rp[row + 1]; k += kWave)
        out[k] = row_first ? sr * v[k] * scol[ci[k]] : scol[ci[k]] * v[k] * sr;
}

void scale_values(const Csr &A, const double *er, const double *ec, bool row_first, double *out,
                  hipStream_t s) {
    if (A.rows == 0) return;
    hipLaunchKernelGGL(scale_values_kernel, dim3(grid_for(A.rows * kWave)), dim3(kBlock), 0, s,
                       A.rows, A.rp, A.ci, A.v, er, ec, row_first ? 1 : 0, out);
    PDCS_HIP(hipGetLastError());
}

__global__ void scale_vectors_kernel(int64_t n, int64_t m, int64_t nb, const double *c,
                                     const double *h, const double *l, const double *u,
                                     const double *e, const double *f, double *cs, double *hs,
                                     double *ls, double *us, double *dx, double *dy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        cs[i] = f[i] * c[i];
        dx[i] = 1.0 / f[i];
        if (i < nb) {
            ls[i] = l[i] / f[i];
            us[i] = u[i] / f[i];
        }
    }
    if (i < m) {
        hs[i] = e[i] * h[i];
        dy[i] = 1.0 / e[i];
    }
}

void scale_problem_vectors(int64_t n, int64_t m, int64_t nb, const double *c, const double *h,
                           const double *l, const double *u, const double *e, const double *f,
                           double *cs, double *hs, double *ls, double *us, double *dx, double *dy,
                           hipStream_t s) {
    const int64_t k = n > m ? n : m;
    if (k == 0) return;
    hipLaunchKernelGGL(scale_vectors_kernel, dim3(grid_for(k)), dim3(kBlock), 0, s, n, m, nb, c, h,
                       l, u, e, f, cs, hs, ls, us, dx, dy);
    PDCS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ reductions
constexpr int kRedBlocks = 512;

template <int MODE>  // 0: sum of squares, 1: max abs
__global__ __launch_bounds__(kBlock) void reduce_stage1(const double *__restrict__ a, int64_t n,
                                                        double *__restrict__ part) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kBlock)
        acc[0] = MODE == 0 ? acc[0] + a[i] * a[i] : fmax(acc[0], fabs(a[i]));
    if (MODE == 0) {
        block_sum_all<1>(acc);
    } else {
        __shared__ double red[kBlock / kWave];
        double w = wave_max(acc[0]);
        if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = w;
        __syncthreads();
        acc[0] = red[0];
        for (int i = 1; i < kBlock / kWave; ++i) acc[0] = fmax(acc[0], red[i]);
    }
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

template <int MODE>
__global__ void reduce_stage2(const double *__restrict__ part, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double r = 0.0;
    for (int i = 0; i < kRedBlocks; ++i) r = MODE == 0 ? r + part[i] : fmax(r, part[i]);
    *out = r;
}

template <int MODE>
static void reduce(const double *a, int64_t n, double *out, hipStream_t s) {
    double *part = nullptr;
    PDCS_HIP(hipMallocAsync((void **)&part, sizeof(double) * kRedBlocks, s));
    hipLaunchKernelGGL(reduce_stage1<MODE>, dim3(kRedBlocks), dim3(kBlock), 0, s, a, n, part);
    hipLaunchKernelGGL(reduce_stage2<MODE>, dim3(1), dim3(64), 0, s, part, out);
    PDCS_HIP(hipGetLastError());
    PDCS_HIP(hipFreeAsync(part, s));
}

void reduce_absmax(const double *a, int64_t n, double *out, hipStream_t s) { reduce<1>(a, n, out, s); }
void reduce_sumsq(const double *a, int64_t n, double *out, hipStream_t s) { reduce<0>(a, n, out, s); }

__global__ void check_finite_kernel(const double *a, int64_t n, int *flag) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
        bad |= !isfinite(a[i]);
    if (bad) atomicOr(flag, 1);
}

void check_finite(const double *a, int64_t n, int *flag, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(check_finite_kernel, dim3(grid_stride(n)), dim3(kBlock), 0, s, a, n, flag);
    PDCS_HIP(hipGetLastError());
}

// -------------------------------------------------------------- elementwise
__global__ void fill_kernel(double *p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
void fill(double *p, int64_t n, double v, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
    PDCS_HIP(hipGetLastError());
}

__global__ void to_float_kernel(const double *in, float *out, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
        out[i] = (float)in[i];
}
void to_float(const double *in, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(to_float_kernel, dim3(grid_stride(n)), dim3(kBlock), 0, s, in, out, n);
    PDCS_HIP(hipGetLastError());
}

__global__ void div_kernel(const double *a, const double *b, double *o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a[i] / b[i];
}
void div_vec(const double *a, const double *b, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(div_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, a, b, out, n);
    PDCS_HIP(hipGetLastError());
}

__global__ void mul_kernel(const double *a, const double *b, double *o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a[i] * b[i];
}
void mul_vec(const double *a, const double *b, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(mul_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, a, b, out, n);
    PDCS_HIP(hipGetLastError());
}

__global__ void copy_kernel(const double *a, double *o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a[i];
}
void copy_vec(const double *a, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, a, out, n);
    PDCS_HIP(hipGetLastError());
}

// v = w / sqrt(sumsq[instance]) (left unchanged where the norm is zero)
__global__ void scale_inv_sqrt_kernel(const double *w, const double *sumsq, const int32_t *map,
                                      double *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lam = sqrt(sumsq[inst_of(map, i)]);
    if (lam > 0.0) v[i] = w[i] / lam;
}
void scale_by_inv_sqrt(const double *w, const double *sumsq, const int32_t *map, double *v,
                       int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(scale_inv_sqrt_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, w, sumsq, map,
                       v, n);
    PDCS_HIP(hipGetLastError());
}

// out[i] = vals[instance of i]
__global__ void fill_by_inst_kernel(double *out, const int32_t *map, const double *vals, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = vals[inst_of(map, i)];
}
void fill_by_inst(double *out, const int32_t *map, const double *vals, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(fill_by_inst_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, out, map, vals, n);
    PDCS_HIP(hipGetLastError());
}

// One workgroup per segment [off[b], off[b+1]): sum of squares (MODE 0) or
// max abs (MODE 1) into out[b], in a fixed order.
template <int MODE>
__global__ __launch_bounds__(kBlock) void reduce_seg_kernel(const double *__restrict__ a,
                                                            const int64_t *__restrict__ off,
                                                            double *__restrict__ out) {
    const int64_t b = blockIdx.x;
    double acc[1] = {0.0};
    for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += kBlock)
        acc[0] = MODE == 0 ? acc[0] + a[i] * a[i] : fmax(acc[0], fabs(a[i]));
    if (MODE == 0) {
        block_sum_all<1>(acc);
    } else {
        __shared__ double red[kBlock / kWave];
        const double w = wave_max(acc[0]);
        if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = w;
        __syncthreads();
        acc[0] = red[0];
        for (int i = 1; i < kBlock / kWave; ++i) acc[0] = fmax(acc[0], red[i]);
    }
    if (threadIdx.x == 0) out[b] = acc[0];
}
void reduce_segments(int mode, const double *a, const int64_t *off, int64_t B, double *out,
                     hipStream_t s) {
    if (B == 0) return;
    if (mode == 0)
        hipLaunchKernelGGL(reduce_seg_kernel<0>, dim3((unsigned)B), dim3(kBlock), 0, s, a, off, out);
    else
        hipLaunchKernelGGL(reduce_seg_kernel<1>, dim3((unsigned)B), dim3(kBlock), 0, s, a, off, out);
    PDCS_HIP(hipGetLastError());
}

// out[i] = in[idx[i]]
__global__ void gather_kernel(double *out, const double *in, const int32_t *idx, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[idx[i]];
}
void gather(double *out, const double *in, const int32_t *idx, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(gather_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, out, in, idx, n);
    PDCS_HIP(hipGetLastError());
}
// out[idx[i] - base] = in[i]
__global__ void scatter_kernel(double *out, const double *in, const int32_t *idx, int64_t n,
                               int64_t base) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[idx[i] - base] = in[i];
}
void scatter(double *out, const double *in, const int32_t *idx, int64_t n, int64_t base,
             hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, out, in, idx, n, base);
    PDCS_HIP(hipGetLastError());
}
// ci[k] = pos[ci[k]]: column indices renumbered
__global__ void relabel_kernel(int32_t *ci, int64_t nnz, const int32_t *pos) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += step)
        ci[k] = pos[ci[k]];
}
// r = 1 / fl(sqrt 2), the constant the host side of the map uses, so both
// sides round the same way
__global__ void rotate_pairs_kernel(double *v, const int64_t *offs, int64_t count, int64_t base,
                                    double r) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int64_t o = offs[t] - base;
    const double a = v[o], b = v[o + 1];
    v[o] = (a + b) * r;
    v[o + 1] = (a - b) * r;
}
void rotate_pairs(double *v, const int64_t *offs, int64_t count, int64_t base, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(rotate_pairs_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       v, offs, count, base, 1.0 / std::sqrt(2.0));
    PDCS_HIP(hipGetLastError());
}

void relabel(int32_t *ci, int64_t nnz, const int32_t *pos, hipStream_t s) {
    if (nnz == 0) return;
    hipLaunchKernelGGL(relabel_kernel, dim3(grid_stride(nnz)), dim3(kBlock), 0, s, ci, nnz, pos);
    PDCS_HIP(hipGetLastError());
}

}  // namespace pdcs
