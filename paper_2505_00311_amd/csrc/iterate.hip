// iterate.hip -- the elementwise steps of Algorithm 1 that sit between the
// projection passes and the sparse products (the step decision runs inside the
// launch of G~^T y^, see spmv.hip):
//   halpern  : ReflectedHalpern (and the same affine map applied to the kept
//              products G~x and G~^T y) fused with the weighted average;
//   reduce_kkt, restart_copy, unscale: pieces of the periodic check.
#include "device_common.hpp"

namespace pdcs {

static unsigned grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}

// z^{k+1} = (k+1)/(k+2) ((1+beta) z^ - beta z^k) + z^0/(k+2) (Algorithm 1), the
// same map on G~x and G~^T y, and sum += eta_used z^{k+1}.
__global__ __launch_bounds__(kBlock) void halpern_kernel(HalpernArgs a) {
    if (a.promote && blockIdx.x == 0)   // no thread of this launch reads halt
        for (int64_t t = threadIdx.x; t < a.n_inst; t += kBlock) a.promote[t].halt = a.promote[t].halt_next;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n + a.m) return;
    const DevState *st = a.st + (i < a.n ? inst_of(a.x_inst, i) : inst_of(a.y_inst, i - a.n));
    if (st->skip_update) return;
    const double ha = st->ha, hb = st->hb, beta = st->beta, w = st->eta_used;
    if (i < a.n) {
        const double xn = ha * ((1.0 + beta) * a.xh[i] - beta * a.x[i]) + hb * a.xa[i];
        a.x[i] = xn;
        a.xsum[i] += w * xn;
        const double atyh = a.at.active() ? a.at.value(a.atyh, i) : a.atyh[i];
        a.aty[i] = ha * ((1.0 + beta) * atyh - beta * a.aty[i]) + hb * a.aty0[i];
    } else {
        const int64_t j = i - a.n;
        const double yn = ha * ((1.0 + beta) * a.yh[j] - beta * a.y[j]) + hb * a.ya[j];
        a.y[j] = yn;
        a.ysum[j] += w * yn;
        a.gx[j] = ha * ((1.0 + beta) * a.gxh[j] - beta * a.gx[j]) + hb * a.gx0[j];
    }
}

void halpern(const HalpernArgs &a, hipStream_t s) {
    if (a.n + a.m == 0) return;
    hipLaunchKernelGGL(halpern_kernel, dim3(grid_for(a.n + a.m)), dim3(kBlock), 0, s, a);
    PDCS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kBlock) void reduce_kkt_kernel(const double *__restrict__ pr,
                                                            const int64_t *ty, int64_t ntr,
                                                            const double *__restrict__ pc,
                                                            const int64_t *tx, int64_t ntc,
                                                            KktRaw *out_all) {
    const int64_t b = blockIdx.x;
    KktRaw *out = out_all + b;
    if (ty) pr += ty[b] * kPartials, ntr = ty[b + 1] - ty[b];
    if (tx) pc += tx[b] * kPartials, ntc = tx[b + 1] - tx[b];
    double s[6] = {0, 0, 0, 0, 0, 0};
    double mx[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t t = threadIdx.x; t < ntr; t += kBlock)
        for (int k = 0; k < 3; ++k) {
            s[k] += pr[t * kPartials + k];
            mx[k] = fmax(mx[k], pr[t * kPartials + 3 + k]);
        }
    for (int64_t t = threadIdx.x; t < ntc; t += kBlock)
        for (int k = 0; k < 3; ++k) {
            s[3 + k] += pc[t * kPartials + k];
            mx[3 + k] = fmax(mx[3 + k], pc[t * kPartials + 3 + k]);
        }
    block_sum_all<6>(s);
    __shared__ double red[kBlock / kWave][6];
    for (int k = 0; k < 6; ++k) mx[k] = wave_max(mx[k]);
    if (threadIdx.x % kWave == 0)
        for (int k = 0; k < 6; ++k) red[threadIdx.x / kWave][k] = mx[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) {
            double r = red[0][k];
            for (int w = 1; w < kBlock / kWave; ++w) r = fmax(r, red[w][k]);
            mx[k] = r;
        }
        for (int k = 0; k < 3; ++k) {
            out->rows_sum[k] = s[k];
            out->rows_max[k] = mx[k];
            out->cols_sum[k] = s[3 + k];
            out->cols_max[k] = mx[3 + k];
        }
    }
}

void reduce_kkt(int64_t B, const double *prow, const int64_t *ty, int64_t ntr, const double *pcol,
                const int64_t *tx, int64_t ntc, KktRaw *out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kkt_kernel, dim3((unsigned)B), dim3(kBlock), 0, s, prow, ty, ntr, pcol,
                       tx, ntc, out);
    PDCS_HIP(hipGetLastError());
}

__global__ void restart_kernel(RestartArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n + a.m) return;
    const bool xs = i < a.n;
    const int64_t j = xs ? i : i - a.n;
    const int code = a.code ? a.code[xs ? inst_of(a.x_inst, j) : inst_of(a.y_inst, j)] : 1;
    if (code == 0) return;
    const int c = code - 1;
    if (xs) {
        a.x[j] = a.xa[j] = a.xc[c][j];
        a.aty[j] = a.aty0[j] = a.atyc[c][j];
        a.xsum[j] = 0.0;
    } else {
        a.y[j] = a.ya[j] = a.yc[c][j];
        a.gx[j] = a.gx0[j] = a.gxc[c][j];
        a.ysum[j] = 0.0;
    }
}

void restart_copy(const RestartArgs &a, hipStream_t s) {
    if (a.n + a.m == 0) return;
    hipLaunchKernelGGL(restart_kernel, dim3(grid_for(a.n + a.m)), dim3(kBlock), 0, s, a);
    PDCS_HIP(hipGetLastError());
}

__global__ void unscale_kernel(const double *xs, const double *f, double *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f[i] * xs[i];
}
void unscale(const double *xs, const double *f, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(unscale_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, xs, f, out, n);
    PDCS_HIP(hipGetLastError());
}

__global__ void scale_in_kernel(const double *xu, const double *f, double *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = xu[i] / f[i];
}
void scale_in(const double *xu, const double *f, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(scale_in_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, xu, f, out, n);
    PDCS_HIP(hipGetLastError());
}

}  // namespace pdcs
