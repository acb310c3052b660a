// iterate.hip -- the scalar and elementwise steps of Algorithm 1 that sit
// between the projection passes and the sparse products:
//   halpern  : ReflectedHalpern (and the same affine map applied to the kept
//              products G~x and G~^T y) fused with the weighted average;
//   reduce_kkt, restart_copy, unscale: pieces of the periodic check.
#include "decide_device.hpp"

namespace pdcs {

static unsigned grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}

// The step decision, one workgroup after the dual pass (a kernel boundary
// orders the passes' partials before it; a fenced last-workgroup hand-off
// would write back an XCD's L2 once per workgroup).
__global__ __launch_bounds__(kBlock) void decide_kernel(DevState *st, const double *px, int64_t ntx,
                                                        const double *py, int64_t nty) {
    if (st->halt) {
        if (threadIdx.x == 0) st->skip_update = 1;
        return;
    }
    decide_body(st, px, ntx, py, nty);
}

void decide(DevState *st, const double *px, int64_t ntx, const double *py, int64_t nty,
            hipStream_t s) {
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(kBlock), 0, s, st, px, ntx, py, nty);
    PDCS_HIP(hipGetLastError());
}

// z^{k+1} = (k+1)/(k+2) ((1+beta) z^ - beta z^k) + z^0/(k+2) (Algorithm 1), the
// same map on G~x and G~^T y, and sum += eta_used z^{k+1}.
__global__ __launch_bounds__(kBlock) void halpern_kernel(HalpernArgs a) {
    const DevState *st = a.st;
    if (st->skip_update) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double ha = st->ha, hb = st->hb, beta = st->beta, w = st->eta_used;
    if (i < a.n) {
        const double xn = ha * ((1.0 + beta) * a.xh[i] - beta * a.x[i]) + hb * a.xa[i];
        a.x[i] = xn;
        a.xsum[i] += w * xn;
        a.aty[i] = ha * ((1.0 + beta) * a.atyh[i] - beta * a.aty[i]) + hb * a.aty0[i];
    } else if (i < a.n + a.m) {
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
                                                            int64_t ntr,
                                                            const double *__restrict__ pc,
                                                            int64_t ntc, KktRaw *out) {
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

void reduce_kkt(const double *prow, int64_t ntr, const double *pcol, int64_t ntc, KktRaw *out,
                hipStream_t s) {
    hipLaunchKernelGGL(reduce_kkt_kernel, dim3(1), dim3(kBlock), 0, s, prow, ntr, pcol, ntc, out);
    PDCS_HIP(hipGetLastError());
}

__global__ void restart_kernel(int64_t n, int64_t m, const double *xc, const double *yc,
                               const double *gxc, const double *atyc, double *x, double *y,
                               double *xa, double *ya, double *gx, double *aty, double *gx0,
                               double *aty0, double *xsum, double *ysum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        x[i] = xa[i] = xc[i];
        aty[i] = aty0[i] = atyc[i];
        xsum[i] = 0.0;
    } else if (i < n + m) {
        const int64_t j = i - n;
        y[j] = ya[j] = yc[j];
        gx[j] = gx0[j] = gxc[j];
        ysum[j] = 0.0;
    }
}

void restart_copy(int64_t n, int64_t m, const double *xc, const double *yc, const double *gxc,
                  const double *atyc, double *x, double *y, double *xa, double *ya, double *gx,
                  double *aty, double *gx0, double *aty0, double *xsum, double *ysum,
                  hipStream_t s) {
    if (n + m == 0) return;
    hipLaunchKernelGGL(restart_kernel, dim3(grid_for(n + m)), dim3(kBlock), 0, s, n, m, xc, yc, gxc,
                       atyc, x, y, xa, ya, gx, aty, gx0, aty0, xsum, ysum);
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
