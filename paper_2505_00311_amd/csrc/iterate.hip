// iterate.hip -- the scalar and elementwise steps of Algorithm 1 that sit
// between the projection passes and the sparse products:
//   decide   : AdaptiveStepPDHG's accept/reject, the next step size and the
//              AdaptiveReflectionParameter, taken by one workgroup on device
//              so the host never waits inside an iteration;
//   halpern  : ReflectedHalpern (and the same affine map applied to the kept
//              products G~x and G~^T y) fused with the weighted average;
//   reduce_kkt, restart_copy, unscale: pieces of the periodic check.
#include "device_common.hpp"

namespace pdcs {

static unsigned grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}

// Step-size rule (reading: PDLP's): eta_bar = ||dz||_omega^2 / (2 |<dy, G~ dx>|),
// accept when eta <= eta_bar; eta' = min((1 - N^-a) eta_bar, (1 + N^-b) eta)
// with N = 1 + attempts so far.  Reflection parameter (reading): grows by
// beta_grow (capped at 1) while ||dz||_omega falls, else shrinks by beta_shrink.
__global__ __launch_bounds__(kBlock) void decide_kernel(DevState *__restrict__ st,
                                                        const double *__restrict__ px, int64_t ntx,
                                                        const double *__restrict__ py,
                                                        int64_t nty) {
    if (st->halt) {
        if (threadIdx.x == 0) st->skip_update = 1;
        return;
    }
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t t = threadIdx.x; t < ntx; t += kBlock) v[0] += px[t * kPartials + 0];
    for (int64_t t = threadIdx.x; t < nty; t += kBlock) {
        v[1] += py[t * kPartials + 0];
        v[2] += py[t * kPartials + 1];
    }
    block_sum_all<3>(v);
    if (threadIdx.x != 0) return;
    const double nx2 = v[0], ny2 = v[1], ip = v[2];
    st->nx2 = nx2, st->ny2 = ny2, st->ip = ip;
    st->attempts_cur += 1;
    const double omega = st->omega, eta = st->eta;
    const double den = 2.0 * fabs(ip);
    const double ebar = den > 0.0 ? (omega * nx2 + ny2 / omega) / den : INFINITY;
    if (ebar != ebar) {
        st->status = 3;
        st->halt = 1;
        st->skip_update = 1;
        return;
    }
    const double nn = (double)(st->attempts_total + st->attempts_cur + 1);
    const double e1 = (1.0 - pow(nn, -st->step_reduce_exp)) * ebar;
    const double e2 = (1.0 + pow(nn, -st->step_grow_exp)) * eta;
    const bool fixed = st->step_mode == 1;   // fixed step: every attempt is accepted
    const double enew = fixed ? eta : (e1 < e2 ? e1 : e2);
    if (fixed || eta <= ebar) {
        const double r = sqrt(omega * nx2 + ny2 / omega);
        double beta;
        if (st->beta_mode == 1)
            beta = st->beta_const;
        else
            beta = r <= st->r_prev ? fmin(1.0, st->beta_grow * st->beta_prev)
                                   : st->beta_shrink * st->beta_prev;
        st->r_prev = r;
        st->beta_prev = beta;
        st->beta = beta;
        const long long k = st->kin;
        st->ha = (double)(k + 1) / (double)(k + 2);
        st->hb = 1.0 / (double)(k + 2);
        st->eta_used = eta;
        st->eta_sum += eta;
        st->eta = enew;
        const long long it = st->n_iter;
        if (it < st->log_cap) {
            st->log_attempts[it] = st->attempts_cur;
            st->log_eta[it] = eta;
            st->log_beta[it] = beta;
            st->log_omega[it] = omega;
        }
        st->attempts_total += st->attempts_cur;
        st->attempts_cur = 0;
        st->n_iter = it + 1;
        st->kin = k + 1;
        st->skip_update = 0;
        if ((k + 1) % st->check_every == 0 || it + 1 >= st->max_iter) st->halt = 1;
    } else {
        st->eta = enew;
        st->skip_update = 1;
        if (st->attempts_cur >= st->max_attempts) {
            st->status = 3;
            st->halt = 1;
        }
    }
    st->tau = st->eta / st->omega;
    st->sigma = st->eta * st->omega;
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
