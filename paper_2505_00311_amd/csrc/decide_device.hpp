// decide_device.hpp -- the on-device step decision of Algorithm 1:
// AdaptiveStepPDHG's accept/reject and next step size, and the
// AdaptiveReflectionParameter, taken by one workgroup on the device so the host
// never waits inside an iteration.
#pragma once
#include "device_common.hpp"

namespace pdcs {

// Step-size rule (reading: PDLP's): eta_bar = ||dz||_omega^2 / (2 |<dy, G~ dx>|),
// accept when eta <= eta_bar; eta' = min((1 - N^-a) eta_bar, (1 + N^-b) eta)
// with N = 1 + attempts so far.  Reflection parameter (reading): grows by
// beta_grow (capped at 1) while ||dz||_omega falls, else shrinks by beta_shrink.
// Runs on all threads of one workgroup; the partials of both passes are
// reduced in a fixed order, then thread 0 decides.  A halt takes effect in
// the next attempt (halt_next, copied to halt by the Halpern step).
__device__ void decide_body(DevState *__restrict__ st, const double *__restrict__ px, int64_t ntx,
                            const double *__restrict__ py, int64_t nty) {
    // four independent strided partial sums per thread keep four loads in
    // flight (the reduction is latency-bound); combined in a fixed order
    double a[4][3] = {};
    for (int64_t t = threadIdx.x; t < ntx; t += 4 * kBlock)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t q = t + u * kBlock;
            if (q < ntx) a[u][0] += px[q * kPartials + 0];
        }
    for (int64_t t = threadIdx.x; t < nty; t += 4 * kBlock)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t q = t + u * kBlock;
            if (q < nty) a[u][1] += py[q * kPartials + 0], a[u][2] += py[q * kPartials + 1];
        }
    double v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = (a[0][k] + a[1][k]) + (a[2][k] + a[3][k]);
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
        st->halt_next = 1;
        st->skip_update = 1;
        return;
    }
    const double nn = (double)(st->attempts_total + st->attempts_cur + 1);
    const double e1 = (1.0 - pow(nn, -st->step_reduce_exp)) * ebar;
    const double e2 = (1.0 + pow(nn, -st->step_grow_exp)) * eta;
    const bool fixed = st->step_mode == 1;   // fixed step: every attempt is accepted
    const double enew = fixed ? eta : (e1 < e2 ? e1 : e2);
    // replay: the other run's attempt count decides acceptance, its beta the branch
    const bool replay = st->n_iter < st->rp_count;
    const bool accept = fixed || (replay ? st->attempts_cur == st->rp_attempts[st->n_iter] : eta <= ebar);
    if (accept) {
        const double r = sqrt(omega * nx2 + ny2 / omega);
        double beta;
        if (st->beta_mode == 1) {
            beta = st->beta_const;
        } else {
            const bool grow = replay ? st->rp_beta[st->n_iter] >= st->beta_prev : r <= st->r_prev;
            beta = grow ? fmin(1.0, st->beta_grow * st->beta_prev) : st->beta_shrink * st->beta_prev;
        }
        st->r_prev = r;
        st->beta_prev = beta;
        st->beta = beta;
        const long long k = st->kin;
        st->ha = st->plain ? 1.0 : (double)(k + 1) / (double)(k + 2);
        st->hb = st->plain ? 0.0 : 1.0 / (double)(k + 2);
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
        if ((k + 1) % st->check_every == 0 || it + 1 >= st->max_iter) st->halt_next = 1;
    } else {
        st->eta = enew;
        st->skip_update = 1;
        if (st->attempts_cur >= st->max_attempts) {
            st->status = 3;
            st->halt_next = 1;
        }
    }
    st->tau = st->eta / st->omega;
    st->sigma = st->eta * st->omega;
}

// Instance b's decision from the per-instance tile ranges (a halted instance
// only marks its update skipped).
__device__ __forceinline__ void decide_instance(DevState *st, int64_t b, const double *px,
                                                const int64_t *tx, int64_t ntx, const double *py,
                                                const int64_t *ty, int64_t nty) {
    DevState *sb = st + b;
    if (sb->halt) {
        if (threadIdx.x == 0) sb->skip_update = 1;
        return;
    }
    const int64_t x0 = tx ? tx[b] : 0, x1 = tx ? tx[b + 1] : ntx;
    const int64_t y0 = ty ? ty[b] : 0, y1 = ty ? ty[b + 1] : nty;
    decide_body(sb, px + x0 * kPartials, x1 - x0, py + y0 * kPartials, y1 - y0);
}

}  // namespace pdcs
