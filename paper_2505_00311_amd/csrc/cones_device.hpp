// cones_device.hpp -- projections onto diagonally rescaled cones on gfx950.
//
//   exponential cone  : Section 3 Theorem 2 / Appendix A.2 Theorem 3, one thread
//                       per cone (the thread-wise strategy of Section 4, Table 3);
//   dual exponential  : Appendix A.2 Remark, Proj_{DK*}(v) = v + Proj_{D^-1 K}(-v);
//   second-order cone : Section 3 Theorem 1, an aligned group of 8..64 lanes per
//                       block for dims up to 256 (values in VGPRs, several
//                       blocks per wavefront) or one workgroup per block.
//
// The fourth case of Theorem 1 is solved in s = t / (1 - 2 lambda) on the
// bracket (max(t,0), ||(t,x)||], where g(s) = sum_i (x_i dh_i)^2 / (dh_i^2 + a)^2
// - s^2 with a = 1 - t/s is positive left of the root and negative right of it;
// a Newton step safeguarded by bisection converges in a handful of reductions.
#pragma once
#include "device_common.hpp"

namespace pdcs {

constexpr double kEps = 2.220446049250313e-16;
constexpr double kE = 2.718281828459045;

// ------------------------------------------------------------- exponential
__device__ __forceinline__ bool in_kexp(double r, double s, double t) {
    if (s > 0.0) return t >= s * exp(r / s);
    return s == 0.0 && t >= 0.0 && r <= 0.0;
}

__device__ __forceinline__ bool in_kexp_dual(double r, double s, double t) {
    if (r < 0.0) return kE * t >= -r * exp(s / r);
    return r == 0.0 && s >= 0.0 && t >= 0.0;
}

__device__ __forceinline__ double exp_flush(double x) { return fabs(x) < 0x1p-960 ? 0.0 : x; }

struct ExpPt {
    double r0, s0, t0, dr, ds, dt, tau, idr, idt;
};

// s_p(rho), r_d(rho) of eq. (sp_rd) with tau = ds / dr.
__device__ __forceinline__ void exp_sprd(const ExpPt &c, double rho, double &sp, double &rd) {
    const double den = rho * rho - rho + c.tau * c.tau;
    sp = (c.s0 * c.tau - c.r0 + c.r0 * rho) / (c.dr * den);
    rd = c.ds * (c.tau * c.r0 - rho * c.s0) / den;
}

// e^{-|rho|} h(rho) of eq. (h_rho) and its derivative: same sign and roots as
// h, no overflow for any rho.  One division per evaluation (1/den); 1/dr and
// 1/dt are the cone's.
__device__ __forceinline__ void exp_hs(const ExpPt &c, double rho, double &f, double &df) {
    const double den = rho * rho - rho + c.tau * c.tau;
    const double iden = 1.0 / den;
    const double ns = c.s0 * c.tau - c.r0 + c.r0 * rho;
    const double nr = c.tau * c.r0 - rho * c.s0;
    const double sp = ns * iden * c.idr;
    const double rd = c.ds * nr * iden;
    const double q = 2.0 * rho - 1.0;
    const double dsp = (c.r0 * den - ns * q) * (iden * iden) * c.idr;
    const double drd = c.ds * (-c.s0 * den - nr * q) * (iden * iden);
    if (rho >= 0.0) {
        const double em = exp(-rho);
        f = c.dt * sp - em * em * rd * c.idt - c.t0 * em;
        df = c.dt * dsp + em * em * (2.0 * rd - drd) * c.idt + c.t0 * em;
    } else {
        const double ep = exp(rho);
        f = c.dt * ep * ep * sp - rd * c.idt - c.t0 * ep;
        df = c.dt * ep * ep * (2.0 * sp + dsp) - drd * c.idt - c.t0 * ep;
    }
}

__device__ __forceinline__ double exp_hs_value(const ExpPt &c, double rho) {
    double f, df;
    exp_hs(c, rho, f, df);
    return f;
}

// Newton's method on the sign bracket [xneg, xpos] from `start` (the bracket's
// midpoint when start is not inside it), with a bisection step whenever Newton
// would leave the bracket, would not halve the step, or meets a non-finite
// value; stops at a step of 4 ulp of max(1, |rho|).
__device__ double exp_root(const ExpPt &c, double xneg, double xpos, double start) {
    double rho = (start >= fmin(xneg, xpos) && start <= fmax(xneg, xpos)) ? start : 0.5 * (xneg + xpos);
    double dxold = fabs(xpos - xneg), dx = dxold;
    bool vneg = false, vpos = false;   // an evaluation here has confirmed the end's sign
    double f, df;
    exp_hs(c, rho, f, df);
    for (int it = 0; it < 200; ++it) {
        if (f == 0.0) return rho;
        if (f < 0.0)
            xneg = rho, vneg = true;
        else
            xpos = rho, vpos = true;
        const bool finite = isfinite(f) && isfinite(df) && df != 0.0;
        const bool out = !finite || ((rho - xpos) * df - f) * ((rho - xneg) * df - f) > 0.0;
        const bool slow = !finite || fabs(2.0 * f) > fabs(dxold * df);
        if (out && finite) {
            // Newton aims past an end that no evaluation here has confirmed
            // (an end of the case-4 interval): when h has the wrong sign there,
            // the root is that end to rounding, which bisection would reach
            // one bit per step
            const double tgt = rho - f / df;
            if (!vpos && (tgt - xpos) * (xpos - xneg) >= 0.0) {
                vpos = true;
                if (!(exp_hs_value(c, xpos) > 0.0)) return xpos;
            } else if (!vneg && (tgt - xneg) * (xneg - xpos) >= 0.0) {
                vneg = true;
                if (!(exp_hs_value(c, xneg) < 0.0)) return xneg;
            }
        }
        dxold = dx;
        if (out || slow) {
            dx = 0.5 * (xpos - xneg);
            rho = xneg + dx;
        } else {
            dx = f / df;
            rho -= dx;
        }
        if (fabs(dx) <= 4.0 * kEps * fmax(1.0, fabs(rho))) return rho;
        exp_hs(c, rho, f, df);
    }
    return rho;
}

// Outward search from a guess g of the root inside [lo, hi], where h < 0 at lo
// and h > 0 at hi: steps of 2^-10 max(1, |g|), doubling, until h changes sign or
// an end is reached.  Leaves a sign bracket [xneg, xpos] around the root.
__device__ __forceinline__ void exp_local_bracket(const ExpPt &c, double g, double lo, double hi,
                                                  double &xneg, double &xpos) {
    const double fg = exp_hs_value(c, g);
    double step = 0x1p-10 * fmax(1.0, fabs(g));
    if (fg < 0.0) {
        xneg = g;
        xpos = fmin(g + step, hi);
        while (xpos < hi && !(exp_hs_value(c, xpos) > 0.0)) {
            xneg = xpos;
            step *= 2.0;
            xpos = fmin(g + step, hi);
        }
    } else {
        xpos = g;
        xneg = fmax(g - step, lo);
        while (xneg > lo && !(exp_hs_value(c, xneg) < 0.0)) {
            xpos = xneg;
            step *= 2.0;
            xneg = fmax(g - step, lo);
        }
    }
}

// Projection of (r0, s0, t0) onto diag(dr, ds, dt) K_exp.  `guess` (NaN for
// none) is a root of h from an earlier, nearby input: when it lies inside the
// case-4 interval the sign bracket is searched outward from it instead of
// from the interval's ends.  `rho_out` receives the root of a case-4
// projection and NaN otherwise.
__device__ void exp_project(double r0, double s0, double t0, double dr, double ds, double dt,
                            double &pr, double &ps, double &pt, double guess, double &rho_out) {
    rho_out = __builtin_nan("");
    // entries below 2^-960 are taken as 0: the case tests divide them by the
    // scales and the interval ends divide them by each other, and denormal
    // quotients misclassify the point or give 0/0 (zeroing moves the
    // projection by at most their size: it is nonexpansive)
    r0 = exp_flush(r0), s0 = exp_flush(s0), t0 = exp_flush(t0);
    if (in_kexp(r0 / dr, s0 / ds, t0 / dt)) {              // case 1
        pr = r0, ps = s0, pt = t0;
        return;
    }
    if (in_kexp_dual(-dr * r0, -ds * s0, -dt * t0)) {      // case 2 (polar)
        pr = ps = pt = 0.0;
        return;
    }
    if (r0 <= 0.0 && s0 <= 0.0) {                         // case 3
        pr = r0, ps = 0.0, pt = t0 > 0.0 ? t0 : 0.0;
        return;
    }
    // case 4: the bracket stays inside |rho| <= 700; an unbounded end is found
    // by doubling steps away from the finite one.  Beyond 700 the projection
    // is its limit to double precision: (0, 0, t0+) when a4 > 700 in case (iii),
    // (r0, s0, dt (s0/ds) e^a3) when a3 < -700 in case (ii).
    constexpr double R = 700.0;
    const ExpPt c{r0, s0, t0, dr, ds, dt, ds / dr, 1.0 / dr, 1.0 / dt};
    double xneg, xpos, lo, hi;   // [lo, hi]: the case-4 interval kept inside |rho| <= R
    int side;                    // 0: both ends finite, 1: (-inf, a3), 2: (a4, inf)
    // the ends from the ratios r0/s0 and s0/r0: with a denormal s0 or r0 the
    // product s0 dr (r0 dr) can round to 0 and 0/0 would give NaN
    const double tau = ds / dr;
    if (r0 > 0.0 && s0 > 0.0) {
        hi = fmin((r0 / s0) * tau, R);
        lo = fmax(1.0 - (s0 / r0) * tau, -R);
        side = 0;
    } else if (s0 > 0.0) {
        const double a3 = (r0 / s0) * tau;
        if (!(a3 >= -R)) {
            pr = r0, ps = s0, pt = dt * (s0 / ds) * exp(a3);
            return;
        }
        lo = -R, hi = a3, side = 1;
    } else {
        const double a4 = 1.0 - (s0 / r0) * tau;
        if (!(a4 <= R)) {
            pr = 0.0, ps = 0.0, pt = t0 > 0.0 ? t0 : 0.0;
            return;
        }
        lo = a4, hi = R, side = 2;
    }
    if (guess > lo && guess < hi) {
        exp_local_bracket(c, guess, lo, hi, xneg, xpos);
    } else if (side == 0) {
        xneg = lo, xpos = hi;
    } else if (side == 1) {
        xpos = hi;
        double step = 1.0;
        xneg = fmax(xpos - step, -R);
        while (!(exp_hs_value(c, xneg) < 0.0) && xneg > -R) {
            step *= 2.0;
            xneg = fmax(xpos - step, -R);
        }
    } else {
        xneg = lo;
        double step = 1.0;
        xpos = fmin(xneg + step, R);
        while (!(exp_hs_value(c, xpos) > 0.0) && xpos < R) {
            step *= 2.0;
            xpos = fmin(xneg + step, R);
        }
    }
    // Newton starts at the guess when there is one (its local bracket holds it)
    const double rho = exp_root(c, xneg, xpos, guess);
    rho_out = rho;
    // v_p = s_p w(rho), w = (dr rho, ds, dt e^rho); at the root v0 - v_p is
    // orthogonal to w, so s_p = <v0, w>/||w||^2 (projection of v0 onto the ray
    // of w), which avoids the cancellation of eq. (sp_rd) near a3 and a4; the
    // ray is scaled by e^-rho for rho > 0 so that nothing overflows.
    double w0, w1, w2;
    if (rho > 0.0) {
        const double em = exp(-rho);
        w0 = dr * rho * em, w1 = ds * em, w2 = dt;
    } else {
        w0 = dr * rho, w1 = ds, w2 = dt * exp(rho);
    }
    double cf = (r0 * w0 + s0 * w1 + t0 * w2) / (w0 * w0 + w1 * w1 + w2 * w2);
    if (!(cf > 0.0)) cf = 0.0;
    pr = cf * w0;
    ps = cf * w1;
    pt = cf * w2;
}

__device__ __forceinline__ void exp_dual_project(double r0, double s0, double t0, double dr,
                                                 double ds, double dt, double &pr, double &ps,
                                                 double &pt, double guess, double &rho_out) {
    double qr, qs, qt;
    exp_project(-r0, -s0, -t0, 1.0 / dr, 1.0 / ds, 1.0 / dt, qr, qs, qt, guess, rho_out);
    pr = r0 + qr, ps = s0 + qs, pt = t0 + qt;
}

// ------------------------------------------------------- second-order cone
// 1/x for finite nonzero x: the hardware estimate refined by two Newton steps
// for the reciprocal (e = 1 - x r, r += r e), each of which squares the
// estimate's relative error; four dependent FMAs after the estimate, against
// the longer sequence of an IEEE division.
__device__ __forceinline__ double nr_recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// A lane's partner value under a DPP pattern (CTRL), for a double.
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over an aligned group of LPB lanes (a power of two <= 64); every lane of
// the group receives the same bits, which keeps the lanes of a group on one
// path through the root finder.  Each stage adds a lane's value to that of its
// partner under an involution (lanes i and j = p(i) exchange), so both hold
// the same sum: within a row of 16 lanes by DPP (quad xor 1, quad xor 2, the
// half-row mirror i <-> 7 - i, the row mirror i <-> 15 - i), across rows by
// lane permutes (xor 16, xor 32).  That needs each exchange to add two rounded
// values: with contraction the compiler may fuse the caller's last product
// into the first exchange, fma(a, a, round(b*b)) in one lane against
// fma(b, b, round(a*a)) in its partner, and the two halves of the group then
// follow different Newton paths.  Contraction is therefore off for these adds.
template <int LPB>
__device__ __forceinline__ double group_sum(double v) {
#pragma clang fp contract(off)
    if (LPB >= 2) v = v + dpp_partner<0xB1>(v);    // quad_perm [1,0,3,2]
    if (LPB >= 4) v = v + dpp_partner<0x4E>(v);    // quad_perm [2,3,0,1]
    if (LPB >= 8) v = v + dpp_partner<0x141>(v);   // row_half_mirror
    if (LPB >= 16) v = v + dpp_partner<0x140>(v);  // row_mirror
    if (LPB >= 32) {
        const double o = __shfl_xor(v, 16, kWave);
        v = v + o;
    }
    if (LPB >= 64) {
        const double o = __shfl_xor(v, 32, kWave);
        v = v + o;
    }
    return v;
}

// soc_project_group below with D = I: the root of the last case of Theorem 1
// is s = (t + ||x||)/2 in closed form, and x is scaled by s/||x||.
template <int LPB, int R>
__device__ void soc_project_group_unit(int dim, const double (&v)[R], double (&p)[R],
                                       double &s_out) {
    s_out = __builtin_nan("");
    const int lane = threadIdx.x % kWave;
    const int g = lane % LPB;
    const double t = __shfl(v[0], lane - g, kWave);
    double snx = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = g + LPB * r;
        const double x = e >= 1 && e < dim ? v[r] : 0.0;
        snx += x * x;
    }
    const double nx = sqrt(group_sum<LPB>(snx));
    if (nx <= t) {                                        // case 2: inside
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] = v[r];
        return;
    }
    const bool polar = t <= 0.0 && nx <= -t;              // case 1: polar -> 0
    const double s = polar ? 0.0 : 0.5 * (t + nx), c = polar ? 0.0 : s / nx;
#pragma unroll
    for (int r = 0; r < R; ++r) p[r] = v[r] * c;
    if (g == 0) p[0] = s;
    if (!polar) s_out = s;
}

// One block per aligned group of LPB lanes; lane g of the group holds entries
// g + LPB r, r < R; entry 0 (t) is in the group's first lane.  Inactive slots
// carry v = 0, d = 1.  Several blocks share a wavefront when LPB < 64, so small
// cones need fewer exchange steps per reduction and keep more lanes busy.
template <int LPB, int R>
__device__ void soc_project_group(int dim, const double (&v)[R], const double (&d)[R],
                                  double (&p)[R], double s_guess, double &s_out) {
    s_out = __builtin_nan("");
    const int lane = threadIdx.x % kWave;
    const int g = lane % LPB;
    const int base = lane - g;
    const double t = __shfl(v[0], base, kWave);
    const double d0 = __shfl(d[0], base, kWave);
    double x[R], dh[R];
    double snd = 0.0, sndi = 0.0, snx = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = g + LPB * r;
        const bool on = e >= 1 && e < dim;
        x[r] = on ? v[r] : 0.0;
        dh[r] = on ? d[r] / d0 : 1.0;
        snd += (dh[r] * x[r]) * (dh[r] * x[r]);
        sndi += (x[r] / dh[r]) * (x[r] / dh[r]);
        snx += x[r] * x[r];
    }
    const double nd = sqrt(group_sum<LPB>(snd));
    const double ndi = sqrt(group_sum<LPB>(sndi));
    const double nx2 = group_sum<LPB>(snx);
    if (t <= 0.0 && nd <= -t) {                           // case 1: polar -> 0
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] = 0.0;
        return;
    }
    if (ndi <= t) {                                       // case 2: inside
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] = v[r];
        return;
    }
    if (t == 0.0) {                                       // case 3: lambda = 1/2
        double s2 = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double q = x[r] / (dh[r] + 1.0 / dh[r]);
            s2 += q * q;
            p[r] = x[r] / (1.0 + 1.0 / (dh[r] * dh[r]));
        }
        s2 = sqrt(group_sum<LPB>(s2));
        if (g == 0) p[0] = s2;
        return;
    }
    // case 4: root of g(s) on (max(t,0), ||(t,x)||]
    double w[R], h2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        w[r] = (x[r] * dh[r]) * (x[r] * dh[r]);
        h2[r] = dh[r] * dh[r];
    }
    const double lo = t > 0.0 ? t : 0.0, hi = sqrt(t * t + nx2);
    double xpos = lo, xneg = hi;                          // g > 0 at lo, g <= 0 at hi
    double s = 0.5 * (t + sqrt(nx2));
    if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
    if (s_guess > lo && s_guess < hi) s = s_guess;        // root of an earlier, nearby input
    double dxold = hi - lo, dx = dxold;
    auto eval = [&](double ss, double &f, double &df) {
        const double is = nr_recip(ss);
        const double a = 1.0 - t * is;
        double g1 = 0.0, g2 = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double iq = nr_recip(h2[r] + a);
            const double u = w[r] * iq * iq;
            g1 += u;
            g2 += u * iq;
        }
        g1 = group_sum<LPB>(g1);
        g2 = group_sum<LPB>(g2);
        f = g1 - ss * ss;
        df = -2.0 * (t * is * is) * g2 - 2.0 * ss;
    };
    double f, df;
    eval(s, f, df);
    for (int it = 0; it < 100; ++it) {
        if (f == 0.0) break;
        if (f > 0.0)
            xpos = s;
        else
            xneg = s;
        const bool finite = isfinite(f) && isfinite(df) && df != 0.0;
        const bool out = !finite || ((s - xpos) * df - f) * ((s - xneg) * df - f) > 0.0;
        const bool slow = !finite || fabs(2.0 * f) > fabs(dxold * df);
        dxold = dx;
        if (out || slow) {
            dx = 0.5 * (xneg - xpos);
            s = xpos + dx;
        } else {
            dx = f * nr_recip(df);
            s -= dx;
        }
        if (fabs(dx) <= 4.0 * kEps * s) break;
        eval(s, f, df);
    }
    const double a = 1.0 - t / s;
#pragma unroll
    for (int r = 0; r < R; ++r) p[r] = x[r] / (1.0 + a / h2[r]);
    if (g == 0) p[0] = s;
    s_out = s;
}

// ------------------------------------------ FP32 projections (mixed form)
// The mixed-precision form (not in the paper) may project the lane-group SOC
// blocks and the exponential cones in FP32 arithmetic: inputs are rounded to
// FP32, the norms, case tests and root search run in FP32, and the result is
// widened back.  FP64 stays where FP32 cannot be trusted: the exponential
// cone's case tests (membership of v0 and -D v0), its bracket ends, and every
// search that leaves the FP32 range or does not converge fall back to the FP64
// routines above on the same input.
constexpr float kEpsF = 1.1920929e-7f;

template <int CTRL>
__device__ __forceinline__ float dpp_partner_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// group_sum for FP32 values: the same involutions, one 32-bit exchange per stage
template <int LPB>
__device__ __forceinline__ float group_sum_f(float v) {
#pragma clang fp contract(off)
    if (LPB >= 2) v = v + dpp_partner_f<0xB1>(v);
    if (LPB >= 4) v = v + dpp_partner_f<0x4E>(v);
    if (LPB >= 8) v = v + dpp_partner_f<0x141>(v);
    if (LPB >= 16) v = v + dpp_partner_f<0x140>(v);
    if (LPB >= 32) {
        const float o = __shfl_xor(v, 16, kWave);
        v = v + o;
    }
    if (LPB >= 64) {
        const float o = __shfl_xor(v, 32, kWave);
        v = v + o;
    }
    return v;
}

// The FP64 routine as the FP32 one's fallback, kept out of line: inlined at
// every call site it would raise the FP32 pass kernels' register count for a
// path that rarely runs.
template <int LPB, int R>
__device__ __noinline__ void soc_project_group_fallback(int dim, const double (&v)[R],
                                                        const double (&d)[R], double (&p)[R],
                                                        double s_guess, double &s_out) {
    soc_project_group<LPB, R>(dim, v, d, p, s_guess, s_out);
}

// soc_project_group in FP32 arithmetic (same cases, bracket and safeguarded
// Newton search).  The FP64 routine takes over, for the whole group, when a
// search value leaves the FP32 range or the search does not settle within 60
// steps (both decisions are taken on group sums, so the group stays together).
template <int LPB, int R>
__device__ void soc_project_group_f(int dim, const double (&v)[R], const double (&d)[R],
                                    double (&p)[R], double s_guess, double &s_out) {
    s_out = __builtin_nan("");
    const int lane = threadIdx.x % kWave;
    const int g = lane % LPB;
    const int base = lane - g;
    const float t = (float)__shfl(v[0], base, kWave);
    const double d0 = __shfl(d[0], base, kWave);
    float x[R], dh[R];
    float snd = 0.0f, sndi = 0.0f, snx = 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = g + LPB * r;
        const bool on = e >= 1 && e < dim;
        x[r] = on ? (float)v[r] : 0.0f;
        dh[r] = on ? (float)(d[r] / d0) : 1.0f;
        snd += (dh[r] * x[r]) * (dh[r] * x[r]);
        sndi += (x[r] / dh[r]) * (x[r] / dh[r]);
        snx += x[r] * x[r];
    }
    const float nd = sqrtf(group_sum_f<LPB>(snd));
    const float ndi = sqrtf(group_sum_f<LPB>(sndi));
    const float nx2 = group_sum_f<LPB>(snx);
    if (!(isfinite(nd) && isfinite(ndi) && isfinite(nx2) && isfinite(t))) {
        soc_project_group_fallback<LPB, R>(dim, v, d, p, s_guess, s_out);
        return;
    }
    if (t <= 0.0f && nd <= -t) {
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] = 0.0;
        return;
    }
    if (ndi <= t) {
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] = v[r];
        return;
    }
    if (t == 0.0f) {
        float s2 = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float q = x[r] / (dh[r] + 1.0f / dh[r]);
            s2 += q * q;
            p[r] = (double)(x[r] / (1.0f + 1.0f / (dh[r] * dh[r])));
        }
        s2 = sqrtf(group_sum_f<LPB>(s2));
        if (g == 0) p[0] = (double)s2;
        return;
    }
    float w[R], h2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        w[r] = (x[r] * dh[r]) * (x[r] * dh[r]);
        h2[r] = dh[r] * dh[r];
    }
    const float lo = t > 0.0f ? t : 0.0f, hi = sqrtf(t * t + nx2);
    float xpos = lo, xneg = hi;
    float s = 0.5f * (t + sqrtf(nx2));
    if (!(s > lo && s < hi)) s = 0.5f * (lo + hi);
    const float sg = (float)s_guess;
    if (sg > lo && sg < hi) s = sg;
    float dxold = hi - lo, dx = dxold;
    auto eval = [&](float ss, float &f, float &df) {
        const float a = 1.0f - t / ss;
        float g1 = 0.0f, g2 = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float iq = 1.0f / (h2[r] + a);
            const float u = w[r] * iq * iq;
            g1 += u;
            g2 += u * iq;
        }
        g1 = group_sum_f<LPB>(g1);
        g2 = group_sum_f<LPB>(g2);
        f = g1 - ss * ss;
        df = -2.0f * (t / (ss * ss)) * g2 - 2.0f * ss;
    };
    float f, df;
    eval(s, f, df);
    bool settled = false;
    for (int it = 0; it < 60; ++it) {
        if (f == 0.0f) {
            settled = true;
            break;
        }
        if (f > 0.0f)
            xpos = s;
        else
            xneg = s;
        const bool finite = isfinite(f) && isfinite(df) && df != 0.0f;
        if (!finite) break;   // out of the FP32 range: FP64 below
        const bool out = ((s - xpos) * df - f) * ((s - xneg) * df - f) > 0.0f;
        const bool slow = fabsf(2.0f * f) > fabsf(dxold * df);
        dxold = dx;
        if (out || slow) {
            dx = 0.5f * (xneg - xpos);
            s = xpos + dx;
        } else {
            dx = f / df;
            s -= dx;
        }
        if (fabsf(dx) <= 4.0f * kEpsF * s) {
            settled = true;
            break;
        }
        eval(s, f, df);
    }
    if (!settled) {
        soc_project_group_fallback<LPB, R>(dim, v, d, p, s_guess, s_out);
        return;
    }
    const float a = 1.0f - t / s;
#pragma unroll
    for (int r = 0; r < R; ++r) p[r] = (double)(x[r] / (1.0f + a / h2[r]));
    if (g == 0) p[0] = (double)s;
    s_out = (double)s;
}

// e^{-|rho|} h(rho) and its derivative in FP32 (exp_hs in FP32 arithmetic).
struct ExpPtF {
    float r0, s0, t0, ds, dt, tau, idr, idt;
};

__device__ __forceinline__ void exp_hs_f(const ExpPtF &c, float rho, float &f, float &df) {
    const float den = rho * rho - rho + c.tau * c.tau;
    const float iden = 1.0f / den;
    const float ns = c.s0 * c.tau - c.r0 + c.r0 * rho;
    const float nr = c.tau * c.r0 - rho * c.s0;
    const float sp = ns * iden * c.idr;
    const float rd = c.ds * nr * iden;
    const float q = 2.0f * rho - 1.0f;
    const float dsp = (c.r0 * den - ns * q) * (iden * iden) * c.idr;
    const float drd = c.ds * (-c.s0 * den - nr * q) * (iden * iden);
    if (rho >= 0.0f) {
        const float em = expf(-rho);
        f = c.dt * sp - em * em * rd * c.idt - c.t0 * em;
        df = c.dt * dsp + em * em * (2.0f * rd - drd) * c.idt + c.t0 * em;
    } else {
        const float ep = expf(rho);
        f = c.dt * ep * ep * sp - rd * c.idt - c.t0 * ep;
        df = c.dt * ep * ep * (2.0f * sp + dsp) - drd * c.idt - c.t0 * ep;
    }
}

// The FP64 routine as the FP32 paths' fallback, kept out of line so that the
// rarely taken fallback does not add its registers to the FP32 path's.
__device__ __noinline__ void exp_project_fallback(double r0, double s0, double t0, double dr,
                                                  double ds, double dt, double &pr, double &ps,
                                                  double &pt, double guess, double &rho_out) {
    exp_project(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho_out);
}

// exp_project with the case-4 root search in FP32 when the search interval
// lies inside |rho| <= 40 (e^{-2|rho|} stays a normal FP32 number); the case
// tests, the interval, every other search and any FP32 search that does not
// settle within 60 steps are the FP64 routine's.
__device__ void exp_project_f(double r0, double s0, double t0, double dr, double ds, double dt,
                              double &pr, double &ps, double &pt, double guess, double &rho_out) {
    constexpr double RF = 40.0;
    r0 = exp_flush(r0), s0 = exp_flush(s0), t0 = exp_flush(t0);   // as exp_project
    const bool c4 = !in_kexp(r0 / dr, s0 / ds, t0 / dt) && !in_kexp_dual(-dr * r0, -ds * s0, -dt * t0) &&
                    !(r0 <= 0.0 && s0 <= 0.0);
    double lo = 0.0, hi = 0.0;
    bool fits = false;
    if (c4) {
        if (r0 > 0.0 && s0 > 0.0) {
            hi = (r0 / s0) * (ds / dr);
            lo = 1.0 - (s0 / r0) * (ds / dr);
            fits = lo >= -RF && hi <= RF;
        }
    }
    if (!fits) {   // cases 1-3, unbounded intervals, or beyond the FP32 range
        exp_project_fallback(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho_out);
        return;
    }
    const ExpPtF c{(float)r0, (float)s0, (float)t0, (float)ds, (float)dt, (float)(ds / dr),
                   (float)(1.0 / dr), (float)(1.0 / dt)};
    float xneg = (float)lo, xpos = (float)hi;
    float rho = (guess > lo && guess < hi) ? (float)guess : 0.5f * (xneg + xpos);
    if (!(rho >= fminf(xneg, xpos) && rho <= fmaxf(xneg, xpos))) rho = 0.5f * (xneg + xpos);
    float dxold = fabsf(xpos - xneg), dx = dxold;
    float f, df;
    exp_hs_f(c, rho, f, df);
    bool settled = false;
    for (int it = 0; it < 60; ++it) {
        if (f == 0.0f) {
            settled = true;
            break;
        }
        if (f < 0.0f)
            xneg = rho;
        else
            xpos = rho;
        const bool finite = isfinite(f) && isfinite(df) && df != 0.0f;
        if (!finite) break;
        const bool out = ((rho - xpos) * df - f) * ((rho - xneg) * df - f) > 0.0f;
        const bool slow = fabsf(2.0f * f) > fabsf(dxold * df);
        dxold = dx;
        if (out || slow) {
            dx = 0.5f * (xpos - xneg);
            rho = xneg + dx;
        } else {
            dx = f / df;
            rho -= dx;
        }
        if (fabsf(dx) <= 4.0f * kEpsF * fmaxf(1.0f, fabsf(rho))) {
            settled = true;
            break;
        }
        exp_hs_f(c, rho, f, df);
    }
    if (!settled) {
        exp_project_fallback(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho_out);
        return;
    }
    rho_out = (double)rho;
    // v_p = projection of v0 onto the ray w(rho), as in exp_project
    float w0, w1, w2;
    if (rho > 0.0f) {
        const float em = expf(-rho);
        w0 = (float)dr * rho * em, w1 = (float)ds * em, w2 = (float)dt;
    } else {
        w0 = (float)dr * rho, w1 = (float)ds, w2 = (float)dt * expf(rho);
    }
    float cf = (c.r0 * w0 + c.s0 * w1 + c.t0 * w2) / (w0 * w0 + w1 * w1 + w2 * w2);
    if (!(cf > 0.0f)) cf = 0.0f;
    const float qr = cf * w0, qs = cf * w1, qt = cf * w2;
    if (!(isfinite(qr) && isfinite(qs) && isfinite(qt))) {   // the ray left the FP32 range
        exp_project_fallback(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho_out);
        return;
    }
    pr = (double)qr;
    ps = (double)qs;
    pt = (double)qt;
}

__device__ __forceinline__ void exp_dual_project_f(double r0, double s0, double t0, double dr,
                                                   double ds, double dt, double &pr, double &ps,
                                                   double &pt, double guess, double &rho_out) {
    double qr, qs, qt;
    exp_project_f(-r0, -s0, -t0, 1.0 / dr, 1.0 / ds, 1.0 / dt, qr, qs, qt, guess, rho_out);
    pr = r0 + qr, ps = s0 + qs, pt = t0 + qt;
}

}  // namespace pdcs
