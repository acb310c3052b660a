/*
 * pdcs_oracle.c -- plain FP64 CPU oracle for PDCS (see pdcs_oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke entry point and the
 * benchmark's CPU-baseline leg, never by the GPU product path.
 *
 * Each function follows one passage of the paper:
 *   - cone projections: Section 3 Theorem 1 (scaled second-order cone) with its
 *     proof in Appendix A.1, Theorem 3 / Appendix A.2 (scaled exponential cone),
 *     the Remark of Appendix A.2 (scaled dual exponential cone), eq. (6) (blocks);
 *   - one PDHG step: Section 2.1 eq. (5);
 *   - the solver loop: Section 3 Algorithm 1 (adaptive step, reflection
 *     parameter, reflected Halpern step, weighted average, restart candidate,
 *     primal weight), on the diagonally rescaled problem of Section 3;
 *   - termination measures: Section 5 eq. (PDCS_terminate_tolerance).
 * Where the paper defers a rule to its companion technical note (step size,
 * reflection parameter, restart trigger, primal weight, rescaling scheme) the
 * code states the reading it takes next to the rule.  The tests pin those rules
 * to hand-worked examples of the readings; against the paper itself they are
 * parity unpinned (the paper does not state them).
 *
 * Vectors are handled whole, in the order the paper writes the steps; nothing
 * is fused, blocked or reordered.
 */
#include "pdcs_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

static double sq(double a) { return a * a; }

/* Timing mode.  With more than one thread the sparse products, the vector
 * passes and the cone blocks of the solver run in OpenMP parallel loops (the
 * reductions then add in another order); with one thread (the default) every
 * loop runs in order in the calling thread, the deterministic mode the parity
 * tests use.  The loops are the same in both modes: the `if` clause of each
 * parallel loop only decides whether a team is started. */
static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n > 1 ? n : 1; }
int orc_get_threads(void) { return g_threads; }
#define ORC_PAR _Pragma("omp parallel for if(g_threads > 1) num_threads(g_threads) schedule(static)")

/* ------------------------------------------------------------------------ */
/* Cone membership (definitions of K_exp and K_exp^* in Appendix A.2)        */
/* ------------------------------------------------------------------------ */
static int in_kexp(double r, double s, double t) {
    if (s > 0.0) return t >= s * exp(r / s);
    return s == 0.0 && t >= 0.0 && r <= 0.0;
}

static int in_kexp_dual(double r, double s, double t) {
    if (r < 0.0) return exp(1.0) * t >= -r * exp(s / r);
    return r == 0.0 && s >= 0.0 && t >= 0.0;
}

/* ------------------------------------------------------------------------ */
/* Theorem 1: projection of (t, x) onto D K_soc.                            */
/* dh_i = d_{i+1} / d_1.  The fourth case is solved for s = t / (1 - 2 lambda)  */
/* (reading: the s-form of eq. (bisection-soc)), by bisection on the finite  */
/* bracket (max(t,0), ||(t,x)||], on which g(s) = ||Dh^-1 y(s)||^2 - s^2     */
/* is positive left of the unique root and negative right of it.             */
/* ------------------------------------------------------------------------ */
static double soc_dhat(const double *d, int64_t i) { return d ? d[i + 1] / d[0] : 1.0; }

static double soc_g(double s, double t, int64_t nx, const double *x, const double *d) {
    double a = 1.0 - t / s; /* = 2 lambda */
    double acc = 0.0;
    for (int64_t i = 0; i < nx; ++i) {
        double dh = soc_dhat(d, i);
        double yi = x[i] / (1.0 + a / (dh * dh));
        acc += sq(yi / dh);
    }
    return acc - s * s;
}

int orc_proj_soc(int64_t dim, const double *v, const double *d, double *out) {
    double t = v[0];
    const double *x = v + 1;
    int64_t nx = dim - 1;
    double nd = 0.0, ndi = 0.0, nx2 = 0.0;
    for (int64_t i = 0; i < nx; ++i) {
        double dh = soc_dhat(d, i);
        nd += sq(dh * x[i]);
        ndi += sq(x[i] / dh);
        nx2 += sq(x[i]);
    }
    nd = sqrt(nd);
    ndi = sqrt(ndi);
    /* case 1: -(t,x) in the dual cone D^-1 K_soc -> origin */
    if (t <= 0.0 && nd <= -t) {
        for (int64_t i = 0; i < dim; ++i) out[i] = 0.0;
        return 1;
    }
    /* case 2: already inside D K_soc */
    if (ndi <= t) {
        for (int64_t i = 0; i < dim; ++i) out[i] = v[i];
        return 2;
    }
    /* case 3: t == 0, lambda = 1/2 closed form */
    if (t == 0.0) {
        double s2 = 0.0;
        for (int64_t i = 0; i < nx; ++i) {
            double dh = soc_dhat(d, i);
            out[i + 1] = x[i] / (1.0 + 1.0 / (dh * dh));
            s2 += sq(x[i] / (dh + 1.0 / dh));
        }
        out[0] = sqrt(s2);
        return 3;
    }
    /* case 4: root of the univariate equation */
    double lo = t > 0.0 ? t : 0.0;
    double hi = sqrt(t * t + nx2);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (soc_g(mid, t, nx, x, d) > 0.0)
            lo = mid;
        else
            hi = mid;
    }
    double s = 0.5 * (lo + hi);
    double a = 1.0 - t / s;
    out[0] = s;
    for (int64_t i = 0; i < nx; ++i) {
        double dh = soc_dhat(d, i);
        out[i + 1] = x[i] / (1.0 + a / (dh * dh));
    }
    return 4;
}

/* ------------------------------------------------------------------------ */
/* Theorem 3: projection of v0 = (r0, s0, t0) onto D K_exp, D = diag(dr,ds,dt) */
/* ------------------------------------------------------------------------ */
typedef struct {
    double r0, s0, t0, dr, ds, dt, tau;
} exp_ctx;

/* s_p(rho), r_d(rho) of eq. (sp_rd), written with tau = ds/dr (proof of Lemma 2). */
static void exp_sp_rd(const exp_ctx *c, double rho, double *sp, double *rd) {
    double den = rho * rho - rho + c->tau * c->tau;
    *sp = (c->s0 * c->tau - c->r0 + c->r0 * rho) / (c->dr * den);
    *rd = c->ds * (c->tau * c->r0 - rho * c->s0) / den;
}

/* h(rho) of eq. (h_rho) multiplied by exp(-|rho|) > 0.  The product has the sign
 * and the roots of h but never overflows, so the same code handles brackets far
 * beyond |rho| = 709 (reading: the paper does not say how to evaluate h there). */
static double exp_hs(const exp_ctx *c, double rho) {
    double sp, rd;
    exp_sp_rd(c, rho, &sp, &rd);
    if (rho >= 0.0) {
        double em = exp(-rho);
        return c->dt * sp - em * em * rd / c->dt - c->t0 * em;
    }
    double ep = exp(rho);
    return c->dt * ep * ep * sp - rd / c->dt - c->t0 * ep;
}

/* derivative of exp_hs */
static double exp_dhs(const exp_ctx *c, double rho) {
    double den = rho * rho - rho + c->tau * c->tau;
    double ns = c->s0 * c->tau - c->r0 + c->r0 * rho;
    double nr = c->tau * c->r0 - rho * c->s0;
    double sp = ns / (c->dr * den);
    double rd = c->ds * nr / den;
    double dsp = (c->r0 * den - ns * (2.0 * rho - 1.0)) / (c->dr * den * den);
    double drd = c->ds * (-c->s0 * den - nr * (2.0 * rho - 1.0)) / (den * den);
    if (rho >= 0.0) {
        double em = exp(-rho);
        return c->dt * dsp + em * em * (2.0 * rd - drd) / c->dt + c->t0 * em;
    }
    double ep = exp(rho);
    return c->dt * ep * ep * (2.0 * sp + dsp) - drd / c->dt - c->t0 * ep;
}

/* Root of h between xneg (h < 0) and xpos (h > 0): Newton's method safeguarded by
 * bisection (the Newton-bisection hybrid of Press et al., "rtsafe"): a bisection
 * step replaces Newton's whenever Newton would leave the sign bracket, would not
 * halve the step, or meets a non-finite value.  Stops when the step falls to
 * 4 ulp of max(1,|rho|), when the function is exactly zero, or after 200 steps
 * (reading: the paper leaves the root-finder open). */
static double exp_root(const exp_ctx *c, double xneg, double xpos) {
    double rho = 0.5 * (xneg + xpos);
    double dxold = fabs(xpos - xneg), dx = dxold;
    double f = exp_hs(c, rho), df = exp_dhs(c, rho);
    for (int it = 0; it < 200; ++it) {
        if (f == 0.0) return rho;
        if (f < 0.0)
            xneg = rho;
        else
            xpos = rho;
        int finite = isfinite(f) && isfinite(df) && df != 0.0;
        int newton_out = !finite || ((rho - xpos) * df - f) * ((rho - xneg) * df - f) > 0.0;
        int newton_slow = !finite || fabs(2.0 * f) > fabs(dxold * df);
        if (newton_out || newton_slow) {
            dxold = dx;
            dx = 0.5 * (xpos - xneg);
            rho = xneg + dx;
        } else {
            dxold = dx;
            dx = f / df;
            rho -= dx;
        }
        if (fabs(dx) <= 4.0 * DBL_EPSILON * fmax(1.0, fabs(rho))) return rho;
        f = exp_hs(c, rho);
        df = exp_dhs(c, rho);
    }
    return rho;
}

/* Reading (floating point, not in the paper): entries below 2^-960 in magnitude
 * are taken as 0.  The case tests divide the entries by the scales and the
 * interval ends divide entries by entries; with denormal entries those
 * quotients round to 0 and misclassify the point (or give 0/0).  Zeroing them
 * moves the projection by at most their size (a projection onto a closed
 * convex set is nonexpansive). */
static double exp_flush(double x) { return fabs(x) < 0x1p-960 ? 0.0 : x; }

int orc_proj_exp(const double *v, const double *d, double *out) {
    double r0 = exp_flush(v[0]), s0 = exp_flush(v[1]), t0 = exp_flush(v[2]);
    double dr = d ? d[0] : 1.0, ds = d ? d[1] : 1.0, dt = d ? d[2] : 1.0;
    /* case 1: v0 in D K_exp, i.e. D^-1 v0 in K_exp */
    if (in_kexp(r0 / dr, s0 / ds, t0 / dt)) {
        out[0] = r0, out[1] = s0, out[2] = t0;
        return 1;
    }
    /* case 2: v0 in the polar cone -D^-1 K_exp^*, i.e. -D v0 in K_exp^* */
    if (in_kexp_dual(-dr * r0, -ds * s0, -dt * t0)) {
        out[0] = out[1] = out[2] = 0.0;
        return 2;
    }
    /* case 3 */
    if (r0 <= 0.0 && s0 <= 0.0) {
        out[0] = r0, out[1] = 0.0, out[2] = t0 > 0.0 ? t0 : 0.0;
        return 3;
    }
    /* case 4: root of h on (l_rho, u_rho), eq. (lrho_urho); h(a3) > 0, h(a4) < 0.
     * Reading for the unbounded and the far ends: the bracket is kept inside
     * |rho| <= 700.  An unbounded end is found by stepping away from the finite
     * one by 1, 2, 4, ... until h changes sign.  In case (iii) with a4 > 700 the
     * root lies beyond a4, where s_p ~ e^-rho t0 / dt, so the projection equals
     * its limit (0, 0, t0^+) to double precision; in case (ii) with a3 < -700
     * it equals (r0, s0, dt (s0/ds) e^a3). */
    const double R = 700.0;
    exp_ctx c = {r0, s0, t0, dr, ds, dt, ds / dr};
    double xneg, xpos;
    /* a3 = (r0/s0)(ds/dr), a4 = 1 - (s0/r0)(ds/dr) as ratios: the products
     * s0 dr and r0 dr round to 0 for denormal s0 or r0, and 0/0 is NaN */
    if (r0 > 0.0 && s0 > 0.0) {
        xpos = fmin((r0 / s0) * c.tau, R);
        xneg = fmax(1.0 - (s0 / r0) * c.tau, -R);
    } else if (s0 > 0.0) { /* r0 <= 0: (-inf, a3) */
        double a3 = (r0 / s0) * c.tau;
        if (!(a3 >= -R)) {
            out[0] = r0, out[1] = s0, out[2] = dt * (s0 / ds) * exp(a3);
            return 4;
        }
        xpos = a3;
        double step = 1.0;
        xneg = fmax(xpos - step, -R);
        while (!(exp_hs(&c, xneg) < 0.0) && xneg > -R) {
            step *= 2.0;
            xneg = fmax(xpos - step, -R);
        }
    } else { /* r0 > 0, s0 <= 0: (a4, inf) */
        double a4 = 1.0 - (s0 / r0) * c.tau;
        if (!(a4 <= R)) {
            out[0] = 0.0, out[1] = 0.0, out[2] = t0 > 0.0 ? t0 : 0.0;
            return 4;
        }
        xneg = a4;
        double step = 1.0;
        xpos = fmin(xneg + step, R);
        while (!(exp_hs(&c, xpos) > 0.0) && xpos < R) {
            step *= 2.0;
            xpos = fmin(xneg + step, R);
        }
    }
    double rho = exp_root(&c, xneg, xpos);
    /* eq. (vpvd_defn): v_p = s_p w(rho), w = (dr rho, ds, dt e^rho).  At the root
     * v_d = v0 - v_p is orthogonal to w (Step 1 of the proof of Theorem 3), so
     * s_p = <v0, w> / ||w||^2: the projection of v0 onto the ray of w.  Evaluated
     * this way (reading) v_p carries an absolute error of order eps ||v0||,
     * where the closed form of eq. (sp_rd) cancels near a3 or a4; for rho > 0
     * the ray is scaled by e^-rho so that nothing overflows. */
    double w0, w1, w2;
    if (rho > 0.0) {
        double em = exp(-rho);
        w0 = dr * rho * em, w1 = ds * em, w2 = dt;
    } else {
        w0 = dr * rho, w1 = ds, w2 = dt * exp(rho);
    }
    double cf = (r0 * w0 + s0 * w1 + t0 * w2) / (w0 * w0 + w1 * w1 + w2 * w2);
    if (!(cf > 0.0)) cf = 0.0;
    out[0] = cf * w0;
    out[1] = cf * w1;
    out[2] = cf * w2;
    return 4;
}

/* Remark of Appendix A.2: Proj_{D K_exp^*}(v0) = v0 + Proj_{D^-1 K_exp}(-v0). */
int orc_proj_exp_dual(const double *v, const double *d, double *out) {
    double mv[3] = {-v[0], -v[1], -v[2]};
    double di[3] = {1.0, 1.0, 1.0};
    if (d) di[0] = 1.0 / d[0], di[1] = 1.0 / d[1], di[2] = 1.0 / d[2];
    double p[3];
    int cs = orc_proj_exp(mv, di, p);
    for (int i = 0; i < 3; ++i) out[i] = v[i] + p[i];
    return cs;
}

/* ------------------------------------------------------------------------ */
/* Eq. (6): a product of cones is projected block by block.                  */
/* ------------------------------------------------------------------------ */
static int dual_type(int t) {
    switch (t) {
    case ORC_ZERO: return ORC_FREE;
    case ORC_FREE: return ORC_ZERO;
    case ORC_EXP: return ORC_EXP_DUAL;
    case ORC_EXP_DUAL: return ORC_EXP;
    default: return t; /* R_+ and the second-order cone are self-dual */
    }
}

void orc_proj_blocks(int64_t nblk, const int32_t *type, const int64_t *dim, int dual,
                     const double *d, double *v) {
    int64_t *offs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nblk > 0 ? nblk : 1));
    int64_t off = 0;
    for (int64_t b = 0; b < nblk; ++b) offs[b] = off, off += dim[b];
#pragma omp parallel for if(g_threads > 1) num_threads(g_threads) schedule(dynamic, 256)
    for (int64_t b = 0; b < nblk; ++b) {
        int t = dual ? dual_type(type[b]) : type[b];
        int64_t k = dim[b];
        double *vb = v + offs[b];
        const double *db = d ? d + offs[b] : NULL;
        double tmp[3];
        switch (t) {
        case ORC_ZERO:
            for (int64_t i = 0; i < k; ++i) vb[i] = 0.0;
            break;
        case ORC_FREE: break;
        case ORC_NONNEG: /* positive diagonal scaling leaves R_+ unchanged */
            for (int64_t i = 0; i < k; ++i) vb[i] = vb[i] > 0.0 ? vb[i] : 0.0;
            break;
        case ORC_SOC: {
            double *o = (double *)malloc(sizeof(double) * (size_t)k);
            orc_proj_soc(k, vb, db, o);
            memcpy(vb, o, sizeof(double) * (size_t)k);
            free(o);
            break;
        }
        case ORC_EXP:
            orc_proj_exp(vb, db, tmp);
            memcpy(vb, tmp, sizeof tmp);
            break;
        case ORC_EXP_DUAL:
            orc_proj_exp_dual(vb, db, tmp);
            memcpy(vb, tmp, sizeof tmp);
            break;
        }
    }
    free(offs);
}

/* ------------------------------------------------------------------------ */
/* Sparse matrix helpers (plain definitions)                                 */
/* ------------------------------------------------------------------------ */
static void spmv(int64_t rows, const int64_t *rp, const int32_t *ci, const double *v,
                 const double *x, double *y) {
#pragma omp parallel for if(g_threads > 1) num_threads(g_threads) schedule(dynamic, 1024)
    for (int64_t i = 0; i < rows; ++i) {
        double acc = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc += v[k] * x[ci[k]];
        y[i] = acc;
    }
}

/* CSR of the transpose; entries of each column keep increasing row order. */
static void transpose(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                      int64_t *trp, int32_t *tci, double *tv) {
    for (int64_t j = 0; j <= n; ++j) trp[j] = 0;
    for (int64_t k = 0; k < rp[m]; ++k) trp[ci[k] + 1]++;
    for (int64_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) next[j] = trp[j];
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t p = next[ci[k]]++;
            tci[p] = (int32_t)i;
            tv[p] = v[k];
        }
    free(next);
}

void orc_spmv(int64_t rows, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
              double *y) {
    spmv(rows, rp, ci, v, x, y);
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for if(g_threads > 1) num_threads(g_threads) schedule(static) reduction(+:s)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2sq(int64_t n, const double *a) { return dot(n, a, a); }

static double nrminf(int64_t n, const double *a) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = fmax(s, fabs(a[i]));
    return s;
}

/* ------------------------------------------------------------------------ */
/* Problem checks                                                            */
/* ------------------------------------------------------------------------ */
static int valid_problem(const orc_problem *p) {
    if (p->n < 0 || p->m < 0 || p->n_box < 0 || p->n_box > p->n) return -1;
    if (p->row_ptr[0] != 0 || p->row_ptr[p->m] != p->nnz) return -1;
    int64_t sx = 0, sr = 0;
    for (int64_t b = 0; b < p->n_xcones; ++b) {
        if (p->xcone_type[b] < ORC_ZERO || p->xcone_type[b] > ORC_EXP_DUAL) return -3;
        if (p->xcone_dim[b] < 1) return -2;
        if ((p->xcone_type[b] == ORC_EXP || p->xcone_type[b] == ORC_EXP_DUAL) &&
            p->xcone_dim[b] != 3)
            return -2;
        sx += p->xcone_dim[b];
    }
    for (int64_t b = 0; b < p->n_rcones; ++b) {
        if (p->rcone_type[b] < ORC_ZERO || p->rcone_type[b] > ORC_EXP_DUAL) return -3;
        if (p->rcone_dim[b] < 1) return -2;
        if ((p->rcone_type[b] == ORC_EXP || p->rcone_type[b] == ORC_EXP_DUAL) &&
            p->rcone_dim[b] != 3)
            return -2;
        sr += p->rcone_dim[b];
    }
    if (sx != p->n - p->n_box || sr != p->m) return -2;
    for (int64_t k = 0; k < p->nnz; ++k)
        if (p->col[k] < 0 || p->col[k] >= p->n) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagonal rescaling (Section 3).  Reading: 10 Ruiz infinity-norm passes    */
/* then one Pock-Chambolle pass with alpha = 1; an empty row or column keeps */
/* its factor.  G~ = E G F.                                                  */
/* ------------------------------------------------------------------------ */
int orc_scaling(const orc_problem *p, const orc_settings *s, double *e, double *f) {
    int64_t m = p->m, n = p->n;
    double *rs = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    double *cs = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t i = 0; i < m; ++i) e[i] = 1.0;
    for (int64_t j = 0; j < n; ++j) f[j] = 1.0;
    for (int it = 0; it < s->ruiz_iters; ++it) {
        for (int64_t i = 0; i < m; ++i) rs[i] = 0.0;
        for (int64_t j = 0; j < n; ++j) cs[j] = 0.0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t k = p->row_ptr[i]; k < p->row_ptr[i + 1]; ++k) {
                double a = fabs(e[i] * p->val[k] * f[p->col[k]]);
                rs[i] = fmax(rs[i], a);
                cs[p->col[k]] = fmax(cs[p->col[k]], a);
            }
        for (int64_t i = 0; i < m; ++i)
            if (rs[i] > 0.0) e[i] /= sqrt(rs[i]);
        for (int64_t j = 0; j < n; ++j)
            if (cs[j] > 0.0) f[j] /= sqrt(cs[j]);
    }
    if (s->pock_chambolle) {
        for (int64_t i = 0; i < m; ++i) rs[i] = 0.0;
        for (int64_t j = 0; j < n; ++j) cs[j] = 0.0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t k = p->row_ptr[i]; k < p->row_ptr[i + 1]; ++k) {
                double a = fabs(e[i] * p->val[k] * f[p->col[k]]);
                rs[i] += a;
                cs[p->col[k]] += a;
            }
        for (int64_t i = 0; i < m; ++i)
            if (rs[i] > 0.0) e[i] /= sqrt(rs[i]);
        for (int64_t j = 0; j < n; ++j)
            if (cs[j] > 0.0) f[j] /= sqrt(cs[j]);
    }
    free(rs);
    free(cs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Termination measures, eq. (PDCS_terminate_tolerance), unscaled space.     */
/* Reading: lambda_1 enters the dual objective through Proj_Lambda(lambda_1) */
/* so that infinite bounds never multiply a nonzero.                         */
/* ------------------------------------------------------------------------ */
static double proj_lambda(double lam, double l, double u) {
    int lf = isfinite(l), uf = isfinite(u);
    if (!lf && !uf) return 0.0;          /* {0}  */
    if (!lf) return lam < 0.0 ? lam : 0.0; /* R^-  */
    if (!uf) return lam > 0.0 ? lam : 0.0; /* R^+  */
    return lam;                          /* R    */
}

int orc_kkt(const orc_problem *p, const double *x, const double *y, double *err_p,
            double *err_d, double *err_gap, double *pobj, double *dobj) {
    int64_t n = p->n, m = p->m, nb = p->n_box;
    double *gx = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *r = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *gty = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *lam = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    /* primal residual: (Gx - h) - Proj_{K_d^*}(Gx - h) */
    spmv(m, p->row_ptr, p->col, p->val, x, gx);
    for (int64_t i = 0; i < m; ++i) r[i] = gx[i] - p->h[i];
    double *pr = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    memcpy(pr, r, sizeof(double) * (size_t)m);
    orc_proj_blocks(p->n_rcones, p->rcone_type, p->rcone_dim, 0, NULL, pr);
    double num_p = 0.0;
    for (int64_t i = 0; i < m; ++i) num_p = fmax(num_p, fabs(r[i] - pr[i]));
    *err_p = num_p / (1.0 + fmax(nrminf(m, p->h), fmax(nrminf(m, gx), nrminf(m, pr))));
    /* dual residual: lambda = c - G^T y */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = p->row_ptr[i]; k < p->row_ptr[i + 1]; ++k)
            gty[p->col[k]] += p->val[k] * y[i];
    for (int64_t j = 0; j < n; ++j) lam[j] = p->c[j] - gty[j];
    double num_d = 0.0;
    for (int64_t j = 0; j < nb; ++j)
        num_d = fmax(num_d, fabs(lam[j] - proj_lambda(lam[j], p->l[j], p->u[j])));
    double *pl = (double *)malloc(sizeof(double) * (size_t)(n - nb > 0 ? n - nb : 1));
    memcpy(pl, lam + nb, sizeof(double) * (size_t)(n - nb));
    orc_proj_blocks(p->n_xcones, p->xcone_type, p->xcone_dim, 1, NULL, pl);
    for (int64_t j = nb; j < n; ++j) num_d = fmax(num_d, fabs(lam[j] - pl[j - nb]));
    *err_d = num_d / (1.0 + fmax(nrminf(n, p->c), nrminf(n, gty)));
    /* gap */
    double po = dot(n, p->c, x);
    double dob = dot(m, y, p->h);
    for (int64_t j = 0; j < nb; ++j) {
        double lp = proj_lambda(lam[j], p->l[j], p->u[j]);
        if (lp > 0.0) dob += p->l[j] * lp;
        if (lp < 0.0) dob -= p->u[j] * (-lp);
    }
    *err_gap = fabs(po - dob) / (1.0 + fmax(fabs(po), fabs(dob)));
    if (pobj) *pobj = po;
    if (dobj) *dobj = dob;
    free(gx), free(r), free(gty), free(lam), free(pr), free(pl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* eq. (5) on the unscaled problem, for hand-checked examples.               */
/* ------------------------------------------------------------------------ */
static void proj_x(const orc_problem *p, const double *l, const double *u, const double *d,
                   double *x) {
    ORC_PAR
    for (int64_t j = 0; j < p->n_box; ++j) x[j] = fmin(fmax(x[j], l[j]), u[j]);
    orc_proj_blocks(p->n_xcones, p->xcone_type, p->xcone_dim, 0, d ? d + p->n_box : NULL,
                    x + p->n_box);
}

static void proj_y(const orc_problem *p, const double *d, double *y) {
    /* y lies in K_d, the dual of the row cones */
    orc_proj_blocks(p->n_rcones, p->rcone_type, p->rcone_dim, 1, d, y);
}

int orc_onepdhg(const orc_problem *p, const double *x, const double *y, double tau,
                double sigma, double *xh, double *yh) {
    int64_t n = p->n, m = p->m;
    double *gty = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *xt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *g = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = p->row_ptr[i]; k < p->row_ptr[i + 1]; ++k)
            gty[p->col[k]] += p->val[k] * y[i];
    for (int64_t j = 0; j < n; ++j) xh[j] = x[j] - tau * (p->c[j] - gty[j]);
    proj_x(p, p->l, p->u, NULL, xh);
    for (int64_t j = 0; j < n; ++j) xt[j] = 2.0 * xh[j] - x[j];
    spmv(m, p->row_ptr, p->col, p->val, xt, g);
    for (int64_t i = 0; i < m; ++i) yh[i] = y[i] + sigma * (p->h[i] - g[i]);
    proj_y(p, NULL, yh);
    free(gty), free(xt), free(g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 on the rescaled problem.                                      */
/* ------------------------------------------------------------------------ */
void orc_settings_default(orc_settings *s) {
    s->tol = 1e-6;
    s->max_iter = 1000000;
    s->check_every = 64;
    s->ruiz_iters = 10;
    s->pock_chambolle = 1;
    s->beta_mode = 0;
    s->beta_const = 1.0;
    s->beta_grow = 1.25;
    s->beta_shrink = 0.5;
    s->step_reduce_exp = 0.3;
    s->step_grow_exp = 0.6;
    s->restart_sufficient = 0.2;
    s->restart_necessary = 0.8;
    s->restart_artificial = 0.36;
    s->max_attempts = 64;
    s->step_mode = 0;
    s->step_fixed = 0.9;
    s->power_iters = 100;
    s->plain_pdhg = 0;
}

typedef struct {
    double err_p, err_d, err_gap, pobj, dobj;
} kkt_t;

/* Relative distance of a deciding quantity a from its threshold b (a
 * decision log entry; 0 means a tie, +inf when both are infinite). */
static double rel_margin(double a, double b) {
    double d = fabs(a - b), s = fmax(fabs(a), fabs(b));
    return s > 0.0 && d == d ? d / s : (a == b ? 0.0 : INFINITY);
}

static double kkt_avg(const kkt_t *k) { return (k->err_p + k->err_d + k->err_gap) / 3.0; }
static double kkt_max(const kkt_t *k) { return fmax(k->err_p, fmax(k->err_d, k->err_gap)); }

/* KKT of a scaled point, measured after unscaling x = F x~, y = E y~. */
static void kkt_scaled(const orc_problem *p, const double *e, const double *f, const double *xs,
                       const double *ys, double *xu, double *yu, kkt_t *k) {
    for (int64_t j = 0; j < p->n; ++j) xu[j] = f[j] * xs[j];
    for (int64_t i = 0; i < p->m; ++i) yu[i] = e[i] * ys[i];
    orc_kkt(p, xu, yu, &k->err_p, &k->err_d, &k->err_gap, &k->pobj, &k->dobj);
}

#define ALLOC(T, k) ((T *)calloc((size_t)((k) > 0 ? (k) : 1), sizeof(T)))

int orc_solve(const orc_problem *p, const orc_settings *s, const double *x0, const double *y0,
              double omega0, double *x_out, double *y_out, orc_info *info, orc_trace *tr) {
    int rc = valid_problem(p);
    if (rc) return rc;
    int64_t n = p->n, m = p->m, nb = p->n_box, nnz = p->nnz;
    memset(info, 0, sizeof *info);
    if (tr) tr->count = 0;

    /* --- rescaled problem: G~ = E G F, c~ = F c, h~ = E h, [l/f, u/f] --- */
    double *e = ALLOC(double, m), *f = ALLOC(double, n);
    orc_scaling(p, s, e, f);
    double *gv = ALLOC(double, nnz);
    double gmax = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = p->row_ptr[i]; k < p->row_ptr[i + 1]; ++k) {
            gv[k] = e[i] * p->val[k] * f[p->col[k]];
            gmax = fmax(gmax, fabs(gv[k]));
        }
    int64_t *trp = ALLOC(int64_t, n + 1);
    int32_t *tci = ALLOC(int32_t, nnz);
    double *tv = ALLOC(double, nnz);
    transpose(m, n, p->row_ptr, p->col, gv, trp, tci, tv);
    double *cs = ALLOC(double, n), *hs = ALLOC(double, m);
    double *ls = ALLOC(double, nb), *us = ALLOC(double, nb);
    double *dx = ALLOC(double, n), *dy = ALLOC(double, m);
    for (int64_t j = 0; j < n; ++j) cs[j] = f[j] * p->c[j], dx[j] = 1.0 / f[j];
    for (int64_t i = 0; i < m; ++i) hs[i] = e[i] * p->h[i], dy[i] = 1.0 / e[i];
    for (int64_t j = 0; j < nb; ++j) ls[j] = p->l[j] / f[j], us[j] = p->u[j] / f[j];
    /* The scaled feasible sets are F^-1 K_p and E^-1 K_d: D = F^-1, E^-1. */

    /* --- initial step size and primal weight (readings) --- */
    double eta = gmax > 0.0 ? 1.0 / gmax : 1.0;
    const int plain = s->plain_pdhg == 1;
    if (s->step_mode == 1 || plain) {
        /* fixed step step_fixed / ||G~||_2, the norm by power iteration on
         * G~^T G~ from the normalised all-ones vector */
        double *pv = ALLOC(double, n), *pu = ALLOC(double, m), *pw = ALLOC(double, n);
        for (int64_t j = 0; j < n; ++j) pv[j] = 1.0 / sqrt((double)n);
        double lam = 0.0;
        for (int it = 0; it < s->power_iters; ++it) {
            spmv(m, p->row_ptr, p->col, gv, pv, pu);
            spmv(n, trp, tci, tv, pu, pw);
            lam = sqrt(nrm2sq(n, pw));
            if (!(lam > 0.0)) break;
            for (int64_t j = 0; j < n; ++j) pv[j] = pw[j] / lam;
        }
        eta = lam > 0.0 ? s->step_fixed / sqrt(lam) : 1.0;
        free(pv), free(pu), free(pw);
    }
    double omega;
    {
        double nc = sqrt(nrm2sq(n, cs)), nh = sqrt(nrm2sq(m, hs));
        omega = (nc > 1e-10 && nh > 1e-10) ? nc / nh : 1.0;
        if (plain) omega = 1.0;   /* the baseline takes the same step on both sides */
        if (omega0 > 0.0) omega = omega0;
    }

    /* --- state --- */
    double *x = ALLOC(double, n), *y = ALLOC(double, m);
    double *xa = ALLOC(double, n), *ya = ALLOC(double, m);
    double *xh = ALLOC(double, n), *yh = ALLOC(double, m);
    double *gty = ALLOC(double, n), *xt = ALLOC(double, n), *gxt = ALLOC(double, m);
    double *ddx = ALLOC(double, n), *ddy = ALLOC(double, m), *gdx = ALLOC(double, m);
    double *xsum = ALLOC(double, n), *ysum = ALLOC(double, m);
    double *xc1 = ALLOC(double, n), *yc1 = ALLOC(double, m);
    double *xc2 = ALLOC(double, n), *yc2 = ALLOC(double, m);
    double *xu = ALLOC(double, n), *yu = ALLOC(double, m);

    /* z^{0,0}: the (mapped) starting point, projected onto X x Y (reading) */
    for (int64_t j = 0; j < n; ++j) x[j] = x0 ? x0[j] / f[j] : 0.0;
    for (int64_t i = 0; i < m; ++i) y[i] = y0 ? y0[i] / e[i] : 0.0;
    proj_x(p, ls, us, dx, x);
    proj_y(p, dy, y);
    memcpy(xa, x, sizeof(double) * (size_t)n);
    memcpy(ya, y, sizeof(double) * (size_t)m);

    kkt_t k_anchor, k_prev, k1, k2;
    kkt_scaled(p, e, f, xa, ya, xu, yu, &k_anchor);
    double kprev_avg = INFINITY;
    int status = -1;
    const double *outx = xa, *outy = ya;
    kkt_t kout = k_anchor;
    if (kkt_max(&k_anchor) <= s->tol) status = ORC_OPTIMAL;
    if (!(kkt_max(&k_anchor) == kkt_max(&k_anchor))) status = ORC_NUMERICAL;
    if (status < 0 && s->max_iter <= 0) status = ORC_ITER_LIMIT;

    int64_t N = 0, kin = 0, snap = 0;
    double beta_prev = 1.0, r_prev = INFINITY, wsum = 0.0;
    (void)k_prev;
    while (status < 0) {
        /* ---- AdaptiveStepPDHG (reading: the PDLP step rule) ---- */
        double tau, sigma, nx2 = 0, ny2 = 0, eta_used = 0;
        double margin = INFINITY;   /* closest decision of this iteration */
        int attempts = 0;
        for (;;) {
            ++attempts;
            tau = eta / omega;
            sigma = eta * omega;
            /* x^ = Proj_X(x - tau (c - G^T y)) */
            spmv(n, trp, tci, tv, y, gty);
            ORC_PAR
            for (int64_t j = 0; j < n; ++j) xh[j] = x[j] - tau * (cs[j] - gty[j]);
            proj_x(p, ls, us, dx, xh);
            /* y^ = Proj_Y(y + sigma (h - G (2 x^ - x))) */
            ORC_PAR
            for (int64_t j = 0; j < n; ++j) xt[j] = 2.0 * xh[j] - x[j];
            spmv(m, p->row_ptr, p->col, gv, xt, gxt);
            ORC_PAR
            for (int64_t i = 0; i < m; ++i) yh[i] = y[i] + sigma * (hs[i] - gxt[i]);
            proj_y(p, dy, yh);
            /* largest step the iteration would have allowed */
            ORC_PAR
            for (int64_t j = 0; j < n; ++j) ddx[j] = xh[j] - x[j];
            ORC_PAR
            for (int64_t i = 0; i < m; ++i) ddy[i] = yh[i] - y[i];
            spmv(m, p->row_ptr, p->col, gv, ddx, gdx);
            nx2 = nrm2sq(n, ddx);
            ny2 = nrm2sq(m, ddy);
            double ip = dot(m, ddy, gdx);
            double den = 2.0 * fabs(ip);
            double ebar = den > 0.0 ? (omega * nx2 + ny2 / omega) / den : INFINITY;
            if (s->step_mode != 1 && !plain) margin = fmin(margin, rel_margin(eta, ebar));
            if (!(ebar == ebar)) {
                status = ORC_NUMERICAL;
                break;
            }
            /* reading (PDLP): the exponent base is 1 + the running count of
             * line-search attempts, the current one included */
            double nn = (double)(info->attempts + attempts + 1);
            double e1 = (1.0 - pow(nn, -s->step_reduce_exp)) * ebar;
            double e2 = (1.0 + pow(nn, -s->step_grow_exp)) * eta;
            double enew = e1 < e2 ? e1 : e2;
            if (s->step_mode == 1 || plain) { /* fixed step: every attempt is accepted */
                eta_used = eta;
                break;
            }
            /* replay: the other run's attempt count decides acceptance */
            int accept = eta <= ebar;
            if (tr && N < tr->replay_count) accept = attempts == tr->replay_attempts[N];
            if (accept) {
                eta_used = eta;
                eta = enew;
                break;
            }
            eta = enew;
            if (attempts >= s->max_attempts) {
                status = ORC_NUMERICAL;
                break;
            }
        }
        if (status >= 0) break;
        info->attempts += attempts;
        double omega_iter = omega;

        /* ---- AdaptiveReflectionParameter (reading) ---- */
        double beta;
        double r = sqrt(omega * nx2 + ny2 / omega);
        if (!plain && s->beta_mode != 1 && r_prev < INFINITY) margin = fmin(margin, rel_margin(r, r_prev));
        if (plain) {
            beta = 0.0;
        } else if (s->beta_mode == 1) {
            beta = s->beta_const;
        } else {
            int grow = r <= r_prev;
            /* replay: the other run's beta says which branch it took */
            if (tr && N < tr->replay_count) grow = tr->replay_beta[N] >= beta_prev;
            beta = grow ? fmin(1.0, s->beta_grow * beta_prev) : s->beta_shrink * beta_prev;
        }
        r_prev = r;
        beta_prev = beta;

        /* ---- ReflectedHalpern (Algorithm 1) ---- */
        /* the baseline PDHG keeps z = z^: weights 1 and 0 */
        double a = plain ? 1.0 : (double)(kin + 1) / (double)(kin + 2);
        double b = plain ? 0.0 : 1.0 / (double)(kin + 2);
        ORC_PAR
        for (int64_t j = 0; j < n; ++j) x[j] = a * ((1.0 + beta) * xh[j] - beta * x[j]) + b * xa[j];
        ORC_PAR
        for (int64_t i = 0; i < m; ++i) y[i] = a * ((1.0 + beta) * yh[i] - beta * y[i]) + b * ya[i];
        /* ---- weighted average (Algorithm 1) ---- */
        ORC_PAR
        for (int64_t j = 0; j < n; ++j) xsum[j] += eta_used * x[j];
        ORC_PAR
        for (int64_t i = 0; i < m; ++i) ysum[i] += eta_used * y[i];
        wsum += eta_used;
        ++kin;
        ++N;

        int64_t rec = N - 1;
        if (tr && rec < tr->cap) {
            tr->attempts[rec] = attempts;
            tr->eta_used[rec] = eta_used;
            tr->beta[rec] = beta;
            tr->omega[rec] = omega_iter;
            tr->check_code[rec] = 0;
            tr->check_kkt[rec] = 0.0;
            if (tr->margin) tr->margin[rec] = margin;
            tr->count = rec + 1;
        }
        if (tr && snap < tr->n_snap && tr->snap_iter[snap] == N) {
            for (int64_t j = 0; j < n; ++j) tr->snap_x[snap * n + j] = f[j] * x[j];
            for (int64_t i = 0; i < m; ++i) tr->snap_y[snap * m + i] = e[i] * y[i];
            ++snap;
        }

        /* ---- GetRestartCandidate, restart and termination (readings) ---- */
        if (kin % s->check_every != 0 && N < s->max_iter) continue;
        memcpy(xc1, x, sizeof(double) * (size_t)n);
        memcpy(yc1, y, sizeof(double) * (size_t)m);
        proj_x(p, ls, us, dx, xc1);
        proj_y(p, dy, yc1);
        kkt_scaled(p, e, f, xc1, yc1, xu, yu, &k1);
        for (int64_t j = 0; j < n; ++j) xc2[j] = xsum[j] / wsum;
        for (int64_t i = 0; i < m; ++i) yc2[i] = ysum[i] / wsum;
        proj_x(p, ls, us, dx, xc2);
        proj_y(p, dy, yc2);
        kkt_scaled(p, e, f, xc2, yc2, xu, yu, &k2);
        int chosen = !plain && kkt_avg(&k2) < kkt_avg(&k1) ? 1 : 0;
        const double *xc = chosen ? xc2 : xc1, *yc = chosen ? yc2 : yc1;
        kkt_t kc = chosen ? k2 : k1;
        double kcv = kkt_avg(&kc), kav = kkt_avg(&k_anchor);
        int reason = 0, stop = 0;
        if (!(kcv == kcv)) {
            status = ORC_NUMERICAL;
            stop = 1;
        } else if (kkt_max(&kc) <= s->tol) {
            status = ORC_OPTIMAL;
            stop = 1;
        } else if (N >= s->max_iter) {
            status = ORC_ITER_LIMIT;
            stop = 1;
        }
        if (!stop && !plain) {
            if (kcv <= s->restart_sufficient * kav)
                reason = 1;
            else if (kcv <= s->restart_necessary * kav && kcv > kprev_avg)
                reason = 2;
            else if ((double)kin >= s->restart_artificial * (double)N)
                reason = 3;
        }
        if (tr && rec < tr->replay_count && tr->replay_check_code[rec] > 0) {
            /* replay: the other run's candidate, restart reason and stop */
            int code = tr->replay_check_code[rec] - 1;
            chosen = code & 1;
            xc = chosen ? xc2 : xc1;
            yc = chosen ? yc2 : yc1;
            kc = chosen ? k2 : k1;
            kcv = kkt_avg(&kc);
            reason = (code >> 1) & 3;
            stop = (code >> 3) & 1;
            status = !stop ? -1 : (N >= s->max_iter && !(kkt_max(&kc) <= s->tol)) ? ORC_ITER_LIMIT
                                                                                     : ORC_OPTIMAL;
        }
        if (tr && rec < tr->cap) {
            tr->check_code[rec] = 1 + chosen + 2 * reason + 8 * stop;
            tr->check_kkt[rec] = kcv;
            if (tr->margin && !plain) {
                /* the candidate comparison and the restart thresholds */
                double mg = fmin(tr->margin[rec], rel_margin(kkt_avg(&k2), kkt_avg(&k1)));
                if (!stop) {
                    mg = fmin(mg, rel_margin(kcv, s->restart_sufficient * kav));
                    mg = fmin(mg, rel_margin(kcv, s->restart_necessary * kav));
                    if (kprev_avg < INFINITY) mg = fmin(mg, rel_margin(kcv, kprev_avg));
                }
                mg = fmin(mg, rel_margin(kkt_max(&kc), s->tol));
                tr->margin[rec] = mg;
            }
        }
        if (stop) {
            outx = xc;
            outy = yc;
            kout = kc;
            break;
        }
        if (reason) {
            /* PrimalWeightUpdate (reading: PDLP's smoothed log-ratio rule) */
            double ddxn = 0.0, ddyn = 0.0;
            for (int64_t j = 0; j < n; ++j) ddxn += sq(xc[j] - xa[j]);
            for (int64_t i = 0; i < m; ++i) ddyn += sq(yc[i] - ya[i]);
            ddxn = sqrt(ddxn);
            ddyn = sqrt(ddyn);
            if (ddxn > 1e-10 && ddyn > 1e-10)
                omega = exp(0.5 * log(ddyn / ddxn) + 0.5 * log(omega));
            memcpy(xa, xc, sizeof(double) * (size_t)n);
            memcpy(ya, yc, sizeof(double) * (size_t)m);
            memcpy(x, xc, sizeof(double) * (size_t)n);
            memcpy(y, yc, sizeof(double) * (size_t)m);
            k_anchor = kc;
            kprev_avg = INFINITY;
            kin = 0;
            memset(xsum, 0, sizeof(double) * (size_t)n);
            memset(ysum, 0, sizeof(double) * (size_t)m);
            wsum = 0.0;
            beta_prev = 1.0;
            r_prev = INFINITY;
            info->restarts++;
        } else {
            kprev_avg = kcv;
        }
    }

    for (int64_t j = 0; j < n; ++j) x_out[j] = f[j] * outx[j];
    for (int64_t i = 0; i < m; ++i) y_out[i] = e[i] * outy[i];
    info->status = status;
    info->iterations = N;
    info->pobj = kout.pobj;
    info->dobj = kout.dobj;
    info->err_p = kout.err_p;
    info->err_d = kout.err_d;
    info->err_gap = kout.err_gap;
    info->omega = omega;
    info->eta = eta;

    free(e), free(f), free(gv), free(trp), free(tci), free(tv), free(cs), free(hs), free(ls),
        free(us), free(dx), free(dy);
    free(x), free(y), free(xa), free(ya), free(xh), free(yh), free(gty), free(xt), free(gxt);
    free(ddx), free(ddy), free(gdx), free(xsum), free(ysum), free(xc1), free(yc1), free(xc2),
        free(yc2), free(xu), free(yu);
    return 0;
}
