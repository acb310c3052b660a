/*
 * pdcs_oracle.h -- plain FP64 CPU oracle for PDCS, the restarted,
 * reflected-Halpern, adaptive-step primal-dual hybrid gradient method for
 * conic programs of Lin, Xiong, Ge and Ye ("A Practical GPU-Enhanced
 * Matrix-Free Primal-Dual Method for Large-Scale Conic Programs").
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke entry point and the
 * benchmark's CPU-baseline leg are the only code that loads this library.
 * The GPU product path never links, imports or calls it, and the two share
 * no source, header, helper or constant table.
 *
 * Problem (Section 2, eq. (1)):
 *     min <c,x>  s.t.  G x - h in K_d^*,  l <= x_1 <= u,  x_2 in K_p,
 * with x = (x_1, x_2), x_1 the first n_box entries.  The caller describes
 * K_p by blocks covering x_2 and the row cones by blocks covering the m
 * rows; a row block of type T states G x - h in T, so K_d = T^*.
 *
 * Everything is double precision and, by default, single threaded and
 * deterministic (see orc_set_threads for the timing mode).
 */
#ifndef PDCS_ORACLE_H
#define PDCS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Cone type codes (the disciplined cones of Section 1.2).  Other codes are
 * rejected (-3).  The rotated second-order cone is rewritten as an SOC by the
 * Python wrapper before a problem reaches this library. */
enum {
    ORC_ZERO = 0,     /* {0}^d                                   */
    ORC_FREE = 1,     /* R^d                                     */
    ORC_NONNEG = 2,   /* R_+^d                                   */
    ORC_SOC = 3,      /* {(t,x): ||x|| <= t}, t first            */
    ORC_EXP = 4,      /* K_exp, (r,s,t) order of Appendix A.2    */
    ORC_EXP_DUAL = 5  /* K_exp^*                                 */
};

/* Solve outcome codes. */
enum { ORC_OPTIMAL = 0, ORC_ITER_LIMIT = 1, ORC_TIME_LIMIT = 2, ORC_NUMERICAL = 3 };

typedef struct {
    int64_t n, m, nnz, n_box;
    const int64_t *row_ptr; /* [m+1] */
    const int32_t *col;     /* [nnz] */
    const double *val;      /* [nnz] */
    const double *c;        /* [n]   */
    const double *h;        /* [m]   */
    const double *l, *u;    /* [n_box], +-INFINITY allowed */
    int64_t n_xcones;
    const int32_t *xcone_type;
    const int64_t *xcone_dim;
    int64_t n_rcones;
    const int32_t *rcone_type;
    const int64_t *rcone_dim;
} orc_problem;

typedef struct {
    double tol;                 /* termination tolerance on max(err_p, err_d, err_gap) */
    int64_t max_iter;           /* accepted PDHG iterations                              */
    int32_t check_every;        /* restart / termination check period                    */
    int32_t ruiz_iters;         /* Ruiz infinity-norm equilibration passes               */
    int32_t pock_chambolle;     /* 1: one Pock-Chambolle (alpha = 1) pass after Ruiz     */
    int32_t beta_mode;          /* 0: adaptive reflection, 1: constant beta_const        */
    double beta_const;
    double beta_grow;           /* adaptive beta: growth factor when the residual falls  */
    double beta_shrink;         /* adaptive beta: factor when the residual grows          */
    double step_reduce_exp;     /* eta' = min((1-(N+1)^-a) eta_bar, (1+(N+1)^-b) eta): a */
    double step_grow_exp;       /* b                                                      */
    double restart_sufficient;  /* restart if KKT(cand) <= this * KKT(anchor)             */
    double restart_necessary;   /* ... or <= this * KKT(anchor) and KKT grew             */
    double restart_artificial;  /* ... or inner iterations >= this * total iterations     */
    int32_t max_attempts;       /* line-search attempts per iteration before NUMERICAL    */
    int32_t step_mode;          /* 0: adaptive step (Algorithm 1), 1: fixed step          */
    double step_fixed;          /* fixed step = step_fixed / ||G~||_2                      */
    int32_t power_iters;        /* power iterations estimating ||G~||_2                    */
    int32_t plain_pdhg;         /* 1: the baseline PDHG of the paper's PDHG-vs-PDCS
                                 * comparison: fixed step step_fixed/||G~||_2 for both
                                 * sides (omega = 1), z = z^ (no reflection or Halpern),
                                 * no restarts, termination at the current iterate   */
} orc_settings;

typedef struct {
    int32_t status;
    int64_t iterations, attempts, restarts;
    double pobj, dobj, err_p, err_d, err_gap;
    double omega, eta;
} orc_info;

/* Optional per-iteration decision log and iterate snapshots. */
typedef struct {
    int64_t cap;            /* capacity of the per-iteration arrays                     */
    int64_t count;          /* out: records written                                     */
    int32_t *attempts;      /* line-search attempts of the iteration                    */
    double *eta_used;       /* step used                                                 */
    double *beta;           /* reflection parameter of the Halpern step                  */
    double *omega;          /* primal weight in force during the iteration               */
    int32_t *check_code;    /* 0: no check; else 1 + chosen + 2*reason + 8*stop          */
    double *check_kkt;      /* KKT average of the chosen candidate (checks only)         */
    int64_t n_snap;         /* snapshots of the current (Halpern) iterate, unscaled       */
    const int64_t *snap_iter;
    double *snap_x;         /* [n_snap * n] */
    double *snap_y;         /* [n_snap * m] */
    /* Replay of another run's decisions (parity harness): for the first
     * replay_count accepted iterations, iteration k is accepted at attempt
     * replay_attempts[k] (whatever eta <= eta_bar says), its reflection
     * parameter grows when replay_beta[k] >= the previous one and shrinks
     * otherwise, and a check after it takes the candidate, restart reason and
     * stop flag of replay_check_code[k] (codes as check_code).  Every
     * continuous quantity is still computed by this run.  0 = no replay. */
    int64_t replay_count;
    const int32_t *replay_attempts;
    const double *replay_beta;
    const int32_t *replay_check_code;
    /* Optional [cap]: per iteration, the smallest relative distance between a
     * deciding quantity and its threshold (eta against eta_bar at every
     * attempt, ||z^ - z||_omega against its previous value, and at a check
     * the two candidates' KKT averages, the restart thresholds and the
     * tolerance); NULL = not recorded. */
    double *margin;
} orc_trace;

void orc_settings_default(orc_settings *s);

/* Threads of the timing mode (default 1).  With n > 1 the sparse products,
 * vector passes and cone blocks of orc_solve run on n OpenMP threads and the
 * reductions add in a different order; n <= 1 restores the deterministic
 * single-thread mode that parity is measured in. */
void orc_set_threads(int n);
int orc_get_threads(void);

/* Projections onto one diagonally rescaled cone D K (Section 3, Theorems 1-3).
 * d is the diagonal of D (NULL = identity); v and out hold one block.
 * Return the case of the theorem that applied (1-4), 0 for elementwise types. */
int orc_proj_soc(int64_t dim, const double *v, const double *d, double *out);
int orc_proj_exp(const double *v, const double *d, double *out);
int orc_proj_exp_dual(const double *v, const double *d, double *out);
/* Projection of a whole vector onto a product of scaled cones (eq. (6)).
 * dual != 0 projects onto the product of the dual cones instead. */
void orc_proj_blocks(int64_t nblk, const int32_t *type, const int64_t *dim, int dual,
                     const double *d, double *v);

/* y = A x for a CSR matrix (plain definition). */
void orc_spmv(int64_t rows, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
              double *y);

/* Diagonal rescaling E (rows, [m]) and F (columns, [n]). */
int orc_scaling(const orc_problem *p, const orc_settings *s, double *e, double *f);

/* Termination measures of eq. (PDCS_terminate_tolerance) at unscaled (x, y). */
int orc_kkt(const orc_problem *p, const double *x, const double *y, double *err_p,
            double *err_d, double *err_gap, double *pobj, double *dobj);

/* One plain PDHG step (eq. (5)) on the unscaled problem. */
int orc_onepdhg(const orc_problem *p, const double *x, const double *y, double tau,
                double sigma, double *xh, double *yh);

/* Algorithm 1 with diagonal rescaling. x0/y0 may be NULL (cold start);
 * omega0 <= 0 selects the default initial primal weight. */
int orc_solve(const orc_problem *p, const orc_settings *s, const double *x0, const double *y0,
              double omega0, double *x_out, double *y_out, orc_info *info, orc_trace *trace);

#ifdef __cplusplus
}
#endif
#endif
