/*
 * pdcs.h -- C ABI of the MI355X (gfx950) PDCS hot path.
 *
 * PDCS (Lin, Xiong, Ge, Ye, "A Practical GPU-Enhanced Matrix-Free
 * Primal-Dual Method for Large-Scale Conic Programs") solves the conic
 * program of Section 2, eq. (1):
 *
 *     min <c, x>  s.t.  G x - h in K_d^*,  l <= x_1 <= u,  x_2 in K_p,
 *
 * with x = (x_1, x_2), x_1 the first n_box entries of x, by Algorithm 1 of
 * Section 3 (adaptive-step PDHG, adaptive reflected Halpern iteration,
 * weighted averaging, restarts, primal weight) on the diagonally rescaled
 * problem of Section 3.  Every step of the iteration runs in this library's
 * HIP kernels on one GPU.
 *
 * Conventions shared by all calls
 *   - Every call returns a pdcs_status; 0 is success, negative values are
 *     errors and pdcs_last_error() then holds a message (thread-local).  No
 *     C++ exception crosses this boundary.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the current device (for example torch tensor
 *     data_ptr()).  All arrays are dense, contiguous, row-major.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls that return results to the host
 *     synchronise it.
 *   - Handles are owned by the library and released by the matching
 *     *_destroy call.  A handle is used by one host thread at a time.
 */
#ifndef PDCS_H
#define PDCS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PDCS_OK = 0,
    PDCS_ERR_INVALID_ARG = -1,   /* null pointer, negative size, bad enum, bad CSR     */
    PDCS_ERR_DIMENSION = -2,     /* cone dimensions do not add up to n - n_box or m    */
    PDCS_ERR_NONFINITE = -3,     /* NaN/inf in G, c or h (l, u may hold +-inf)         */
    PDCS_ERR_OOM = -4,           /* device allocation failed                           */
    PDCS_ERR_HIP = -5,           /* a HIP runtime call failed                          */
    PDCS_ERR_NOT_SUPPORTED = -6  /* valid request outside what the library implements */
} pdcs_status;

/* Disciplined cones of Section 1.2.  A block of dimension d.
 *   SOC: (t, x) with ||x|| <= t, t first.  EXP, EXP_DUAL: d = 3, entries in the
 *   (r, s, t) order of Appendix A.2.
 * For x_2 a block of type T requires x_block in T.  For the rows a block of
 * type T requires (G x - h)_block in T, i.e. it describes K_d^* and the dual
 * variable y_block lies in T^* (ZERO <-> FREE, EXP <-> EXP_DUAL, NONNEG and SOC
 * self-dual). */
enum {
    PDCS_CONE_ZERO = 0,
    PDCS_CONE_FREE = 1,
    PDCS_CONE_NONNEG = 2,
    PDCS_CONE_SOC = 3,
    PDCS_CONE_EXP = 4,
    PDCS_CONE_EXP_DUAL = 5,
    /* Rotated SOC, d >= 2: (u, v, w) with 2 u v >= ||w||^2, u, v >= 0 (the
     * cone of the paper's Lasso form).  The orthogonal, self-inverse map
     * T(u, v, w) = ((u + v)/sqrt 2, (u - v)/sqrt 2, w) takes it onto SOC of the
     * same dimension, so at creation a row block of this type is replaced by
     * T applied to its rows of G and h, and an x block by G T and T c on its
     * first two entries; both become SOC blocks.  Starting points and
     * solutions are mapped by T at the boundary (entries of G that the map
     * makes exactly zero are dropped).  The cone is self-dual.  Supported by
     * pdcs_problem_create and pdcs_batch_create (host arrays; the device
     * form returns NOT_SUPPORTED) and by the projections with d_dev = NULL
     * (NOT_SUPPORTED otherwise).  pdcs_solve, pdcs_spmv, pdcs_spmv32 and
     * pdcs_kkt take and return points of the caller's problem; the
     * termination measures and pdcs_scaling are those of the mapped problem
     * (T keeps 2-norms, the infinity norms of the measures differ by at most
     * a factor sqrt 2). */
    PDCS_CONE_RSOC = 6
};

/* Outcome of a solve (distinct from the call's pdcs_status). */
enum {
    PDCS_SOLVE_OPTIMAL = 0,     /* max(err_p, err_d, err_gap) <= tol                   */
    PDCS_SOLVE_ITER_LIMIT = 1,  /* max_iter accepted iterations reached                */
    PDCS_SOLVE_TIME_LIMIT = 2,  /* time_limit seconds reached (checked at checks)      */
    PDCS_SOLVE_NUMERICAL = 3    /* a non-finite step-size or KKT quantity was detected */
};

/* Problem data of eq. (1), CSR for G (rows sorted or not; duplicates are not
 * merged).  nnz must be below 2^31.  In pdcs_problem_create every pointer is
 * host memory; in pdcs_problem_create_device the bulk arrays (row_ptr, col,
 * val, c, h, l, u) are device memory and the cone lists stay on the host.
 * The caller keeps ownership; the library copies what it needs. */
typedef struct {
    int64_t n, m, nnz, n_box;
    const int64_t *row_ptr;   /* [m+1], row_ptr[0] = 0, row_ptr[m] = nnz          */
    const int32_t *col;       /* [nnz], 0 <= col < n                              */
    const double *val;        /* [nnz]                                            */
    const double *c;          /* [n]                                              */
    const double *h;          /* [m]                                              */
    const double *l, *u;      /* [n_box], -INFINITY / +INFINITY allowed           */
    int64_t n_xcones;         /* blocks partitioning x_2 (entries n_box .. n-1)   */
    const int32_t *xcone_type;
    const int64_t *xcone_dim;
    int64_t n_rcones;         /* blocks partitioning the m rows                   */
    const int32_t *rcone_type;
    const int64_t *rcone_dim;
} pdcs_problem_desc;

/* Algorithm 1 parameters.  The paper defers the step-size, reflection,
 * restart, primal-weight and rescaling rules to its companion technical note;
 * the fields below are the constants of the rules this library implements. */
typedef struct {
    double tol;                 /* termination on max(err_p, err_d, err_gap), Section 5  */
    int64_t max_iter;           /* accepted PDHG iterations                              */
    double time_limit;          /* seconds, <= 0 = none                                   */
    int32_t check_every;        /* restart/termination check period (inner iterations)   */
    int32_t ruiz_iters;         /* Ruiz infinity-norm passes of the rescaling            */
    int32_t pock_chambolle;     /* 1: one Pock-Chambolle (alpha = 1) pass after Ruiz     */
    int32_t beta_mode;          /* 0: adaptive reflection parameter, 1: constant         */
    double beta_const;
    double beta_grow, beta_shrink;
    double step_reduce_exp, step_grow_exp;
    double restart_sufficient, restart_necessary, restart_artificial;
    int32_t max_attempts;       /* line-search attempts per iteration before NUMERICAL   */
    int32_t out_on_device;      /* 1: x_out / y_out of pdcs_solve are device pointers    */
    int32_t step_mode;          /* 0: adaptive step of Algorithm 1; 1: fixed step        */
    double step_fixed;          /* fixed step = step_fixed / ||G~||_2 (step_mode 1)      */
    int32_t power_iters;        /* power iterations estimating ||G~||_2 (step_mode 1)    */
    int32_t use_graph;          /* 1: replay batches of 64 step attempts as a HIP graph  */
    int32_t time_kernels;       /* 1: time each step-attempt kernel with HIP events on
                                 * the solve stream (launches eagerly, no graph); the
                                 * sums land in pdcs_info.kernel_ms / kernel_launches */
    /* Mixed precision (not in the paper): precision 1 runs the two products of
     * every step attempt with FP32 matrix values and FP32 copies of x^ and y^
     * (products and sums in FP64); iterates, anchors, averages, projections,
     * step decisions and every check stay FP64.  precision 2 also projects
     * the SOC blocks of at most 256 entries and the exponential cones of the
     * two step passes in FP32 (see pdcs_project_fp32; the exponential cone's
     * case tests and range safeguards stay FP64).  The solve switches to the
     * FP64 products and projections for good (the polish phase) once the
     * chosen candidate's max(err_p, err_d, err_gap) <= polish_tol, or after
     * polish_stall checks in a row without a new best; the kept products
     * G~x, G~^T y and those of the anchor are then recomputed in FP64.  A
     * batch switches as a whole, as soon as any of its running instances
     * meets that rule.  precision 0 is plain FP64. */
    int32_t precision;
    double polish_tol;
    int32_t polish_stall;
    /* 1: before the first solve of a problem or batch, time every launch
     * configuration of the two products (CSR-stream; row-split with 2, 4, ...,
     * 64 lanes per row) on its own matrices with HIP events and keep the
     * fastest for that handle (not in the paper).  0: fixed rule. */
    int32_t autotune;
    /* Batches: 1 hands the instances still running to problems of their own
     * (restarted at their chosen candidate with their primal weight) once they
     * hold at most 1/8 of the batch's nonzeros (not in the paper).  2 does so
     * only when, in addition, a step attempt over the batch has come to cost
     * more than 4 times what the running instances' own attempts would (their
     * share of the nonzeros times the cost per attempt at the first check, at
     * least 25 us each), measured between checks: the launches then mostly
     * dispatch workgroups of finished instances.  Default 0: the restart at
     * the hand-over can cost a straggler more iterations than the batch-wide
     * launches cost it. */
    int32_t batch_dropout;
    /* 1: the baseline PDHG the paper compares PDCS with (its appendix on PDHG
     * versus PDCS): step step_fixed / ||G~||_2 on both sides (omega = 1 unless
     * omega0 is given), z = z^ (no reflection, no Halpern anchor), no
     * restarts, termination measured at the current iterate; the rescaling
     * still applies.  0: Algorithm 1. */
    int32_t plain_pdhg;
    /* > 0: at a check, when at least this many seconds have passed since the
     * last line, print one progress line to stderr (elapsed time, instances
     * still running, their largest iteration count and worst max-KKT).
     * 0: silent. */
    double log_every;
} pdcs_settings;

/* Kernels of one step attempt, in launch order (indices of pdcs_info.kernel_ms). */
enum {
    PDCS_K_PRIMAL = 0,          /* primal update and projection of eq. (5)               */
    PDCS_K_SPMV_G = 1,          /* G~ x^                                                 */
    PDCS_K_DUAL = 2,            /* dual update and projection of eq. (5)                 */
    PDCS_K_DECIDE = 3,          /* step acceptance, next step size, reflection parameter */
    PDCS_K_SPMV_GT = 4,         /* G~^T y^                                               */
    PDCS_K_HALPERN = 5,         /* reflected Halpern step and weighted average           */
    PDCS_K_COUNT = 6
};

typedef struct {
    int32_t status;             /* PDCS_SOLVE_*                                          */
    int64_t iterations;         /* accepted PDHG iterations                              */
    int64_t attempts;           /* step-size attempts (>= iterations)                    */
    int64_t restarts;
    int64_t spmv;               /* sparse products with G or G^T issued                  */
    double pobj, dobj;          /* objectives of eq. (1) / eq. (2) at the output         */
    double err_p, err_d, err_gap;
    double omega, eta;          /* final primal weight and step size                     */
    double setup_s;             /* rescaling and initialisation, seconds                 */
    double solve_s;             /* iterations and checks, seconds                        */
    /* With settings.time_kernels: summed event-to-event milliseconds of each
     * step-attempt kernel (PDCS_K_*) over the attempts that did work, and the
     * number of such launches.  Launches on attempts past a due check are
     * excluded; SPMV_GT and HALPERN count accepted attempts only, but their
     * sums include the early-exit launches of rejected attempts.  Zero
     * otherwise. */
    double kernel_ms[PDCS_K_COUNT];
    int64_t kernel_launches[PDCS_K_COUNT];
    int64_t polish_iter;        /* precision 1: accepted iterations before the switch to
                                 * FP64 products (-1: never switched); 0 otherwise     */
    double done_s;              /* seconds from the first iteration until this problem
                                 * stopped: in a batch, the check at which this
                                 * instance finished (solve_s is the whole batch's)  */
} pdcs_info;

/* Optional decision log and iterate snapshots of pdcs_solve, host memory.
 * Record k (0-based) describes accepted iteration k+1.  check_code is 0 when
 * no check followed the iteration, else 1 + chosen + 2*reason + 8*stop, with
 * chosen 0 = current iterate, 1 = average; reason 0 = no restart, 1 =
 * sufficient decay, 2 = necessary decay and growth, 3 = artificial.  Snapshot
 * i holds the unscaled current iterate after accepted iteration snap_iter[i]
 * (ascending).  Asking for a log or snapshots makes the solve synchronise
 * after every step attempt. */
typedef struct {
    int64_t cap;
    int64_t count;              /* out */
    int32_t *attempts;
    double *eta_used;
    double *beta;
    double *omega;
    int32_t *check_code;
    double *check_kkt;
    int64_t n_snap;
    const int64_t *snap_iter;
    double *snap_x;             /* [n_snap * n] */
    double *snap_y;             /* [n_snap * m] */
    /* Replay of another run's decisions (a parity harness: the decision log
     * of the reference implementation, same settings).  For the first
     * replay_count accepted iterations (host arrays of that length),
     * iteration k is accepted at attempt replay_attempts[k] (>= 1) whatever
     * eta <= eta_bar says here, its reflection parameter grows when
     * replay_beta[k] >= the previous one and shrinks otherwise, and a check
     * after it takes the candidate, restart reason and stop flag encoded in
     * replay_check_code[k] (codes as check_code).  Every continuous quantity
     * (step sizes, reflection parameters, primal weights, iterates) is still
     * computed by this run, so two implementations can be compared iterate by
     * iterate past a decision that rounding tips the other way.
     * replay_count 0 = no replay. */
    int64_t replay_count;
    const int32_t *replay_attempts;
    const double *replay_beta;
    const int32_t *replay_check_code;
} pdcs_trace;

typedef struct pdcs_problem pdcs_problem;

/* Fills the default parameters (tol 1e-6, check every 64, 10 Ruiz passes and a
 * Pock-Chambolle pass, adaptive reflection, PDLP-style step/restart/weight
 * constants).  Errors: INVALID_ARG on NULL. */
pdcs_status pdcs_settings_default(pdcs_settings *s);

/* Validates the problem of eq. (1), copies it to the device, builds the CSR
 * of G^T and the cone dispatch plans (the thread-, wavefront-, workgroup- and
 * grid-level projection strategies of Section 4, Table 3; an SOC block of at
 * least 8192 entries is spread over one workgroup per 4096 entries, at most
 * 64, while the plan holds at most 256 such blocks).
 * Errors: INVALID_ARG, DIMENSION, NONFINITE, OOM, HIP.  On error *out = NULL. */
pdcs_status pdcs_problem_create(const pdcs_problem_desc *desc, void *hip_stream,
                                pdcs_problem **out);

/* As pdcs_problem_create, with the bulk arrays in device memory (see
 * pdcs_problem_desc).  They are copied, so the caller may free them after the
 * call returns. */
pdcs_status pdcs_problem_create_device(const pdcs_problem_desc *desc, void *hip_stream,
                                       pdcs_problem **out);

void pdcs_problem_destroy(pdcs_problem *p);

/* Algorithm 1 (Section 3) with diagonal rescaling, run to the tolerance of
 * Section 5, eq. (PDCS_terminate_tolerance).  x0 [n] / y0 [m] (host, nullable:
 * cold start from zero) are an unscaled starting point; omega0 <= 0 selects
 * the default primal weight.  x_out [n] and y_out [m] receive the unscaled
 * solution (host memory unless settings->out_on_device).  info and trace are
 * nullable.  Errors: INVALID_ARG, OOM, HIP (also when a grid-level SOC
 * projection timed out waiting for its workgroups, detected at the next
 * check); the solve outcome is info->status. */
pdcs_status pdcs_solve(pdcs_problem *p, const pdcs_settings *settings, const double *x0,
                       const double *y0, double omega0, double *x_out, double *y_out,
                       pdcs_info *info, pdcs_trace *trace);

/* Rescaling factors of Section 3 that pdcs_solve uses with these settings:
 * e_out [m] (rows, E) and f_out [n] (columns, F), host memory, G~ = E G F. */
pdcs_status pdcs_scaling(pdcs_problem *p, const pdcs_settings *settings, double *e_out,
                         double *f_out);

/* Sparse product with the unscaled G (transpose = 0: y_dev[m] = G x_dev[n]) or
 * G^T (transpose = 1: y_dev[n] = G^T x_dev[m]); device pointers, enqueued on
 * hip_stream.  The products SpMV G x and G^T y of eq. (5). */
pdcs_status pdcs_spmv(pdcs_problem *p, int transpose, const double *x_dev, double *y_dev,
                      void *hip_stream);

/* The FP32 product of the mixed-precision form (not in the paper), on the
 * unscaled G: the values and x_dev are rounded to FP32, products and sums are
 * formed in FP64, y_dev is FP64.  Same shapes, memory and stream rules as
 * pdcs_spmv; the first call allocates the FP32 copies of the values. */
pdcs_status pdcs_spmv32(pdcs_problem *p, int transpose, const double *x_dev, double *y_dev,
                        void *hip_stream);

/* Kernel layout of the two products of eq. (5) (not in the paper; the same
 * sums, formed in another order):
 *   PDCS_LAYOUT_DEFAULT (0)  chosen from the shape at creation;
 *   PDCS_LAYOUT_STREAM (-1)  CSR-stream: workgroups stream row ranges of at
 *                            most 2048 entries through LDS;
 *   L in {2,4,...,64}        row-split: L lanes per row;
 *   PDCS_LAYOUT_SLABS(S)     S in {1,2,4,8} column slabs of equal entry counts,
 *                            each slab's workgroups on 8/S of the 8 XCDs, so
 *                            an XCD gathers from 1/S of the vector; the S slab
 *                            sums of a row are added in slab order.
 * In every layout a row with more entries than the layout's threshold
 * (max(64, 32 L), L the lanes of the row-split rule for the mean row length,
 * at most 2048 in the streamed layouts) is summed in chunks of 4096 entries,
 * added in chunk order.  pdcs_set_layout
 * rebuilds the plans of G x (layout_g) and G^T y (layout_gt) and keeps them
 * (pdcs_settings.autotune then leaves them alone); pdcs_get_layout reports the
 * layouts in use (0 only before any is chosen).  Errors: INVALID_ARG for an
 * unknown code, NOT_SUPPORTED for slabs with 2^31 or more rows or entries. */
#define PDCS_LAYOUT_DEFAULT 0
#define PDCS_LAYOUT_STREAM (-1)
#define PDCS_LAYOUT_SLABS(S) (-10 - (S))
pdcs_status pdcs_set_layout(pdcs_problem *p, int layout_g, int layout_gt);
pdcs_status pdcs_get_layout(const pdcs_problem *p, int *layout_g, int *layout_gt);

/* Termination measures of eq. (PDCS_terminate_tolerance) at the unscaled
 * point (x_dev [n], y_dev [m], device memory).  out[5] (host) receives
 * err_p, err_d, err_gap, primal objective, dual objective. */
pdcs_status pdcs_kkt(pdcs_problem *p, const double *x_dev, const double *y_dev, double *out);

/* Projection of v_dev (device, length sum(dims)) in place onto the product of
 * diagonally rescaled cones D K_1 x ... x D K_nblocks (eq. (6); Theorem 1 for
 * SOC, Theorem 3 for EXP, the Appendix A.2 remark for EXP_DUAL; RSOC as
 * T P_SOC(T v), D = I only).  types and dims are host arrays; d_dev (device,
 * nullable = identity) is the diagonal of D.  dual != 0 projects onto the
 * product of the dual cones instead.  With d_dev null, an SOC block outside
 * the cone and its polar takes the closed form of the identity case,
 * s = (t + ||x||)/2 (the root of Theorem 1's equation when D = I), instead
 * of the root search.
 * Errors: INVALID_ARG, DIMENSION, HIP (also when a grid-level block timed out
 * waiting for its workgroups); NOT_SUPPORTED for RSOC with d_dev. */
pdcs_status pdcs_project(int64_t nblocks, const int32_t *types, const int64_t *dims, int dual,
                         const double *d_dev, double *v_dev, void *hip_stream);

/* pdcs_project in the arithmetic of the mixed-precision form's FP32
 * projections (not in the paper; settings.precision 2): SOC blocks of at most
 * 256 entries and exponential cones are projected in FP32 (inputs rounded to
 * FP32, norms, case tests and the root search in FP32, results widened), with
 * the FP64 routine taking over wherever FP32 cannot be trusted (the
 * exponential cone's case tests and unbounded or wide search intervals, and
 * any search that leaves the FP32 range or does not settle).  Other blocks as
 * pdcs_project.  A test and measurement hook; same arguments and errors. */
pdcs_status pdcs_project_fp32(int64_t nblocks, const int32_t *types, const int64_t *dims, int dual,
                              const double *d_dev, double *v_dev, void *hip_stream);

/* pdcs_project for callers that cannot allocate device memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid
 * it).  Same arguments, arithmetic and results as pdcs_project, but the tile
 * plan, per-tile partial sums, barrier state of grid-level SOC blocks and the
 * rotated blocks' offsets live in a fixed device array of
 * PDCS_PROJECT_NOALLOC_SCRATCH_BYTES per GPU (held by each GPU the library
 * runs on until the process ends); no device memory is allocated or freed.
 * Plans are built on the host (host memory only) and copied in.  Calls on one
 * GPU share that array and the last call's contents stay in it: calls that
 * overlap on one GPU (several threads or streams at once) race; the barrier
 * counters are cleared by a kernel at the start of every call.  The call
 * waits for its stream.  Errors: as pdcs_project, plus NOT_SUPPORTED when the
 * cone list needs more scratch than the array holds (the message gives both
 * sizes).  Per unit: 12 bytes per SOC block plus 72 bytes per tile of up to
 * 32 blocks, 8 bytes per exponential cone plus 72 per tile of 64 to 256 cones, 72 bytes per
 * 2048 elementwise entries, about 40 KB per SOC block of 8192 entries or more
 * (when at most 256 such blocks are present), 8 bytes per rotated block;
 * 1e5 SOC blocks of dim <= 8 thus take about 1.4 MB. */
#define PDCS_PROJECT_NOALLOC_SCRATCH_BYTES (16u << 20)
pdcs_status pdcs_project_noalloc(int64_t nblocks, const int32_t *types, const int64_t *dims,
                                 int dual, const double *d_dev, double *v_dev, void *hip_stream);

/* A projection plan for one product of cones, built once and reused: the
 * dispatch of pdcs_project (the thread-, wavefront- and workgroup-level
 * classes of Section 4) kept on the device.  pdcs_cones_create takes host
 * arrays types/dims (copied); pdcs_cones_project enqueues the projection of
 * v_dev (device, length sum(dims)) in place on hip_stream without waiting,
 * with d_dev (device, nullable = identity) the diagonal of D and dual != 0
 * for the dual cones.  Calls on one plan must not overlap (they share its
 * scratch and the barrier state of its grid-level SOC blocks); each call
 * first clears that barrier state.  The call does not wait, so a barrier
 * wait that times out (the launch's projections are then invalid) is not
 * reported here; pdcs_project and pdcs_solve, which wait, report it.  Errors:
 * INVALID_ARG, DIMENSION, OOM, HIP; NOT_SUPPORTED for a plan with RSOC blocks
 * given a d_dev. */
typedef struct pdcs_cones pdcs_cones;
pdcs_status pdcs_cones_create(int64_t nblocks, const int32_t *types, const int64_t *dims,
                              void *hip_stream, pdcs_cones **out);
pdcs_status pdcs_cones_project(pdcs_cones *c, int dual, const double *d_dev, double *v_dev,
                               void *hip_stream);
void pdcs_cones_destroy(pdcs_cones *c);


/* ---------------------------------------------------------------------------
 * Batches (not in the paper): `count` independent problems solved together.
 * Their data are laid out block-diagonally on the device and every kernel of a
 * step attempt covers all instances at once (one launch per kernel, replayed
 * from a captured HIP graph), each instance with its own step size, primal
 * weight, reflection parameter, restarts and termination.  An instance that
 * has converged stops taking work.  descs: host arrays of every instance,
 * deep-copied.  Each instance's nnz, and the totals of n and m, must stay
 * below 2^31; the total nnz may exceed it (indices into the batch's entries
 * are 64-bit, G^T is built instance by instance).  Same errors as
 * pdcs_problem_create, plus NOT_SUPPORTED for device arrays. */
typedef struct pdcs_batch pdcs_batch;
pdcs_status pdcs_batch_create(const pdcs_problem_desc *descs, int64_t count, void *hip_stream,
                              pdcs_batch **out);
/* Solve of every instance: x0, y0 (arrays of count host pointers, or NULL;
 * a NULL entry is a cold start) and omega0 (count values, <= 0 for the
 * default, or NULL) as in pdcs_solve; x_out[b] (n_b) and y_out[b] (m_b) as in
 * pdcs_solve (host memory, or device memory with settings.out_on_device);
 * infos: array of count results, the times are the batch's. */
pdcs_status pdcs_batch_solve(pdcs_batch *b, const pdcs_settings *settings, const double *const *x0,
                             const double *const *y0, const double *omega0, double *const *x_out,
                             double *const *y_out, pdcs_info *infos);
int64_t pdcs_batch_size(const pdcs_batch *b);
void pdcs_batch_destroy(pdcs_batch *b);

/* ---------------------------------------------------------------------------
 * Learned warm start (not in the paper).  A perceptron with two hidden ReLU
 * layers maps the parameters theta of a parametric family to a starting point
 * (x0, y0) and log omega0 of pdcs_solve.  GEMM operands are BF16 with FP32
 * accumulation on the matrix cores; master parameters, biases, the loss and
 * the Adam moments are FP32.
 *
 * Parameters: one flat FP32 array of pdcs_mlp_num_params entries laid out
 * [W1 (hid x in), b1 (hid), W2 (hid x hid), b2 (hid), W3 (out x hid), b3 (out)],
 * weights row-major by output unit.  Activations: row-major, one row per
 * sample.  params (host) is copied at create; max_batch bounds every call's
 * batch.  All data pointers named *_dev are device memory; work is enqueued on
 * the stream given at create. */
typedef struct pdcs_mlp pdcs_mlp;
pdcs_status pdcs_mlp_create(int64_t in, int64_t hid, int64_t out, int64_t max_batch,
                            const float *params, void *hip_stream, pdcs_mlp **mlp);
int64_t pdcs_mlp_num_params(const pdcs_mlp *m);
/* out_dev [batch x out] = network(theta_dev [batch x in]) */
pdcs_status pdcs_mlp_forward(pdcs_mlp *m, const float *theta_dev, int64_t batch, float *out_dev);
/* Gradient of L = sum (out - target)^2 / (2 batch out) with respect to the
 * parameters (grad_host: the flat layout above, may be NULL) and L. */
pdcs_status pdcs_mlp_gradient(pdcs_mlp *m, const float *theta_dev, const float *target_dev,
                              int64_t batch, float *grad_host, double *loss);
/* The gradient above followed by one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected) with step size lr. */
pdcs_status pdcs_mlp_train_step(pdcs_mlp *m, const float *theta_dev, const float *target_dev,
                                int64_t batch, float lr, double *loss);
pdcs_status pdcs_mlp_get_params(const pdcs_mlp *m, float *params_host);
void pdcs_mlp_destroy(pdcs_mlp *m);

/* The network's GEMM on the matrix cores: C [M x N] = op(A) op(B) (+ bias[n])
 * (then max(., 0) when relu), A and B BF16 (raw 16-bit patterns), FP32
 * accumulation; C written as FP32 to c32 and/or rounded to BF16 (nearest even)
 * to c16, row-major with leading dimension ldc.  op(A)(m, k) = a[m lda + k]
 * (ta = 0) or a[k lda + m] (ta = 1); op(B)(k, n) = b[k ldb + n] (tb = 0) or
 * b[n ldb + k] (tb = 1).  Device pointers; enqueued on hip_stream. */
pdcs_status pdcs_gemm_bf16(int ta, int tb, int64_t M, int64_t N, int64_t K, const uint16_t *a,
                           int64_t lda, const uint16_t *b, int64_t ldb, const float *bias, int relu,
                           float *c32, uint16_t *c16, int64_t ldc, void *hip_stream);

const char *pdcs_status_string(pdcs_status s);
const char *pdcs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
