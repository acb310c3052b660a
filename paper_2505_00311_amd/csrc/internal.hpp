// internal.hpp -- declarations shared by the HIP translation units of libpdcs.
//
// Layout in HBM (one problem, FP64):
//   G   : CSR, int64 row_ptr[m+1], int32 col[nnz], double val[nnz] (+ scaled copy)
//   G^T : CSR of the transpose built on the device (same layout, n rows)
//   x-side vectors [n] and y-side vectors [m], structure of arrays, contiguous
//   cone plans: tile lists that route each workgroup to one class of work
//   (elementwise entries, wavefront-per-SOC, workgroup-per-SOC, thread-per-exp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace pdcs {

constexpr int kBlock = 256;          // threads per workgroup of every pass kernel
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kSocWaveMax = 256;     // SOC blocks up to this dim: a lane group each
constexpr int kElemPerTile = 2048;   // entries per elementwise tile
// exponential cones per tile (one thread each): 256 (four wavefronts) when a
// cone list still gets kExpMinTiles tiles that way, else 128, else 64
constexpr int kExpPerTile = 64;
constexpr int kExpMinTiles = 512;
static_assert(4 * kExpPerTile <= kBlock, "an exponential tile holds at most one cone per thread");
constexpr int kPartials = 6;         // per-tile partial slots: 3 sums, 3 maxima
// SOC blocks of at least kSocGridMin entries are spread over several
// workgroups (one per kSocGridChunk entries, at most kSocGridMaxParts)
constexpr int kSocGridMin = 8192;
constexpr int kSocGridChunk = 4096;
constexpr int kSocGridMaxParts = 512;   // at most the workgroups one launch keeps resident
constexpr int kSocGridTargetParts = 1536;  // parts of all grid-level blocks of a cone list
constexpr int kSocGridMinCap = 4;        // the part cap when many such blocks share it
constexpr int kSocGridPartCode = 1024;  // a grid tile's count: part + kSocGridPartCode * parts
constexpr int kSocGridMaxBlocks = 256;   // more large blocks than this: one workgroup each
constexpr int kSocGridSlot = 5;          // values per part in one reduction round

// cone type codes of the C ABI
enum ConeType : int32_t { kZero = 0, kFree = 1, kNonneg = 2, kSoc = 3, kExp = 4, kExpDual = 5,
                          kRsoc = 6 };   // rotated SOC: mapped to kSoc at the boundary

// tile kinds of a cone plan
enum TileKind : int32_t {
    kTileBox = 0,
    kTileZero = 1,
    kTileFree = 2,
    kTileNonneg = 3,
    kTileSocBlock = 5,   // one SOC block per workgroup (dim > 256)
    kTileExp = 6,
    kTileExpDual = 7,
    kTileSoc8 = 8,       // SOC blocks of dim <= 8, 8 lanes each (32 per tile)
    kTileSoc16 = 9,      // dim <= 16, 16 lanes each (16 per tile)
    kTileSoc32 = 10,     // dim <= 32, 16 lanes with 2 entries each (16 per tile)
    kTileSoc64 = 11,     // dim <= 64, 16 lanes with 4 entries each (16 per tile)
    kTileSoc128 = 12,    // dim <= 128, 32 lanes with 4 entries each (8 per tile)
    kTileSoc256 = 13,    // dim <= 256, one wavefront, 4 entries per lane (4 per tile)
    kTileSocGrid = 14    // one part of an SOC block of dim >= kSocGridMin (start = block,
                         // count = part + kSocGridPartCode * parts, pad = grid slot)
};

struct Tile {
    int32_t kind;
    int32_t count;   // entries (elementwise), blocks (SOC wave, exp) or 1 (SOC block)
    int64_t start;   // first entry (elementwise) or first block index
    int32_t inst;    // instance of a batch the tile belongs to (0 for a single problem)
    int32_t pad;
};

// Device view of a cone plan for one side (x or y).
struct ConePlan {
    int64_t ntiles = 0;
    Tile *tiles = nullptr;
    int64_t *soc_off = nullptr;   // global entry offset of each SOC block
    int32_t *soc_dim = nullptr;
    int64_t *exp_off = nullptr;   // global entry offset of each exp block
    int64_t n_soc = 0, n_exp = 0;
    double *soc_root = nullptr;   // last case-4 root per SOC block (s), NaN = none
    double *exp_root = nullptr;   // last case-4 root per exp block (rho), NaN = none
    int64_t *inst_tiles = nullptr;  // [B+1]: tiles of instance b are [inst_tiles[b], inst_tiles[b+1])
    // grid-level SOC blocks (slots): a barrier counter each (it only grows),
    // two rounds of per-part partial sums [slot][round][part][kSocGridSlot], and a
    // sticky flag set when a barrier wait timed out
    int64_t n_grid = 0;
    unsigned long long *grid_ctr = nullptr;
    double *grid_part = nullptr;
    int *grid_err = nullptr;
};

// Instance of each entry of a batch (null for a single problem: instance 0).
__host__ __device__ inline int inst_of(const int32_t *map, int64_t i) { return map ? map[i] : 0; }

struct Csr {
    int64_t rows = 0, cols = 0, nnz = 0;
    int64_t *rp = nullptr;
    int32_t *ci = nullptr;
    double *v = nullptr;
    float *v32 = nullptr;   // FP32 copy of v (mixed-precision form), or null
    // v and v32 in the entry order of a column-slab plan (null unless the
    // matrix is used with one; filled by slab_values)
    double *sv = nullptr;
    float *sv32 = nullptr;
};

// Launch plan of one sparse product: short rows take `lanes` lanes each; rows
// longer than long_thr are cut into chunks of kLongChunk entries, one
// workgroup per chunk, and summed per row in chunk order.
constexpr int64_t kLongChunk = 4096;
constexpr int kStreamNnz = 2048;   // entries per streamed workgroup (CSR-stream, slabs)
constexpr int kStreamRows = 1024;  // rows per streamed workgroup
constexpr int kMaxSlabs = 8;
// Hot slab: the first columns of x (the internal order puts the columns of
// highest degree first), at most kHotCols of them (the entries of one
// streamed block's LDS), staged in LDS by every block of that slab
constexpr int kHotCols = kStreamNnz;
constexpr int kXcds = 8;           // MI355X: workgroup i runs on XCD i mod 8
constexpr double kXcdL2Bytes = 4.0 * 1024 * 1024;   // L2 of one XCD
// One workgroup of the column-slab kernel: rows [r0, r1) of slab `slab`, whose
// entries are [k0, k0 + cnt) of the slab arrays; cs = cnt | slab << 16.  One
// 16-byte load.
struct alignas(16) SlabBlock {
    int32_t r0, r1, k0, cs;
};
struct SpmvPlan {
    int lanes = 8;
    int stream = 0;                    // 1: CSR-stream kernel for the short rows
    int64_t n_sblocks = 0;
    int64_t *sblock = nullptr;         // [2 n_sblocks] row ranges [sblock[2b], sblock[2b+1])
    int64_t long_thr = 0;
    int64_t n_long = 0;
    int64_t n_chunks = 0;
    int32_t *long_rows = nullptr;      // [n_long]
    int64_t *long_chunk_ptr = nullptr; // [n_long+1]
    int32_t *chunk_row = nullptr;      // [n_chunks] long-row index
    int64_t *chunk_begin = nullptr;    // [n_chunks] first nnz
    int64_t *chunk_end = nullptr;      // [n_chunks] one past the last nnz
    double *chunk_part = nullptr;      // [n_chunks]
    // Column-slab form (n_slabs > 0): the columns are cut into n_slabs ranges
    // of equal entry counts and each slab is a CSR matrix over all rows, its
    // entries held contiguously from slab_base[s] (column slab_ci, values in
    // the matrix's sv/sv32, taken from entry slab_perm of the plain CSR); its
    // workgroups run on the XCDs given to it, so each XCD gathers from one
    // slab of x, and the slab sums of a row are added in slab order.
    int n_slabs = 0;                   // slabs in all, the hot slab included
    int hot_cols = 0;                  // > 0: slab 0 is the hot slab, columns [0, hot_cols)
    int64_t n_slab_blocks = 0;
    int64_t slab_base[kMaxSlabs + 2] = {};
    int32_t *slab_rp = nullptr;        // [n_slabs (rows+1)] row pointers into the slab arrays
    int32_t *slab_ci = nullptr;        // [nnz - long-row entries]
    int32_t *slab_perm = nullptr;      // [same]
    SlabBlock *slab_blk = nullptr;     // [n_slab_blocks]
    double *slab_part = nullptr;       // [n_slabs rows] per-slab row sums
    int32_t *long_of = nullptr;        // [rows] index of a long row in long_rows, else -1
                                       // (null when there is no long row)
};

// The finishing step of a sparse product (the slab sums of a row, or the chunk
// sums of a long row), left to the kernel that consumes the product so that
// the product costs one launch: value(y, i) is row i of the product, where y
// is what the product's first kernel wrote.  The sums are formed in the order
// of spmv's own finishing kernels (slab order, chunk order), so the results
// are the same bits.
struct ProductTail {
    const double *part = nullptr;   // [n_slabs rows] slab sums, or null
    int64_t rows = 0;
    int n_slabs = 0;
    const int32_t *long_of = nullptr;
    const int64_t *long_chunk_ptr = nullptr;
    const double *chunk_part = nullptr;
    __host__ __device__ bool active() const { return n_slabs > 0 || long_of != nullptr; }
#ifdef __HIPCC__
    __device__ double value(const double *y, int64_t i) const {
        if (long_of) {
            const int32_t l = long_of[i];
            if (l >= 0) {
                double s = 0.0;
                for (int64_t c = long_chunk_ptr[l]; c < long_chunk_ptr[l + 1]; ++c) s += chunk_part[c];
                return s;
            }
        }
        if (n_slabs == 0) return y[i];
        double acc = part[i];
        for (int k = 1; k < n_slabs; ++k) acc += part[k * rows + i];
        return acc;
    }
#endif
};

inline ProductTail tail_of(const SpmvPlan &p, int64_t rows) {
    ProductTail t;
    t.part = p.n_slabs > 0 ? p.slab_part : nullptr;
    t.rows = rows;
    t.n_slabs = p.n_slabs;
    t.long_of = p.n_long > 0 ? p.long_of : nullptr;
    t.long_chunk_ptr = p.long_chunk_ptr;
    t.chunk_part = p.chunk_part;
    return t;
}

// Iteration state kept on the device, read and written by the step kernels.
struct DevState {
    double eta, omega, tau, sigma;
    double beta_prev, r_prev;
    double eta_used, beta, ha, hb;    // last accepted step: Halpern weights (k+1)/(k+2), 1/(k+2)
    double eta_sum;                   // sum of eta_used since the restart
    double nx2, ny2, ip;              // reductions of the last attempt
    long long n_iter, kin, attempts_total, max_iter;
    int attempts_cur, halt, skip_update, status;
    // the step decision sets halt_next; the Halpern step of the same attempt
    // copies it to halt (the kernels of that attempt read a halt that does not
    // change under them); the host writes both
    int halt_next, pad_halt;
    int check_every, max_attempts, beta_mode, step_mode;
    int plain, pad_plain;             // plain: baseline PDHG, Halpern weights 1 and 0
    double beta_const, beta_grow, beta_shrink, step_reduce_exp, step_grow_exp;
    long long log_cap;
    int *log_attempts;
    double *log_eta, *log_beta, *log_omega;
    // replay of another run's decisions for the first rp_count accepted
    // iterations (parity harness): accept at attempt rp_attempts[k]; the
    // reflection parameter grows when rp_beta[k] >= beta_prev
    long long rp_count;
    const int *rp_attempts;
    const double *rp_beta;
};

// Per-candidate raw KKT reductions (unscaled quantities), see kkt kernels.
struct KktRaw {
    double rows_sum[3];   // y.h, ||y - y_anchor||^2 (scaled), unused
    double rows_max[3];   // max|r - P(r)|, max|Gx|, max|P(r)|
    double cols_sum[3];   // c.x, l.lam+ - u.lam-, ||x - x_anchor||^2 (scaled)
    double cols_max[3];   // max dist(lambda), max|G^T y|, unused
};

// ------------------------------------------------------------------ errors
struct HipError {
    hipError_t code;
    std::string where;
};
[[noreturn]] void throw_hip(hipError_t e, const char *what, const char *file, int line);
#define PDCS_HIP(call)                                                   \
    do {                                                                 \
        hipError_t _e = (call);                                          \
        if (_e != hipSuccess) ::pdcs::throw_hip(_e, #call, __FILE__, __LINE__); \
    } while (0)

// ------------------------------------------------------------ launch wrappers
// spmv.hip
// Rows whose instance's flag is set are skipped: `skip` names the flag in the
// per-instance states (SkipNone, SkipHalt: st[b].halt, SkipUpdate:
// st[b].skip_update), `row_inst` the instance of each row (null: instance 0).
enum SkipFlag { SkipNone = 0, SkipHalt = 1, SkipUpdate = 2 };
struct SpmvSkip {
    const DevState *st = nullptr;
    const int32_t *row_inst = nullptr;
    int flag = SkipNone;
};
void spmv(const Csr &A, const SpmvPlan &plan, const double *x, double *y, const SpmvSkip &skip,
          hipStream_t s);
// FP32 values (A.v32) and FP32 x, FP64 products and sums
void spmv32(const Csr &A, const SpmvPlan &plan, const float *x, double *y, const SpmvSkip &skip,
            hipStream_t s);
// The step decision of each instance, run by extra workgroups of a product's
// launch (see spmv_head): the partials of the primal and dual passes and
// their per-instance tile ranges (null for one problem).
struct DecideArgs {
    DevState *st = nullptr;   // null: no decision in this launch
    int64_t B = 0;
    const double *px = nullptr, *py = nullptr;
    const int64_t *tx = nullptr, *ty = nullptr;
    int64_t ntx = 0, nty = 0;
    int64_t nblk = 0;         // workgroups given to it (set by the launcher)
};
// The product's first kernel only; row i is then tail_of(plan, rows).value(y, i).
// With dec.st set, the launch also takes the step decision (workgroups
// [0, B rounded up to a multiple of 8), ahead of the product's, so the slab
// workgroups keep their XCDs).
void spmv_head(const Csr &A, const SpmvPlan &plan, const double *x, double *y,
               const SpmvSkip &skip, hipStream_t s, const DecideArgs &dec = DecideArgs{});
void spmv32_head(const Csr &A, const SpmvPlan &plan, const float *x, double *y,
                 const SpmvSkip &skip, hipStream_t s, const DecideArgs &dec = DecideArgs{});
void to_float(const double *in, float *out, int64_t n, hipStream_t s);
int choose_lanes(double avg_row_nnz);
// Workgroups of the first kernel of a product under `plan` (the step
// decision's workgroups not counted).  A launch holds at most
// kMaxLaunchBlocks workgroups of kBlock work-items (2^31 work-items).
int64_t spmv_blocks(const Csr &A, const SpmvPlan &plan);
constexpr int64_t kMaxLaunchBlocks = (((int64_t)1 << 31) - 1) / kBlock - 64;

// setup.hip
// One diagonal block of a block-diagonal CSR matrix (an instance of a batch).
struct TBlock {
    int64_t r0, rows, c0, cols, k0, nnz;
};
// At (arrays preallocated) = A^T, block by block; each block below 2^31 entries
void transpose_csr(const Csr &A, Csr &At, const TBlock *blocks, int64_t nblocks, hipStream_t s);
void fill(double *p, int64_t n, double v, hipStream_t s);
void rows_absmax_scaled(const Csr &A, const double *er, const double *ec, bool row_first,
                        double *out, hipStream_t s);
void rows_abssum_scaled(const Csr &A, const double *er, const double *ec, bool row_first,
                        double *out, hipStream_t s);
void divide_by_sqrt(double *e, const double *r, int64_t n, hipStream_t s);
void scale_values(const Csr &A, const double *er, const double *ec, bool row_first, double *out,
                  hipStream_t s);
void scale_problem_vectors(int64_t n, int64_t m, int64_t n_box, const double *c,
                           const double *h, const double *l, const double *u, const double *e,
                           const double *f, double *cs, double *hs, double *ls, double *us,
                           double *dx, double *dy, hipStream_t s);
// out[0] += sum(a*a) style helpers: single-pass deterministic reductions
void reduce_absmax(const double *a, int64_t n, double *out, hipStream_t s);
void reduce_sumsq(const double *a, int64_t n, double *out, hipStream_t s);
void check_finite(const double *a, int64_t n, int *flag, hipStream_t s);
void div_vec(const double *a, const double *b, double *out, int64_t n, hipStream_t s);
void mul_vec(const double *a, const double *b, double *out, int64_t n, hipStream_t s);
void copy_vec(const double *a, double *out, int64_t n, hipStream_t s);
// v = w / sqrt(*sumsq) on the device (no host round trip)
void scale_by_inv_sqrt(const double *w, const double *sumsq, const int32_t *map, double *v,
                       int64_t n, hipStream_t s);
void fill_by_inst(double *out, const int32_t *map, const double *vals, int64_t n, hipStream_t s);
void gather(double *out, const double *in, const int32_t *idx, int64_t n, hipStream_t s);
void scatter(double *out, const double *in, const int32_t *idx, int64_t n, int64_t base,
             hipStream_t s);
void relabel(int32_t *ci, int64_t nnz, const int32_t *pos, hipStream_t s);
// (v[o], v[o+1]) <- ((v[o] + v[o+1])/sqrt 2, (v[o] - v[o+1])/sqrt 2) for each
// o = offs[t] - base, t < count: the map between a rotated SOC and an SOC.
void rotate_pairs(double *v, const int64_t *offs, int64_t count, int64_t base, hipStream_t s);
// A.sv (and A.sv32 when both A.v32 and A.sv32 are set) <- the values in the
// slab order of p (the caller allocates them).  No-op for a plan without slabs.
void slab_values(const Csr &A, const SpmvPlan &p, hipStream_t s);
void reduce_segments(int mode, const double *a, const int64_t *off, int64_t B, double *out,
                     hipStream_t s);

// cone_pass.hip
// `st` points at the batch's array of per-instance states (one for a single problem).
struct PrimalArgs {
    const double *x, *aty, *cs, *ls, *us, *dx;
    double *xh;
    const DevState *st;
    float *xh32 = nullptr;   // FP32 copy of x^ for the FP32 product (mixed form)
    int fp32proj = 0;        // 1: lane-group SOC and exponential projections in FP32
};
struct DualArgs {
    const double *y, *gxh, *gx, *hs, *dy;
    double *yh;
    const DevState *st;
    float *yh32 = nullptr;   // FP32 copy of y^ for the FP32 product (mixed form)
    int fp32proj = 0;        // 1: lane-group SOC and exponential projections in FP32
    // when active, G~x^ is finished here from what spmv_head left in gxh, and
    // written to gxh_out
    ProductTail gt{};
    double *gxh_out = nullptr;
};
struct CandArgs {  // projection of src / div onto the scaled set, into dst
    const double *src, *ls, *us, *d;
    const DevState *st;   // div = st->eta_sum when use_avg
    int use_avg;
    double *dst;
};
struct KktRowsArgs {
    const double *gxc, *h, *e, *yc, *ya;
    double *tmp;
};
struct KktColsArgs {
    const double *atyc, *c, *f, *l, *u, *xc, *xa;
    double *tmp;
};
struct ProjArgs {
    double *v;
    const double *d;
    int fp32proj = 0;        // 1: lane-group SOC and exponential projections in FP32
};
void pass_primal(const ConePlan &p, const PrimalArgs &a, double *partials, hipStream_t s);
void pass_dual(const ConePlan &p, const DualArgs &a, double *partials, hipStream_t s);
void pass_candidate(const ConePlan &p, bool y_side, const CandArgs &a, double *partials,
                    hipStream_t s);
void pass_kkt_rows(const ConePlan &p, const KktRowsArgs &a, double *partials, hipStream_t s);
void pass_kkt_cols(const ConePlan &p, const KktColsArgs &a, double *partials, hipStream_t s);
void pass_project(const ConePlan &p, bool dual, const ProjArgs &a, double *partials,
                  hipStream_t s);
// Zeroes the grid-level SOC blocks' barrier counters and error flag (a kernel,
// so the clear may also sit in a captured graph).
void clear_grid(const ConePlan &p, hipStream_t s);

// iterate.hip
struct HalpernArgs {
    double *x, *aty, *xsum;
    const double *xh, *atyh, *xa, *aty0;
    double *y, *gx, *ysum;
    const double *yh, *gxh, *ya, *gx0;
    int64_t n, m;
    const DevState *st;
    const int32_t *x_inst = nullptr, *y_inst = nullptr;   // batch: instance per entry
    // when active, G~^T y^ is finished here from what spmv_head left in atyh
    // (atyh itself is not updated)
    ProductTail at{};
    // when set, halt <- halt_next for these n_inst states (the decision ran in
    // the same attempt's G~^T launch)
    DevState *promote = nullptr;
    int64_t n_inst = 0;
};
void halpern(const HalpernArgs &a, hipStream_t s);
void reduce_kkt(int64_t B, const double *prow, const int64_t *ty, int64_t ntr, const double *pcol,
                const int64_t *tx, int64_t ntc, KktRaw *out, hipStream_t s);
// Restart of each instance b with code[b] = 1 (from candidate set 0) or 2 (set
// 1), 0 = untouched; code null: every entry from set 0.
struct RestartArgs {
    int64_t n, m;
    const double *xc[2], *yc[2], *gxc[2], *atyc[2];
    const int32_t *code, *x_inst, *y_inst;
    double *x, *y, *xa, *ya, *gx, *aty, *gx0, *aty0, *xsum, *ysum;
};
void restart_copy(const RestartArgs &a, hipStream_t s);
void unscale(const double *xs, const double *f, double *out, int64_t n, hipStream_t s);

// mlp.hip
void gemm_bf16(int ta, int tb, int64_t M, int64_t N, int64_t K, const uint16_t *a, int64_t lda,
               const uint16_t *b, int64_t ldb, const float *bias, int relu, float *c32,
               uint16_t *c16, int64_t ldc, hipStream_t s);
// gemm_bf16 for ta = 0, tb = 1 with K split over chunks whose partial products
// go to ws (ws_elems floats), added in chunk order by a second kernel; false
// (nothing launched) when the shape has enough output tiles, K is short, the
// operands are not 16-byte aligned or ws holds fewer than two chunks.
bool gemm_bf16_split(int64_t M, int64_t N, int64_t K, const uint16_t *a, int64_t lda,
                     const uint16_t *b, int64_t ldb, const float *bias, int relu, float *c32,
                     uint16_t *c16, int64_t ldc, float *ws, int64_t ws_elems, hipStream_t s);
void to_bf16(const float *in, uint16_t *out, int64_t n, hipStream_t s);
// Both hidden layers of the network in one launch (theta FP32 in; theta's BF16
// copy, h1 and h2 in FP32 and BF16 out); false (nothing launched) for shapes
// it does not cover.
bool mlp_hidden(int64_t B, int64_t in, int64_t hid, const float *theta, const uint16_t *w1,
                const float *b1, const uint16_t *w2, const float *b2, uint16_t *xb, float *h1,
                uint16_t *h1b, float *h2, uint16_t *h2b, hipStream_t s);
void mse_grad(const float *out, const float *target, int64_t n, int64_t cols, int64_t ld16,
              float inv, float *d32, uint16_t *d16, double *part, hipStream_t s);
void transpose_bf16(const uint16_t *in, int64_t rows, int64_t cols, int64_t ldi, uint16_t *out,
                    int64_t ldo, hipStream_t s);
void relu_back(const float *dh, const float *z, int64_t n, float *dz32, uint16_t *dz16, hipStream_t s);
void colsum(const float *d, int64_t rows, int64_t cols, float *db, hipStream_t s);
void adam(float *p, const float *g, float *m1, float *m2, int64_t n, float lr, float b1, float b2,
          float eps, float c1, float c2, uint16_t *p16, hipStream_t s);
void scale_in(const double *xu, const double *f, double *out, int64_t n, hipStream_t s);

}  // namespace pdcs
