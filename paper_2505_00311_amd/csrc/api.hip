// api.hip -- the C ABI of include/pdcs.h and the host controller of
// Algorithm 1 (Section 3).
//
// The controller enqueues step attempts in batches on the caller's stream.  An
// attempt is: primal pass (x^ and ||dx||^2), SpMV G~x^, dual pass (y^, ||dy||^2,
// <dy, G~dx>), the on-device step decision, SpMV G~^T y^ and the Halpern/average
// update; the last two are skipped on the device when the step is rejected and
// everything is skipped once the device flags a due check.  The host
// synchronises once per batch (every 64 accepted iterations), evaluates the
// two restart candidates there, and decides restart, primal weight and
// termination from about twenty reduced scalars.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <vector>

#include "../../include/pdcs.h"
#include "internal.hpp"

namespace pdcs {

[[noreturn]] void throw_hip(hipError_t e, const char *what, const char *file, int line) {
    throw HipError{e, std::string(what) + " failed at " + file + ":" + std::to_string(line) + ": " +
                          hipGetErrorString(e)};
}

struct ApiError {
    pdcs_status code;
    std::string msg;
};

[[noreturn]] static void fail(pdcs_status c, const std::string &m) { throw ApiError{c, m}; }

static thread_local std::string g_last_error;

// ------------------------------------------------------------- device memory
struct DevMem {
    std::vector<void *> ptrs;
    template <class T>
    T *alloc(int64_t n) {
        void *p = nullptr;
        const size_t bytes = sizeof(T) * (size_t)(n > 0 ? n : 1);
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess)
            fail(e == hipErrorOutOfMemory ? PDCS_ERR_OOM : PDCS_ERR_HIP,
                 "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
        ptrs.push_back(p);
        return (T *)p;
    }
    ~DevMem() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

template <class T>
static void h2d(T *dst, const T *src, int64_t n, hipStream_t s) {
    if (n > 0) PDCS_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyHostToDevice, s));
}
template <class T>
static void d2h(T *dst, const T *src, int64_t n, hipStream_t s) {
    if (n > 0) PDCS_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyDeviceToHost, s));
}
template <class T>
static void d2d(T *dst, const T *src, int64_t n, hipStream_t s) {
    if (n > 0) PDCS_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
}

// ---------------------------------------------------------------- plans
struct HostPlan {
    std::vector<Tile> tiles;
    std::vector<int64_t> soc_off, exp_off;
    std::vector<int32_t> soc_dim;
};

static int elem_kind(int32_t t) {
    return t == kZero ? kTileZero : t == kFree ? kTileFree : kTileNonneg;
}

// Tiles for entries [0, n_box) (box) and the cone blocks starting at `base`.
// Heavy classes come first so that they start early: large SOC (workgroup),
// small SOC (wavefront), exponential (thread), then elementwise runs.
static HostPlan build_plan(int64_t base, int64_t n_box, const std::vector<int32_t> &types,
                           const std::vector<int64_t> &dims) {
    HostPlan P;
    std::vector<Tile> elem;
    auto push_run = [&](int kind, int64_t start, int64_t len) {
        for (int64_t o = 0; o < len; o += kElemPerTile)
            elem.push_back(Tile{kind, (int32_t)std::min<int64_t>(kElemPerTile, len - o), start + o});
    };
    push_run(kTileBox, 0, n_box);
    // SOC size classes: lanes per block 8, 16, 32, 64 (1 entry per lane), then
    // one wavefront with 2 or 4 entries per lane, then a workgroup per block
    constexpr int kClasses = 7;
    const int class_kind[kClasses] = {kTileSoc8, kTileSoc16, kTileSoc32, kTileSoc64,
                                      kTileSoc128, kTileSoc256, kTileSocBlock};
    const int class_per_tile[kClasses] = {32, 16, 8, 4, 4, 4, 1};
    auto soc_class = [](int64_t d) {
        return d <= 8 ? 0 : d <= 16 ? 1 : d <= 32 ? 2 : d <= 64 ? 3 : d <= 128 ? 4 : d <= 256 ? 5 : 6;
    };
    std::vector<std::pair<int64_t, int64_t>> soc[kClasses];
    std::vector<int64_t> ep, ed;
    int run_kind = -1;
    int64_t run_start = 0, run_len = 0, off = base;
    for (size_t b = 0; b < types.size(); ++b) {
        const int32_t t = types[b];
        const int64_t d = dims[b];
        if (t == kZero || t == kFree || t == kNonneg) {
            const int k = elem_kind(t);
            if (k == run_kind && run_start + run_len == off) {
                run_len += d;
            } else {
                if (run_len) push_run(run_kind, run_start, run_len);
                run_kind = k, run_start = off, run_len = d;
            }
        } else if (t == kSoc) {
            soc[soc_class(d)].push_back({off, d});
        } else if (t == kExp) {
            ep.push_back(off);
        } else {
            ed.push_back(off);
        }
        off += d;
    }
    if (run_len) push_run(run_kind, run_start, run_len);
    // largest classes first: they run longest
    for (int c = kClasses - 1; c >= 0; --c) {
        const int64_t first = (int64_t)P.soc_off.size();
        for (auto &p : soc[c]) P.soc_off.push_back(p.first), P.soc_dim.push_back((int32_t)p.second);
        const int64_t cnt = (int64_t)soc[c].size();
        for (int64_t i = 0; i < cnt; i += class_per_tile[c])
            P.tiles.push_back(Tile{class_kind[c],
                                   (int32_t)std::min<int64_t>(class_per_tile[c], cnt - i), first + i});
    }
    for (auto o : ep) P.exp_off.push_back(o);
    for (auto o : ed) P.exp_off.push_back(o);
    for (int64_t i = 0; i < (int64_t)ep.size(); i += kExpPerTile)
        P.tiles.push_back(Tile{kTileExp, (int32_t)std::min<int64_t>(kExpPerTile, ep.size() - i), i});
    for (int64_t i = 0; i < (int64_t)ed.size(); i += kExpPerTile)
        P.tiles.push_back(Tile{kTileExpDual, (int32_t)std::min<int64_t>(kExpPerTile, ed.size() - i),
                               (int64_t)ep.size() + i});
    for (auto &t : elem) P.tiles.push_back(t);
    return P;
}

static ConePlan upload_plan(DevMem &mem, const HostPlan &H, hipStream_t s) {
    ConePlan P;
    P.ntiles = (int64_t)H.tiles.size();
    P.tiles = mem.alloc<Tile>(P.ntiles);
    P.soc_off = mem.alloc<int64_t>((int64_t)H.soc_off.size());
    P.soc_dim = mem.alloc<int32_t>((int64_t)H.soc_dim.size());
    P.exp_off = mem.alloc<int64_t>((int64_t)H.exp_off.size());
    h2d(P.tiles, H.tiles.data(), P.ntiles, s);
    h2d(P.soc_off, H.soc_off.data(), (int64_t)H.soc_off.size(), s);
    h2d(P.soc_dim, H.soc_dim.data(), (int64_t)H.soc_dim.size(), s);
    h2d(P.exp_off, H.exp_off.data(), (int64_t)H.exp_off.size(), s);
    P.n_soc = (int64_t)H.soc_off.size();
    P.n_exp = (int64_t)H.exp_off.size();
    PDCS_HIP(hipStreamSynchronize(s));  // the host vectors die with the caller's frame
    return P;
}

static SpmvPlan build_spmv_plan(DevMem &mem, const std::vector<int64_t> &rp, hipStream_t s) {
    SpmvPlan P;
    const int64_t rows = (int64_t)rp.size() - 1;
    const int64_t nnz = rp.back();
    const double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
    P.lanes = choose_lanes(rows > 0 ? avg : 1.0);
    P.long_thr = std::max<int64_t>(64, 32 * P.lanes);
    P.stream = avg < 12.0 ? 1 : 0;
    if (P.stream) P.long_thr = std::min<int64_t>(P.long_thr, kStreamNnz);
    // rows longer than long_thr: chunks of kLongChunk entries
    std::vector<int32_t> lr, crow;
    std::vector<int64_t> cptr{0}, cbeg;
    for (int64_t i = 0; i < rows; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        if (len <= P.long_thr) continue;
        const int32_t li = (int32_t)lr.size();
        lr.push_back((int32_t)i);
        for (int64_t b = rp[i]; b < rp[i + 1]; b += kLongChunk) crow.push_back(li), cbeg.push_back(b);
        cptr.push_back((int64_t)cbeg.size());
    }
    // CSR-stream row ranges (start, end) of consecutive short rows whose entries
    // fit in kStreamNnz; a long row closes the range
    std::vector<int64_t> sb;
    if (P.stream) {
        int64_t start = 0, acc = 0;
        for (int64_t i = 0; i < rows; ++i) {
            const int64_t len = rp[i + 1] - rp[i];
            if (len > P.long_thr) {
                if (i > start) sb.push_back(start), sb.push_back(i);
                start = i + 1, acc = 0;
                continue;
            }
            if (acc + len > kStreamNnz) {
                sb.push_back(start), sb.push_back(i);
                start = i, acc = 0;
            }
            acc += len;
        }
        if (rows > start) sb.push_back(start), sb.push_back(rows);
    }
    P.n_long = (int64_t)lr.size();
    P.n_chunks = (int64_t)cbeg.size();
    P.n_sblocks = (int64_t)sb.size() / 2;
    P.long_rows = mem.alloc<int32_t>(P.n_long);
    P.long_chunk_ptr = mem.alloc<int64_t>(P.n_long + 1);
    P.chunk_row = mem.alloc<int32_t>(P.n_chunks);
    P.chunk_begin = mem.alloc<int64_t>(P.n_chunks);
    P.chunk_part = mem.alloc<double>(P.n_chunks);
    P.sblock = mem.alloc<int64_t>((int64_t)sb.size());
    h2d(P.long_rows, lr.data(), P.n_long, s);
    h2d(P.long_chunk_ptr, cptr.data(), P.n_long + 1, s);
    h2d(P.chunk_row, crow.data(), P.n_chunks, s);
    h2d(P.chunk_begin, cbeg.data(), P.n_chunks, s);
    h2d(P.sblock, sb.data(), (int64_t)sb.size(), s);
    PDCS_HIP(hipStreamSynchronize(s));
    return P;
}

}  // namespace pdcs

using namespace pdcs;

// ------------------------------------------------------------------ problem
struct pdcs_problem {
    int64_t n = 0, m = 0, nnz = 0, n_box = 0;
    hipStream_t stream = nullptr;
    DevMem mem;
    std::vector<int32_t> xt, rt;
    std::vector<int64_t> xd, rd;
    Csr G, Gt;                     // unscaled
    Csr Gs, Gts;                   // scaled values, shared structure
    SpmvPlan pG, pGt;
    ConePlan planX, planY;
    double *c, *h, *l, *u, *ones_n, *ones_m;
    double *e, *f, *cs, *hs, *ls, *us, *dx, *dy;
    double *x, *y, *xa, *ya, *xh, *yh, *aty, *gx, *aty0, *gx0, *atyh, *gxh, *xsum, *ysum;
    double *xc[2], *yc[2], *gxc[2], *atyc[2], *tmp_n, *tmp_m;
    double *partX, *partY, *scal;
    KktRaw *kraw;
    DevState *st;
    int *flag;
    double cinf = 0, hinf = 0;
    int scaled_ruiz = -1, scaled_pc = -1;
    double gmax = 0, cs_norm = 0, hs_norm = 0;
    // a captured batch of step attempts, replayed on a library stream
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t gexec = nullptr;
    // timing events of settings.time_kernels: (PDCS_K_COUNT + 1) per attempt
    std::vector<hipEvent_t> tev;
    ~pdcs_problem() {
        for (hipEvent_t e : tev) (void)hipEventDestroy(e);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (gstream) (void)hipStreamDestroy(gstream);
    }
};

constexpr int kGraphBatch = 64;   // step attempts per captured graph

static void validate_cones(int64_t nblk, const int32_t *t, const int64_t *d, int64_t expect,
                           const char *what, std::vector<int32_t> &ot, std::vector<int64_t> &od) {
    if (nblk < 0 || (nblk > 0 && (!t || !d))) fail(PDCS_ERR_INVALID_ARG, std::string(what) + ": bad cone list");
    int64_t sum = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        if (t[b] < kZero || t[b] > kExpDual) fail(PDCS_ERR_INVALID_ARG, std::string(what) + ": unknown cone type");
        if (d[b] < 1) fail(PDCS_ERR_DIMENSION, std::string(what) + ": cone of dimension < 1");
        if ((t[b] == kExp || t[b] == kExpDual) && d[b] != 3)
            fail(PDCS_ERR_DIMENSION, std::string(what) + ": exponential cone of dimension != 3");
        if (d[b] > INT32_MAX) fail(PDCS_ERR_NOT_SUPPORTED, std::string(what) + ": cone too large");
        sum += d[b];
        ot.push_back(t[b]);
        od.push_back(d[b]);
    }
    if (sum != expect)
        fail(PDCS_ERR_DIMENSION, std::string(what) + ": cone dimensions sum to " + std::to_string(sum) +
                                     ", expected " + std::to_string(expect));
}

__global__ void validate_csr_kernel(const int64_t *rp, int64_t m, const int32_t *ci, int64_t nnz,
                                    int64_t n, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && rp[i] > rp[i + 1]) atomicOr(flag, 2);
    if (i == 0 && (rp[0] != 0 || rp[m] != nnz)) atomicOr(flag, 2);
    if (i < nnz && (ci[i] < 0 || ci[i] >= n)) atomicOr(flag, 2);
}

__global__ void validate_bounds_kernel(const double *l, const double *u, int64_t nb, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb && (l[i] != l[i] || u[i] != u[i] || l[i] > u[i] || l[i] == INFINITY ||
                   u[i] == -INFINITY))
        atomicOr(flag, 4);
}

static pdcs_problem *create_impl(const pdcs_problem_desc *D, void *stream, bool on_device) {
    if (!D) fail(PDCS_ERR_INVALID_ARG, "desc is NULL");
    if (D->n < 1 || D->m < 0 || D->nnz < 0 || D->n_box < 0 || D->n_box > D->n)
        fail(PDCS_ERR_INVALID_ARG, "bad sizes");
    if (D->nnz >= ((int64_t)1 << 31)) fail(PDCS_ERR_NOT_SUPPORTED, "nnz must be below 2^31");
    if (D->n >= ((int64_t)1 << 31) || D->m >= ((int64_t)1 << 31))
        fail(PDCS_ERR_NOT_SUPPORTED, "n and m must be below 2^31");
    if (!D->row_ptr || (D->nnz > 0 && (!D->col || !D->val)) || !D->c || (D->m > 0 && !D->h) ||
        (D->n_box > 0 && (!D->l || !D->u)))
        fail(PDCS_ERR_INVALID_ARG, "NULL array");
    auto P = std::make_unique<pdcs_problem>();
    P->n = D->n, P->m = D->m, P->nnz = D->nnz, P->n_box = D->n_box;
    P->stream = (hipStream_t)stream;
    validate_cones(D->n_xcones, D->xcone_type, D->xcone_dim, D->n - D->n_box, "x cones", P->xt, P->xd);
    validate_cones(D->n_rcones, D->rcone_type, D->rcone_dim, D->m, "row cones", P->rt, P->rd);
    const int64_t n = P->n, m = P->m, nnz = P->nnz, nb = P->n_box;
    hipStream_t s = P->stream;
    DevMem &M = P->mem;
    P->G = Csr{m, n, nnz, M.alloc<int64_t>(m + 1), M.alloc<int32_t>(nnz), M.alloc<double>(nnz)};
    P->Gt = Csr{n, m, nnz, M.alloc<int64_t>(n + 1), M.alloc<int32_t>(nnz), M.alloc<double>(nnz)};
    P->c = M.alloc<double>(n);
    P->h = M.alloc<double>(m);
    P->l = M.alloc<double>(nb);
    P->u = M.alloc<double>(nb);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        if (bytes) PDCS_HIP(hipMemcpyAsync(dst, src, bytes, kind, s));
    };
    cp(P->G.rp, D->row_ptr, sizeof(int64_t) * (m + 1));
    cp(P->G.ci, D->col, sizeof(int32_t) * nnz);
    cp(P->G.v, D->val, sizeof(double) * nnz);
    cp(P->c, D->c, sizeof(double) * n);
    cp(P->h, D->h, sizeof(double) * m);
    cp(P->l, D->l, sizeof(double) * nb);
    cp(P->u, D->u, sizeof(double) * nb);
    P->flag = M.alloc<int>(4);
    PDCS_HIP(hipMemsetAsync(P->flag, 0, sizeof(int) * 4, s));
    const int64_t vk = std::max(m + 1, nnz);
    hipLaunchKernelGGL(validate_csr_kernel, dim3((unsigned)((vk + 255) / 256)), dim3(256), 0, s,
                       P->G.rp, m, P->G.ci, nnz, n, P->flag);
    if (nb > 0)
        hipLaunchKernelGGL(validate_bounds_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0,
                           s, P->l, P->u, nb, P->flag);
    check_finite(P->G.v, nnz, P->flag, s);
    check_finite(P->c, n, P->flag, s);
    check_finite(P->h, m, P->flag, s);
    int flag = 0;
    d2h(&flag, P->flag, 1, s);
    PDCS_HIP(hipStreamSynchronize(s));
    if (flag & 2) fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
    if (flag & 4) fail(PDCS_ERR_INVALID_ARG, "bounds: NaN, l > u, l = +inf or u = -inf");
    if (flag & 1) fail(PDCS_ERR_NONFINITE, "non-finite value in G, c or h");

    transpose_csr(P->G, P->Gt, s);
    std::vector<int64_t> hrp(m + 1), hrpt(n + 1);
    d2h(hrp.data(), P->G.rp, m + 1, s);
    d2h(hrpt.data(), P->Gt.rp, n + 1, s);
    PDCS_HIP(hipStreamSynchronize(s));
    P->pG = build_spmv_plan(M, hrp, s);
    P->pGt = build_spmv_plan(M, hrpt, s);
    P->planX = upload_plan(M, build_plan(nb, nb, P->xt, P->xd), s);
    P->planY = upload_plan(M, build_plan(0, 0, P->rt, P->rd), s);

    P->Gs = Csr{m, n, nnz, P->G.rp, P->G.ci, M.alloc<double>(nnz)};
    P->Gts = Csr{n, m, nnz, P->Gt.rp, P->Gt.ci, M.alloc<double>(nnz)};
    P->ones_n = M.alloc<double>(n);
    P->ones_m = M.alloc<double>(m);
    fill(P->ones_n, n, 1.0, s);
    fill(P->ones_m, m, 1.0, s);
    P->e = M.alloc<double>(m), P->f = M.alloc<double>(n);
    P->cs = M.alloc<double>(n), P->hs = M.alloc<double>(m);
    P->ls = M.alloc<double>(nb), P->us = M.alloc<double>(nb);
    P->dx = M.alloc<double>(n), P->dy = M.alloc<double>(m);
    double **xs[] = {&P->x, &P->xa, &P->xh, &P->aty, &P->aty0, &P->atyh, &P->xsum, &P->tmp_n,
                     &P->xc[0], &P->xc[1], &P->atyc[0], &P->atyc[1]};
    for (double **v : xs) *v = M.alloc<double>(n);
    double **ys[] = {&P->y, &P->ya, &P->yh, &P->gx, &P->gx0, &P->gxh, &P->ysum, &P->tmp_m,
                     &P->yc[0], &P->yc[1], &P->gxc[0], &P->gxc[1]};
    for (double **v : ys) *v = M.alloc<double>(m);
    for (ConePlan *pl : {&P->planX, &P->planY}) {
        pl->soc_root = M.alloc<double>(pl->n_soc);
        pl->exp_root = M.alloc<double>(pl->n_exp);
    }
    P->partX = M.alloc<double>(P->planX.ntiles * kPartials);
    P->partY = M.alloc<double>(P->planY.ntiles * kPartials);
    P->scal = M.alloc<double>(8);
    P->kraw = M.alloc<KktRaw>(3);
    P->st = M.alloc<DevState>(1);
    reduce_absmax(P->c, n, P->scal + 0, s);
    reduce_absmax(P->h, m, P->scal + 1, s);
    double nrm[2] = {0, 0};
    d2h(nrm, P->scal, 2, s);
    PDCS_HIP(hipStreamSynchronize(s));
    P->cinf = nrm[0], P->hinf = m > 0 ? nrm[1] : 0.0;
    return P.release();
}

// Rescaling of Section 3 (reading: Ruiz passes + one Pock-Chambolle pass),
// cached for the parameters it was computed with.
static void ensure_scaling(pdcs_problem *P, int ruiz, int pc) {
    if (P->scaled_ruiz == ruiz && P->scaled_pc == pc) return;
    hipStream_t s = P->stream;
    const int64_t n = P->n, m = P->m;
    fill(P->e, m, 1.0, s);
    fill(P->f, n, 1.0, s);
    for (int it = 0; it < ruiz + (pc ? 1 : 0); ++it) {
        const bool is_pc = it >= ruiz;
        if (is_pc) {
            rows_abssum_scaled(P->G, P->e, P->f, true, P->tmp_m, s);
            rows_abssum_scaled(P->Gt, P->f, P->e, false, P->tmp_n, s);
        } else {
            rows_absmax_scaled(P->G, P->e, P->f, true, P->tmp_m, s);
            rows_absmax_scaled(P->Gt, P->f, P->e, false, P->tmp_n, s);
        }
        divide_by_sqrt(P->e, P->tmp_m, m, s);
        divide_by_sqrt(P->f, P->tmp_n, n, s);
    }
    scale_values(P->G, P->e, P->f, true, P->Gs.v, s);
    scale_values(P->Gt, P->f, P->e, false, P->Gts.v, s);
    scale_problem_vectors(n, m, P->n_box, P->c, P->h, P->l, P->u, P->e, P->f, P->cs, P->hs, P->ls,
                          P->us, P->dx, P->dy, s);
    reduce_absmax(P->Gs.v, P->nnz, P->scal + 2, s);
    reduce_sumsq(P->cs, n, P->scal + 3, s);
    reduce_sumsq(P->hs, m, P->scal + 4, s);
    double r[3] = {0, 0, 0};
    d2h(r, P->scal + 2, 3, s);
    PDCS_HIP(hipStreamSynchronize(s));
    P->gmax = P->nnz > 0 ? r[0] : 0.0;
    P->cs_norm = std::sqrt(r[1]);
    P->hs_norm = m > 0 ? std::sqrt(r[2]) : 0.0;
    P->scaled_ruiz = ruiz, P->scaled_pc = pc;
}

// Fixed step step_fixed / ||G~||_2, the norm by power iteration on G~^T G~ from
// the normalised all-ones vector (the plain-PDHG step of the ablation).
static double fixed_step(pdcs_problem *P, const pdcs_settings *S) {
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    fill(P->tmp_n, n, 1.0 / std::sqrt((double)n), s);
    for (int it = 0; it < S->power_iters; ++it) {
        spmv(P->Gs, P->pG, P->tmp_n, P->tmp_m, nullptr, s);
        spmv(P->Gts, P->pGt, P->tmp_m, P->atyh, nullptr, s);
        reduce_sumsq(P->atyh, n, P->scal + 5, s);
        scale_by_inv_sqrt(P->atyh, P->scal + 5, P->tmp_n, n, s);
    }
    double lam2 = 0.0;
    d2h(&lam2, P->scal + 5, 1, s);
    PDCS_HIP(hipStreamSynchronize(s));
    const double lam = std::sqrt(lam2);
    return (S->power_iters > 0 && lam > 0.0) ? S->step_fixed / std::sqrt(lam) : 1.0;
}

struct Kkt {
    double err_p, err_d, err_gap, pobj, dobj, dx2, dy2;
    double avg() const { return (err_p + err_d + err_gap) / 3.0; }
    double mx() const { return std::max(err_p, std::max(err_d, err_gap)); }
};

static Kkt kkt_from_raw(const pdcs_problem *P, const KktRaw &r) {
    Kkt k;
    k.err_p = r.rows_max[0] / (1.0 + std::max(P->hinf, std::max(r.rows_max[1], r.rows_max[2])));
    k.err_d = r.cols_max[0] / (1.0 + std::max(P->cinf, r.cols_max[1]));
    k.pobj = r.cols_sum[0];
    k.dobj = r.rows_sum[0] + r.cols_sum[1];
    k.err_gap = std::fabs(k.pobj - k.dobj) / (1.0 + std::max(std::fabs(k.pobj), std::fabs(k.dobj)));
    k.dx2 = r.cols_sum[2];
    k.dy2 = r.rows_sum[1];
    return k;
}

// Enqueue the termination measures of the scaled point (xc, yc) with products
// gxc = G~xc and atyc = G~^T yc into kraw[slot]; distances are to (xa, ya).
static void enqueue_kkt(pdcs_problem *P, const double *xc, const double *yc, const double *gxc,
                        const double *atyc, const double *xa, const double *ya, const double *e,
                        const double *f, int slot) {
    hipStream_t s = P->stream;
    pass_kkt_rows(P->planY, KktRowsArgs{gxc, P->h, e, yc, ya, P->tmp_m}, P->partY, s);
    pass_kkt_cols(P->planX, KktColsArgs{atyc, P->c, f, P->l, P->u, xc, xa, P->tmp_n}, P->partX, s);
    reduce_kkt(P->partY, P->planY.ntiles, P->partX, P->planX.ntiles, P->kraw + slot, s);
}

static void fill_info(pdcs_info *info, int status, const DevState &hs, long long restarts,
                      long long spmv, const Kkt &k, double setup_s, double solve_s) {
    if (!info) return;
    info->status = status;
    info->iterations = hs.n_iter;
    info->attempts = hs.attempts_total;
    info->restarts = restarts;
    info->spmv = spmv;
    info->pobj = k.pobj, info->dobj = k.dobj;
    info->err_p = k.err_p, info->err_d = k.err_d, info->err_gap = k.err_gap;
    info->omega = hs.omega, info->eta = hs.eta;
    info->setup_s = setup_s, info->solve_s = solve_s;
    for (int j = 0; j < PDCS_K_COUNT; ++j) info->kernel_ms[j] = 0.0, info->kernel_launches[j] = 0;
}

// One step attempt of Algorithm 1 (see the file header), `batch` times.  With
// `ev`, event ev[(PDCS_K_COUNT + 1) b + j] is recorded before kernel j of
// attempt b and ev[(PDCS_K_COUNT + 1) b + PDCS_K_COUNT] after its last kernel.
static void enqueue_attempts(pdcs_problem *P, long long batch, hipStream_t s,
                             const hipEvent_t *ev = nullptr) {
    const PrimalArgs pa{P->x, P->aty, P->cs, P->ls, P->us, P->dx, P->xh, P->st};
    const DualArgs da{P->y, P->gxh, P->gx, P->hs, P->dy, P->yh, P->st};
    const HalpernArgs ha{P->x, P->aty, P->xsum, P->xh, P->atyh, P->xa, P->aty0,
                         P->y, P->gx, P->ysum, P->yh, P->gxh, P->ya, P->gx0, P->n, P->m, P->st};
    constexpr int E = PDCS_K_COUNT + 1;
    auto mark = [&](long long b, int j) {
        if (ev) PDCS_HIP(hipEventRecord(ev[E * b + j], s));
    };
    for (long long b = 0; b < batch; ++b) {
        mark(b, PDCS_K_PRIMAL);
        pass_primal(P->planX, pa, P->partX, s);
        mark(b, PDCS_K_SPMV_G);
        spmv(P->Gs, P->pG, P->xh, P->gxh, &P->st->halt, s);
        mark(b, PDCS_K_DUAL);
        pass_dual(P->planY, da, P->partY, s);
        mark(b, PDCS_K_DECIDE);
        decide(P->st, P->partX, P->planX.ntiles, P->partY, P->planY.ntiles, s);
        mark(b, PDCS_K_SPMV_GT);
        spmv(P->Gts, P->pGt, P->yh, P->atyh, &P->st->skip_update, s);
        mark(b, PDCS_K_HALPERN);
        halpern(ha, s);
        mark(b, PDCS_K_COUNT);
    }
}

// Captures kGraphBatch attempts once per problem on a library-owned stream
// (the caller's stream may be the null stream, which cannot be captured).
static void ensure_graph(pdcs_problem *P) {
    if (P->gexec) return;
    if (!P->gstream) PDCS_HIP(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
    if (!P->ev_in) PDCS_HIP(hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming));
    if (!P->ev_out) PDCS_HIP(hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming));
    hipGraph_t g = nullptr;
    PDCS_HIP(hipStreamBeginCapture(P->gstream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_attempts(P, kGraphBatch, P->gstream);
    } catch (...) {
        (void)hipStreamEndCapture(P->gstream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    PDCS_HIP(hipStreamEndCapture(P->gstream, &g));
    hipError_t e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    PDCS_HIP(e);
}

static void run_graph(pdcs_problem *P, hipStream_t s) {
    PDCS_HIP(hipEventRecord(P->ev_in, s));
    PDCS_HIP(hipStreamWaitEvent(P->gstream, P->ev_in, 0));
    PDCS_HIP(hipGraphLaunch(P->gexec, P->gstream));
    PDCS_HIP(hipEventRecord(P->ev_out, P->gstream));
    PDCS_HIP(hipStreamWaitEvent(s, P->ev_out, 0));
}

static void solve_impl(pdcs_problem *P, const pdcs_settings *S, const double *x0, const double *y0,
                       double omega0, double *xo, double *yo, pdcs_info *info, pdcs_trace *tr) {
    using clk = std::chrono::steady_clock;
    if (!S || !xo || !yo) fail(PDCS_ERR_INVALID_ARG, "settings, x_out and y_out are required");
    if (S->check_every < 1 || S->ruiz_iters < 0 || S->max_attempts < 1 || !(S->tol >= 0.0) ||
        S->step_mode < 0 || S->step_mode > 1 || (S->step_mode == 1 && !(S->step_fixed > 0.0)))
        fail(PDCS_ERR_INVALID_ARG, "bad settings");
    if (tr && (tr->cap < 0 || tr->n_snap < 0 || (tr->n_snap > 0 && (!tr->snap_iter || !tr->snap_x || !tr->snap_y)) ||
               (tr->cap > 0 && (!tr->attempts || !tr->eta_used || !tr->beta || !tr->omega ||
                                !tr->check_code || !tr->check_kkt))))
        fail(PDCS_ERR_INVALID_ARG, "bad trace");
    const auto t_start = clk::now();
    hipStream_t s = P->stream;
    const int64_t n = P->n, m = P->m;
    ensure_scaling(P, S->ruiz_iters, S->pock_chambolle ? 1 : 0);

    // trace buffers
    const int64_t cap = tr ? tr->cap : 0;
    DevMem tmem;
    int *log_att = tmem.alloc<int>(cap);
    double *log_eta = tmem.alloc<double>(cap), *log_beta = tmem.alloc<double>(cap),
           *log_om = tmem.alloc<double>(cap);
    if (tr) {
        tr->count = 0;
        for (int64_t i = 0; i < cap; ++i) tr->check_code[i] = 0, tr->check_kkt[i] = 0.0;
    }

    // no root guesses yet: every solve starts from the same state
    for (ConePlan *pl : {&P->planX, &P->planY}) {
        fill(pl->soc_root, pl->n_soc, NAN, s);
        fill(pl->exp_root, pl->n_exp, NAN, s);
    }

    // z^{0,0}: the mapped starting point projected onto X x Y (reading)
    if (x0) {
        h2d(P->tmp_n, x0, n, s);
        scale_in(P->tmp_n, P->f, P->x, n, s);
    } else {
        fill(P->x, n, 0.0, s);
    }
    if (y0) {
        h2d(P->tmp_m, y0, m, s);
        scale_in(P->tmp_m, P->e, P->y, m, s);
    } else {
        fill(P->y, m, 0.0, s);
    }
    pass_candidate(P->planX, false, CandArgs{P->x, P->ls, P->us, P->dx, P->st, 0, P->xa}, P->partX, s);
    pass_candidate(P->planY, true, CandArgs{P->y, P->ls, P->us, P->dy, P->st, 0, P->ya}, P->partY, s);
    spmv(P->Gs, P->pG, P->xa, P->gx0, nullptr, s);
    spmv(P->Gts, P->pGt, P->ya, P->aty0, nullptr, s);
    restart_copy(n, m, P->xa, P->ya, P->gx0, P->aty0, P->x, P->y, P->xa, P->ya, P->gx, P->aty,
                 P->gx0, P->aty0, P->xsum, P->ysum, s);
    long long spmv_count = 2;
    enqueue_kkt(P, P->xa, P->ya, P->gx0, P->aty0, P->xa, P->ya, P->e, P->f, 2);
    KktRaw raw[3];
    d2h(raw + 2, P->kraw + 2, 1, s);

    DevState hs{};
    hs.eta = P->gmax > 0.0 ? 1.0 / P->gmax : 1.0;
    if (S->step_mode == 1) hs.eta = fixed_step(P, S);
    hs.omega = (P->cs_norm > 1e-10 && P->hs_norm > 1e-10) ? P->cs_norm / P->hs_norm : 1.0;
    if (omega0 > 0.0) hs.omega = omega0;
    hs.tau = hs.eta / hs.omega, hs.sigma = hs.eta * hs.omega;
    hs.beta_prev = 1.0, hs.r_prev = INFINITY;
    hs.max_iter = S->max_iter, hs.check_every = S->check_every, hs.max_attempts = S->max_attempts;
    hs.beta_mode = S->beta_mode, hs.beta_const = S->beta_const, hs.beta_grow = S->beta_grow;
    hs.step_mode = S->step_mode;
    hs.beta_shrink = S->beta_shrink, hs.step_reduce_exp = S->step_reduce_exp;
    hs.step_grow_exp = S->step_grow_exp;
    hs.log_cap = cap, hs.log_attempts = log_att, hs.log_eta = log_eta, hs.log_beta = log_beta,
    hs.log_omega = log_om;
    hs.skip_update = 1, hs.status = -1;
    PDCS_HIP(hipStreamSynchronize(s));
    Kkt k_anchor = kkt_from_raw(P, raw[2]);
    int status = -1;
    Kkt kout = k_anchor;
    const double *outx = P->xa, *outy = P->ya;
    if (k_anchor.mx() <= S->tol) status = PDCS_SOLVE_OPTIMAL;
    if (!(k_anchor.mx() == k_anchor.mx())) status = PDCS_SOLVE_NUMERICAL;
    if (status < 0 && S->max_iter <= 0) status = PDCS_SOLVE_ITER_LIMIT;
    hs.halt = status >= 0 ? 1 : 0;
    h2d(P->st, &hs, 1, s);
    const auto t_iter = clk::now();
    const double setup_s = std::chrono::duration<double>(t_iter - t_start).count();

    double kprev_avg = INFINITY;
    long long restarts = 0;
    int64_t snap = 0;
    const bool stepwise = tr && (tr->cap > 0 || tr->n_snap > 0);
    long long prev_attempts = 0;
    constexpr int E = PDCS_K_COUNT + 1;
    double kms[PDCS_K_COUNT] = {};
    int64_t klaunch[PDCS_K_COUNT] = {};
    if (S->time_kernels && P->tev.empty()) {
        P->tev.resize(E * kGraphBatch, nullptr);
        for (hipEvent_t &e : P->tev) PDCS_HIP(hipEventCreate(&e));
    }
    while (status < 0) {
        // ---- step attempts until the device asks for a check ----
        while (!hs.halt) {
            const long long todo = S->check_every - hs.kin % S->check_every;
            const long long batch =
                stepwise ? 1 : std::max<long long>(1, std::min<long long>(todo, kGraphBatch));
            if (S->time_kernels) {
                enqueue_attempts(P, batch, s, P->tev.data());
            } else if (S->use_graph && batch == kGraphBatch) {
                ensure_graph(P);
                run_graph(P, s);
            } else {
                enqueue_attempts(P, batch, s);
            }
            const long long it_before = hs.n_iter;
            const long long att_before = hs.attempts_total + hs.attempts_cur;
            d2h(&hs, P->st, 1, s);
            PDCS_HIP(hipStreamSynchronize(s));
            if (S->time_kernels) {
                // attempts run in order and the device halts only at the end of a
                // batch, so the first `worked` attempts are the ones that did work
                const long long worked = hs.attempts_total + hs.attempts_cur - att_before;
                for (long long b = 0; b < worked && b < batch; ++b)
                    for (int j = 0; j < PDCS_K_COUNT; ++j) {
                        float ms = 0.0f;
                        PDCS_HIP(hipEventElapsedTime(&ms, P->tev[E * b + j], P->tev[E * b + j + 1]));
                        kms[j] += ms;
                    }
                const long long acc = hs.n_iter - it_before;
                klaunch[PDCS_K_PRIMAL] += worked, klaunch[PDCS_K_SPMV_G] += worked;
                klaunch[PDCS_K_DUAL] += worked, klaunch[PDCS_K_DECIDE] += worked;
                klaunch[PDCS_K_SPMV_GT] += acc, klaunch[PDCS_K_HALPERN] += acc;
            }
            spmv_count += (hs.attempts_total + hs.attempts_cur - prev_attempts) + (hs.n_iter - it_before);
            prev_attempts = hs.attempts_total + hs.attempts_cur;
            if (tr && snap < tr->n_snap && hs.n_iter > it_before && tr->snap_iter[snap] == hs.n_iter) {
                unscale(P->x, P->f, P->tmp_n, n, s);
                unscale(P->y, P->e, P->tmp_m, m, s);
                d2h(tr->snap_x + snap * n, P->tmp_n, n, s);
                d2h(tr->snap_y + snap * m, P->tmp_m, m, s);
                PDCS_HIP(hipStreamSynchronize(s));
                ++snap;
            }
        }
        if (hs.status == PDCS_SOLVE_NUMERICAL) {
            status = PDCS_SOLVE_NUMERICAL;
            break;
        }
        // ---- check: candidates P(z^{t,k}) and P(z_bar^{t,k}) ----
        pass_candidate(P->planX, false, CandArgs{P->x, P->ls, P->us, P->dx, P->st, 0, P->xc[0]}, P->partX, s);
        pass_candidate(P->planY, true, CandArgs{P->y, P->ls, P->us, P->dy, P->st, 0, P->yc[0]}, P->partY, s);
        pass_candidate(P->planX, false, CandArgs{P->xsum, P->ls, P->us, P->dx, P->st, 1, P->xc[1]}, P->partX, s);
        pass_candidate(P->planY, true, CandArgs{P->ysum, P->ls, P->us, P->dy, P->st, 1, P->yc[1]}, P->partY, s);
        for (int cnd = 0; cnd < 2; ++cnd) {
            spmv(P->Gs, P->pG, P->xc[cnd], P->gxc[cnd], nullptr, s);
            spmv(P->Gts, P->pGt, P->yc[cnd], P->atyc[cnd], nullptr, s);
            enqueue_kkt(P, P->xc[cnd], P->yc[cnd], P->gxc[cnd], P->atyc[cnd], P->xa, P->ya, P->e, P->f, cnd);
        }
        spmv_count += 4;
        d2h(raw, P->kraw, 2, s);
        PDCS_HIP(hipStreamSynchronize(s));
        const Kkt k1 = kkt_from_raw(P, raw[0]), k2 = kkt_from_raw(P, raw[1]);
        const int chosen = k2.avg() < k1.avg() ? 1 : 0;
        const Kkt kc = chosen ? k2 : k1;
        const double kcv = kc.avg(), kav = k_anchor.avg();
        int reason = 0, stop = 0;
        const double elapsed = std::chrono::duration<double>(clk::now() - t_iter).count();
        if (!(kcv == kcv)) {
            status = PDCS_SOLVE_NUMERICAL, stop = 1;
        } else if (kc.mx() <= S->tol) {
            status = PDCS_SOLVE_OPTIMAL, stop = 1;
        } else if (hs.n_iter >= S->max_iter) {
            status = PDCS_SOLVE_ITER_LIMIT, stop = 1;
        } else if (S->time_limit > 0.0 && elapsed >= S->time_limit) {
            status = PDCS_SOLVE_TIME_LIMIT, stop = 1;
        }
        if (!stop) {
            if (kcv <= S->restart_sufficient * kav)
                reason = 1;
            else if (kcv <= S->restart_necessary * kav && kcv > kprev_avg)
                reason = 2;
            else if ((double)hs.kin >= S->restart_artificial * (double)hs.n_iter)
                reason = 3;
        }
        const int64_t rec = hs.n_iter - 1;
        if (tr && rec >= 0 && rec < cap) {
            tr->check_code[rec] = 1 + chosen + 2 * reason + 8 * stop;
            tr->check_kkt[rec] = kcv;
        }
        if (stop) {
            outx = P->xc[chosen], outy = P->yc[chosen];
            kout = kc;
            break;
        }
        if (reason) {
            // PrimalWeightUpdate (reading: PDLP's smoothed log-ratio rule)
            const double ddx = std::sqrt(kc.dx2), ddy = std::sqrt(kc.dy2);
            if (ddx > 1e-10 && ddy > 1e-10)
                hs.omega = std::exp(0.5 * std::log(ddy / ddx) + 0.5 * std::log(hs.omega));
            restart_copy(n, m, P->xc[chosen], P->yc[chosen], P->gxc[chosen], P->atyc[chosen], P->x,
                         P->y, P->xa, P->ya, P->gx, P->aty, P->gx0, P->aty0, P->xsum, P->ysum, s);
            k_anchor = kc;
            kprev_avg = INFINITY;
            hs.kin = 0;
            hs.eta_sum = 0.0;
            hs.beta_prev = 1.0;
            hs.r_prev = INFINITY;
            hs.tau = hs.eta / hs.omega, hs.sigma = hs.eta * hs.omega;
            ++restarts;
        } else {
            kprev_avg = kcv;
        }
        hs.halt = 0;
        h2d(P->st, &hs, 1, s);
    }

    // ---- outputs (unscaled) ----
    if (S->out_on_device) {
        unscale(outx, P->f, xo, n, s);
        unscale(outy, P->e, yo, m, s);
    } else {
        unscale(outx, P->f, P->tmp_n, n, s);
        unscale(outy, P->e, P->tmp_m, m, s);
        d2h(xo, P->tmp_n, n, s);
        d2h(yo, P->tmp_m, m, s);
    }
    if (tr && cap > 0) {
        const int64_t cnt = std::min<int64_t>(cap, hs.n_iter);
        d2h(tr->attempts, log_att, cnt, s);
        d2h(tr->eta_used, log_eta, cnt, s);
        d2h(tr->beta, log_beta, cnt, s);
        d2h(tr->omega, log_om, cnt, s);
        tr->count = cnt;
    }
    PDCS_HIP(hipStreamSynchronize(s));
    const double solve_s = std::chrono::duration<double>(clk::now() - t_iter).count();
    fill_info(info, status, hs, restarts, spmv_count, kout, setup_s, solve_s);
    if (info)
        for (int j = 0; j < PDCS_K_COUNT; ++j) info->kernel_ms[j] = kms[j], info->kernel_launches[j] = klaunch[j];
}

// --------------------------------------------------------------------- ABI
template <class F>
static pdcs_status guarded(F &&f) {
    try {
        f();
        return PDCS_OK;
    } catch (const ApiError &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const HipError &e) {
        g_last_error = e.where;
        return e.code == hipErrorOutOfMemory ? PDCS_ERR_OOM : PDCS_ERR_HIP;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return PDCS_ERR_OOM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return PDCS_ERR_HIP;
    } catch (...) {
        g_last_error = "unknown error";
        return PDCS_ERR_HIP;
    }
}

extern "C" {

pdcs_status pdcs_settings_default(pdcs_settings *s) {
    if (!s) {
        g_last_error = "settings is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    std::memset(s, 0, sizeof *s);
    s->tol = 1e-6;
    s->max_iter = 1000000;
    s->time_limit = 0.0;
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
    s->out_on_device = 0;
    s->step_mode = 0;
    s->step_fixed = 0.9;
    s->power_iters = 100;
    s->use_graph = 1;
    s->time_kernels = 0;
    return PDCS_OK;
}

pdcs_status pdcs_problem_create(const pdcs_problem_desc *desc, void *hip_stream, pdcs_problem **out) {
    if (!out) {
        g_last_error = "out is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    return guarded([&] { *out = create_impl(desc, hip_stream, false); });
}

pdcs_status pdcs_problem_create_device(const pdcs_problem_desc *desc, void *hip_stream,
                                       pdcs_problem **out) {
    if (!out) {
        g_last_error = "out is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    return guarded([&] { *out = create_impl(desc, hip_stream, true); });
}

void pdcs_problem_destroy(pdcs_problem *p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    delete p;
}

pdcs_status pdcs_solve(pdcs_problem *p, const pdcs_settings *settings, const double *x0,
                       const double *y0, double omega0, double *x_out, double *y_out,
                       pdcs_info *info, pdcs_trace *trace) {
    return guarded([&] {
        if (!p) fail(PDCS_ERR_INVALID_ARG, "problem is NULL");
        solve_impl(p, settings, x0, y0, omega0, x_out, y_out, info, trace);
    });
}

pdcs_status pdcs_scaling(pdcs_problem *p, const pdcs_settings *settings, double *e_out,
                         double *f_out) {
    return guarded([&] {
        if (!p || !settings || !e_out || !f_out) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        ensure_scaling(p, settings->ruiz_iters, settings->pock_chambolle ? 1 : 0);
        d2h(e_out, p->e, p->m, p->stream);
        d2h(f_out, p->f, p->n, p->stream);
        PDCS_HIP(hipStreamSynchronize(p->stream));
    });
}

pdcs_status pdcs_spmv(pdcs_problem *p, int transpose, const double *x_dev, double *y_dev,
                      void *hip_stream) {
    return guarded([&] {
        if (!p || !x_dev || !y_dev) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        if (transpose)
            spmv(p->Gt, p->pGt, x_dev, y_dev, nullptr, s);
        else
            spmv(p->G, p->pG, x_dev, y_dev, nullptr, s);
    });
}

pdcs_status pdcs_kkt(pdcs_problem *p, const double *x_dev, const double *y_dev, double *out) {
    return guarded([&] {
        if (!p || !x_dev || !y_dev || !out) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        hipStream_t s = p->stream;
        spmv(p->G, p->pG, x_dev, p->gxc[0], nullptr, s);
        spmv(p->Gt, p->pGt, y_dev, p->atyc[0], nullptr, s);
        enqueue_kkt(p, x_dev, y_dev, p->gxc[0], p->atyc[0], x_dev, y_dev, p->ones_m, p->ones_n, 0);
        KktRaw r;
        d2h(&r, p->kraw, 1, s);
        PDCS_HIP(hipStreamSynchronize(s));
        const Kkt k = kkt_from_raw(p, r);
        out[0] = k.err_p, out[1] = k.err_d, out[2] = k.err_gap, out[3] = k.pobj, out[4] = k.dobj;
    });
}

pdcs_status pdcs_project(int64_t nblocks, const int32_t *types, const int64_t *dims, int dual,
                         const double *d_dev, double *v_dev, void *hip_stream) {
    return guarded([&] {
        if (nblocks < 0 || (nblocks > 0 && (!types || !dims || !v_dev)))
            fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        int64_t len = 0;
        for (int64_t b = 0; b < nblocks; ++b) len += dims[b];
        std::vector<int32_t> t;
        std::vector<int64_t> d;
        validate_cones(nblocks, types, dims, len, "cones", t, d);
        hipStream_t s = (hipStream_t)hip_stream;
        DevMem mem;
        ConePlan plan = upload_plan(mem, build_plan(0, 0, t, d), s);
        double *part = mem.alloc<double>(plan.ntiles * kPartials);
        pass_project(plan, dual != 0, ProjArgs{v_dev, d_dev}, part, s);
        PDCS_HIP(hipStreamSynchronize(s));
    });
}

const char *pdcs_status_string(pdcs_status s) {
    switch (s) {
    case PDCS_OK: return "ok";
    case PDCS_ERR_INVALID_ARG: return "invalid argument";
    case PDCS_ERR_DIMENSION: return "cone dimensions do not match";
    case PDCS_ERR_NONFINITE: return "non-finite data";
    case PDCS_ERR_OOM: return "out of memory";
    case PDCS_ERR_HIP: return "HIP runtime error";
    case PDCS_ERR_NOT_SUPPORTED: return "not supported";
    }
    return "unknown status";
}

const char *pdcs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
