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
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
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
    std::vector<int64_t> inst_tiles{0};   // tiles of instance b: [inst_tiles[b], inst_tiles[b+1])
    int64_t n_grid = 0;                    // grid-level SOC blocks
};

static int elem_kind(int32_t t) {
    return t == kZero ? kTileZero : t == kFree ? kTileFree : kTileNonneg;
}

// Appends the tiles of one instance: box entries [box0, box0 + n_box) and the
// cone blocks laid out from `base`.  Within an instance heavy classes come
// first so that they start early: large SOC (workgroup), small SOC
// (wavefront), exponential (thread), then elementwise runs.
static void append_plan(HostPlan &P, int32_t inst, int64_t box0, int64_t n_box, int64_t base,
                        const int32_t *types, const int64_t *dims, int64_t nblk) {
    std::vector<Tile> elem;
    auto tile = [&](int kind, int64_t count, int64_t start) {
        return Tile{kind, (int32_t)count, start, inst, 0};
    };
    auto push_run = [&](int kind, int64_t start, int64_t len) {
        for (int64_t o = 0; o < len; o += kElemPerTile)
            elem.push_back(tile(kind, std::min<int64_t>(kElemPerTile, len - o), start + o));
    };
    push_run(kTileBox, box0, n_box);
    // SOC size classes (dims up to 8, 16, 32, 64, 128, 256): lane groups of 8,
    // 16, 16, 16, 32 and 64 lanes with 1, 1, 2, 4, 4 and 4 entries per lane,
    // so a wavefront holds 8, 4, 4, 4, 2 and 1 blocks; then a workgroup per
    // block, then several workgroups per block (grid level)
    constexpr int kClasses = 8;
    const int class_kind[kClasses] = {kTileSoc8, kTileSoc16, kTileSoc32, kTileSoc64,
                                      kTileSoc128, kTileSoc256, kTileSocBlock, kTileSocGrid};
    const int class_per_tile[kClasses] = {32, 16, 16, 16, 8, 4, 1, 1};
    // The grid level pays for its barriers only while the large blocks alone
    // cannot fill the chip: with more than kSocGridMaxBlocks of them (one
    // workgroup each already covers every CU) they stay at the workgroup level.
    int64_t n_large = 0;
    for (int64_t b = 0; b < nblk; ++b) n_large += types[b] == kSoc && dims[b] >= kSocGridMin;
    const bool grid = n_large <= kSocGridMaxBlocks;
    auto soc_class = [grid](int64_t d) {
        return d <= 8 ? 0 : d <= 16 ? 1 : d <= 32 ? 2 : d <= 64 ? 3 : d <= 128 ? 4 : d <= 256 ? 5
               : (d < kSocGridMin || !grid) ? 6 : 7;
    };
    std::vector<std::pair<int64_t, int64_t>> soc[kClasses];
    std::vector<int64_t> ep, ed;
    int run_kind = -1;
    int64_t run_start = 0, run_len = 0, off = base;
    for (int64_t b = 0; b < nblk; ++b) {
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
    // largest classes first: they run longest.  A grid-level block becomes G
    // consecutive tiles, one per part, so its workgroups are dispatched together.
    for (int c = kClasses - 1; c >= 0; --c) {
        const int64_t first = (int64_t)P.soc_off.size();
        for (auto &p : soc[c]) P.soc_off.push_back(p.first), P.soc_dim.push_back((int32_t)p.second);
        const int64_t cnt = (int64_t)soc[c].size();
        if (class_kind[c] == kTileSocGrid) {
            // parts per block: one per kSocGridChunk entries, capped so that
            // all blocks together take about kSocGridTargetParts workgroups
            // (a block waits at each barrier for its slowest part, and parts
            // beyond what the chip keeps resident only queue behind it)
            const int64_t cap = std::max<int64_t>(
                kSocGridMinCap, std::min<int64_t>(kSocGridMaxParts, kSocGridTargetParts / std::max<int64_t>(cnt, 1)));
            for (int64_t i = 0; i < cnt; ++i) {
                const int64_t d = soc[c][i].second;
                const int G = (int)std::min<int64_t>(cap, (d + kSocGridChunk - 1) / kSocGridChunk);
                for (int p = 0; p < G; ++p)
                    P.tiles.push_back(Tile{kTileSocGrid, p + kSocGridPartCode * G, first + i, inst, (int32_t)P.n_grid});
                ++P.n_grid;
            }
            continue;
        }
        for (int64_t i = 0; i < cnt; i += class_per_tile[c])
            P.tiles.push_back(tile(class_kind[c], std::min<int64_t>(class_per_tile[c], cnt - i), first + i));
    }
    const int64_t e0 = (int64_t)P.exp_off.size();
    for (auto o : ep) P.exp_off.push_back(o);
    for (auto o : ed) P.exp_off.push_back(o);
    // a tile of 64 cones keeps one of its four wavefronts busy: with many
    // cones, wider tiles keep more root searches in flight per CU
    auto exp_per_tile = [](int64_t cnt) {
        for (int per : {4 * kExpPerTile, 2 * kExpPerTile})
            if (cnt >= (int64_t)per * kExpMinTiles) return (int64_t)per;
        return (int64_t)kExpPerTile;
    };
    const int64_t pe = exp_per_tile((int64_t)ep.size()), pd = exp_per_tile((int64_t)ed.size());
    for (int64_t i = 0; i < (int64_t)ep.size(); i += pe)
        P.tiles.push_back(tile(kTileExp, std::min<int64_t>(pe, ep.size() - i), e0 + i));
    for (int64_t i = 0; i < (int64_t)ed.size(); i += pd)
        P.tiles.push_back(tile(kTileExpDual, std::min<int64_t>(pd, ed.size() - i),
                               e0 + (int64_t)ep.size() + i));
    for (auto &t : elem) P.tiles.push_back(t);
    P.inst_tiles.push_back((int64_t)P.tiles.size());
}

static HostPlan build_plan(int64_t base, int64_t n_box, const std::vector<int32_t> &types,
                           const std::vector<int64_t> &dims) {
    HostPlan P;
    append_plan(P, 0, 0, n_box, base, types.data(), dims.data(), (int64_t)types.size());
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
    P.n_grid = H.n_grid;
    P.grid_ctr = mem.alloc<unsigned long long>(P.n_grid);
    P.grid_part = mem.alloc<double>(P.n_grid * 2 * kSocGridMaxParts * kSocGridSlot);
    P.grid_err = mem.alloc<int>(1);
    PDCS_HIP(hipMemsetAsync(P.grid_ctr, 0, sizeof(unsigned long long) * (size_t)std::max<int64_t>(P.n_grid, 1), s));
    PDCS_HIP(hipMemsetAsync(P.grid_err, 0, sizeof(int), s));
    if (H.inst_tiles.size() > 2) {   // a batch: per-instance tile ranges
        P.inst_tiles = mem.alloc<int64_t>((int64_t)H.inst_tiles.size());
        h2d(P.inst_tiles, H.inst_tiles.data(), (int64_t)H.inst_tiles.size(), s);
    }
    PDCS_HIP(hipStreamSynchronize(s));  // the host vectors die with the caller's frame
    return P;
}

// A barrier of a grid-level SOC block that timed out leaves the plan's flag
// set (the projections of that launch are then not valid): report it.
static void check_grid(const ConePlan &pl, hipStream_t s) {
    if (pl.n_grid == 0) return;
    int e = 0;
    d2h(&e, pl.grid_err, 1, s);
    PDCS_HIP(hipStreamSynchronize(s));
    if (e) fail(PDCS_ERR_HIP, "a grid-level SOC projection timed out waiting for its workgroups");
}

// Product layouts by code: 0 = default, -1 = CSR-stream, L > 0 = row-split
// with L lanes per row, slab_code(S) = column slabs (S in 1, 2, 4, 8).
static int slab_code(int S) { return -10 - S; }
static int slabs_of(int code) { return code <= -10 ? -10 - code : 0; }

// Host copies of the structure a column-slab plan is cut from: the column
// indices and, per column, the running count of entries (the row pointers of
// the transpose).
struct SlabSource {
    const std::vector<int32_t> *ci = nullptr;
    const std::vector<int64_t> *col_cum = nullptr;
};

// Column slabs: slab k takes the columns [cb[k], cb[k+1]) that hold about
// nnz k/S .. nnz (k+1)/S entries (after a hot slab of the first columns, when
// there is one).  Each slab's arrays hold first the entries
// of its short rows (in row order, CSR order within a row), cut into streamed
// blocks of at most kStreamNnz entries and kStreamRows rows, then the slab's
// entries of the long rows (rows of more than long_thr entries), row after
// row, cut into chunks of at most kLongChunk entries.  A long row's chunks are
// listed slab by slab, and its sum adds them in that order.  Block i of the
// launch runs on XCD i mod kXcds; XCDs k g .. k g + g - 1 (g = kXcds / S)
// take the blocks of slab k (its chunks first: they are the longest), padded
// with empty blocks so that every slab keeps its XCDs.
static void add_slabs(DevMem &mem, SpmvPlan &P, const std::vector<int64_t> &rp,
                      const SlabSource &src, int S, hipStream_t s) {
    if (!src.ci || !src.col_cum) fail(PDCS_ERR_NOT_SUPPORTED, "column-slab plan without its structure");
    if (S != 1 && S != 2 && S != 4 && S != 8) fail(PDCS_ERR_NOT_SUPPORTED, "slab count must divide 8");
    const std::vector<int32_t> &ci = *src.ci;
    const std::vector<int64_t> &cc = *src.col_cum;
    const int64_t rows = (int64_t)rp.size() - 1, nnz = rp.back(), cols = (int64_t)cc.size() - 1;
    if (rows >= INT32_MAX || nnz >= INT32_MAX)
        fail(PDCS_ERR_NOT_SUPPORTED, "column-slab plan limited to 2^31 rows and entries");
    // The hot slab: the first min(cols, kHotCols) columns, when they hold at
    // least 1/(2 S) of the entries.  Their gathers then come from LDS, and its
    // blocks spread over every XCD; the S cold slabs share the remaining
    // entries equally.
    const int64_t H = S >= 2 ? std::min<int64_t>(cols, kHotCols) : 0;
    const int hot = H > 0 && 2 * S * cc[H] >= nnz ? 1 : 0;
    const int S_cold = S;
    S = S_cold + hot;
    std::vector<int64_t> cb(S + 1, 0);
    cb[S] = cols;
    if (hot) cb[1] = H;
    const int64_t e0 = hot ? cc[H] : 0;
    for (int k = 1; k < S_cold; ++k) {
        const int64_t t = e0 + (nnz - e0) * k / S_cold;
        int64_t c = std::lower_bound(cc.begin(), cc.end(), t) - cc.begin();
        cb[hot + k] = std::min(cols, std::max(cb[hot + k - 1], c));
    }
    std::vector<int8_t> slab_of(cols);
    for (int k = 0; k < S; ++k)
        for (int64_t j = cb[k]; j < cb[k + 1]; ++j) slab_of[j] = (int8_t)k;
    const int64_t R1 = rows + 1;
    auto is_long = [&](int64_t r) { return rp[r + 1] - rp[r] > P.long_thr; };
    std::vector<int32_t> lr;   // long rows
    for (int64_t r = 0; r < rows; ++r)
        if (is_long(r)) lr.push_back((int32_t)r);
    const int64_t NL = (int64_t)lr.size();
    // entries per (slab, short row) and per (slab, long row)
    std::vector<int32_t> lrp((size_t)(S * R1), 0);
    std::vector<int64_t> lcnt((size_t)(S * NL), 0);
    for (int64_t r = 0, l = 0; r < rows; ++r) {
        const bool lg = l < NL && lr[l] == r;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int k = slab_of[ci[e]];
            if (lg)
                ++lcnt[k * NL + l];
            else
                ++lrp[k * R1 + r + 1];
        }
        if (lg) ++l;
    }
    P.n_slabs = S;
    P.hot_cols = hot ? (int)H : 0;
    P.slab_base[0] = 0;
    std::vector<int64_t> long0(S);   // start of slab k's long-row region
    for (int k = 0; k < S; ++k) {
        int32_t *l = lrp.data() + k * R1;
        for (int64_t r = 0; r < rows; ++r) l[r + 1] += l[r];
        int64_t nlong = 0;
        for (int64_t q = 0; q < NL; ++q) nlong += lcnt[k * NL + q];
        long0[k] = P.slab_base[k] + l[rows];
        P.slab_base[k + 1] = long0[k] + nlong;
    }
    for (int k = S + 1; k <= kMaxSlabs + 1; ++k) P.slab_base[k] = P.slab_base[S];
    const int64_t total = P.slab_base[S];
    // place the entries
    std::vector<int32_t> sci(total), sperm(total), cur(lrp);
    std::vector<int64_t> lpos(S * NL);   // next position of (slab, long row)
    for (int k = 0; k < S; ++k) {
        int64_t o = long0[k];
        for (int64_t q = 0; q < NL; ++q) lpos[k * NL + q] = o, o += lcnt[k * NL + q];
    }
    std::vector<int64_t> lstart(lpos);
    for (int64_t r = 0, l = 0; r < rows; ++r) {
        const bool lg = l < NL && lr[l] == r;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int k = slab_of[ci[e]];
            const int64_t q = lg ? lpos[k * NL + l]++ : P.slab_base[k] + cur[k * R1 + r]++;
            sci[q] = ci[e], sperm[q] = (int32_t)e;
        }
        if (lg) ++l;
    }
    for (int k = 0; k < S; ++k)   // row pointers into the concatenated slab arrays
        for (int64_t r = 0; r <= rows; ++r) lrp[k * R1 + r] += (int32_t)P.slab_base[k];
    // chunks of the long rows, row by row, slab by slab
    std::vector<std::vector<SlabBlock>> lists(S);
    std::vector<int32_t> crow;
    std::vector<int64_t> cptr{0};
    for (int64_t q = 0; q < NL; ++q) {
        for (int k = 0; k < S; ++k) {
            const int64_t a = lstart[k * NL + q], n = lcnt[k * NL + q];
            for (int64_t o = 0; o < n; o += kLongChunk) {
                const int64_t c = (int64_t)crow.size();
                const int64_t cnt = std::min<int64_t>(kLongChunk, n - o);
                lists[k].push_back({(int32_t)(-1 - c), 0, (int32_t)(a + o), (int32_t)cnt | (k << 16)});
                crow.push_back((int32_t)q);
            }
        }
        cptr.push_back((int64_t)crow.size());
    }
    // streamed blocks of the short rows
    for (int k = 0; k < S; ++k) {
        const int32_t *l = lrp.data() + k * R1;
        auto close = [&](int64_t a, int64_t b) {
            lists[k].push_back({(int32_t)a, (int32_t)b, l[a], (l[b] - l[a]) | (k << 16)});
        };
        int64_t start = 0, acc = 0;
        for (int64_t r = 0; r < rows; ++r) {
            const int64_t len = l[r + 1] - l[r];
            if (acc + len > kStreamNnz || r - start >= kStreamRows) {
                close(start, r);
                start = r, acc = 0;
            }
            acc += len;
        }
        if (rows > start) close(start, rows);
    }
    // per XCD: the blocks of its cold slab (every g-th of them), then its
    // share of the hot slab's blocks (every kXcds-th)
    const int g = kXcds / S_cold;
    std::vector<std::vector<SlabBlock>> per(kXcds);
    for (int k = 0; k < S_cold; ++k)
        for (size_t j = 0; j < lists[hot + k].size(); ++j) per[k * g + j % g].push_back(lists[hot + k][j]);
    if (hot)
        for (size_t j = 0; j < lists[0].size(); ++j) per[j % kXcds].push_back(lists[0][j]);
    size_t rounds = 0;
    for (int x = 0; x < kXcds; ++x) rounds = std::max(rounds, per[x].size());
    std::vector<SlabBlock> blk(rounds * kXcds, SlabBlock{0, 0, 0, 0});
    for (int x = 0; x < kXcds; ++x)
        for (size_t j = 0; j < per[x].size(); ++j) blk[j * kXcds + x] = per[x][j];
    P.n_slab_blocks = (int64_t)blk.size();
    P.slab_rp = mem.alloc<int32_t>(S * R1);
    P.slab_ci = mem.alloc<int32_t>(total);
    P.slab_perm = mem.alloc<int32_t>(total);
    P.slab_blk = mem.alloc<SlabBlock>(P.n_slab_blocks);
    P.slab_part = mem.alloc<double>(S * rows);
    h2d(P.slab_rp, lrp.data(), S * R1, s);
    h2d(P.slab_ci, sci.data(), total, s);
    h2d(P.slab_perm, sperm.data(), total, s);
    h2d(P.slab_blk, blk.data(), P.n_slab_blocks, s);
    // the long rows as the finishing steps see them (chunk sums in list order)
    P.n_long = NL;
    P.n_chunks = (int64_t)crow.size();
    P.long_rows = mem.alloc<int32_t>(NL);
    P.long_chunk_ptr = mem.alloc<int64_t>(NL + 1);
    P.chunk_row = mem.alloc<int32_t>(P.n_chunks);
    P.chunk_part = mem.alloc<double>(P.n_chunks);
    h2d(P.long_rows, lr.data(), NL, s);
    h2d(P.long_chunk_ptr, cptr.data(), NL + 1, s);
    h2d(P.chunk_row, crow.data(), P.n_chunks, s);
    if (NL > 0) {
        std::vector<int32_t> lof(rows, -1);
        for (int64_t q = 0; q < NL; ++q) lof[lr[q]] = (int32_t)q;
        P.long_of = mem.alloc<int32_t>(rows);
        h2d(P.long_of, lof.data(), rows, s);
    }
    PDCS_HIP(hipStreamSynchronize(s));
}

// Launch plan of one product (layout codes above).  Default: CSR-stream when
// rows average fewer than 12 entries, else `choose_lanes` lanes per row.  Rows
// longer than max(64, 32 L) entries (L = choose_lanes or the forced lanes,
// at most kStreamNnz in the streamed layouts) are long.
static SpmvPlan build_spmv_plan(DevMem &mem, const std::vector<int64_t> &rp, hipStream_t s,
                                int force = 0, const SlabSource &src = SlabSource{}) {
    SpmvPlan P;
    const int64_t rows = (int64_t)rp.size() - 1;
    const int64_t nnz = rp.back();
    const double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
    const int slabs = slabs_of(force);
    P.lanes = force > 0 ? force : choose_lanes(rows > 0 ? avg : 1.0);
    P.long_thr = std::max<int64_t>(64, 32 * P.lanes);
    P.stream = force == -1 ? 1 : force != 0 ? 0 : (avg < 12.0 ? 1 : 0);
    // rows one thread adds up in a streamed block stay short: longer rows go
    // to the chunks
    if (P.stream || slabs) P.long_thr = std::min<int64_t>(P.long_thr, kStreamNnz);
    if (slabs) {   // its long rows are chunked inside the slabs
        add_slabs(mem, P, rp, src, slabs, s);
        return P;
    }
    // rows longer than long_thr: chunks of kLongChunk entries
    std::vector<int32_t> lr, crow;
    std::vector<int64_t> cptr{0}, cbeg, cend;
    for (int64_t i = 0; i < rows; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        if (len <= P.long_thr) continue;
        const int32_t li = (int32_t)lr.size();
        lr.push_back((int32_t)i);
        for (int64_t b = rp[i]; b < rp[i + 1]; b += kLongChunk)
            crow.push_back(li), cbeg.push_back(b), cend.push_back(std::min(b + kLongChunk, rp[i + 1]));
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
            if (acc + len > kStreamNnz || i - start >= kStreamRows) {
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
    P.chunk_end = mem.alloc<int64_t>(P.n_chunks);
    P.chunk_part = mem.alloc<double>(P.n_chunks);
    P.sblock = mem.alloc<int64_t>((int64_t)sb.size());
    if (P.n_long > 0) {
        std::vector<int32_t> lof(rows, -1);
        for (int64_t l = 0; l < P.n_long; ++l) lof[lr[l]] = (int32_t)l;
        P.long_of = mem.alloc<int32_t>(rows);
        h2d(P.long_of, lof.data(), rows, s);
    }
    h2d(P.long_rows, lr.data(), P.n_long, s);
    h2d(P.long_chunk_ptr, cptr.data(), P.n_long + 1, s);
    h2d(P.chunk_row, crow.data(), P.n_chunks, s);
    h2d(P.chunk_begin, cbeg.data(), P.n_chunks, s);
    h2d(P.chunk_end, cend.data(), P.n_chunks, s);
    h2d(P.sblock, sb.data(), (int64_t)sb.size(), s);
    PDCS_HIP(hipStreamSynchronize(s));
    return P;
}

}  // namespace pdcs

using namespace pdcs;

// ------------------------------------------------------------------ problem
// Sizes and offsets of one instance inside the (block-diagonal) layout.
struct InstDims {
    int64_t x0 = 0, n = 0, y0 = 0, m = 0, nb = 0, k0 = 0, nnz = 0;
    int64_t nb_in = 0;   // entries of the internal box run (box, zero, free, nonnegative)
};

struct pdcs_problem {
    int64_t n = 0, m = 0, nnz = 0;     // totals over the instances
    int64_t B = 1;                     // instances (1: a single problem)
    std::vector<InstDims> inst;
    hipStream_t stream = nullptr;
    DevMem mem;
    std::vector<int32_t> xt, rt;       // cone lists of all instances, in order
    std::vector<int64_t> xd, rd;
    std::vector<int64_t> xblk, rblk;   // [B+1]: cone blocks of instance b (the caller's order)
    // Internal order of x (column popularity): xperm[p] = the caller's index of
    // internal entry p, xpos its inverse; the x-cone lists in internal order.
    int32_t *xperm = nullptr, *xpos = nullptr;
    std::vector<int32_t> ixt;
    std::vector<int64_t> ixd, ixblk;
    Csr G, Gt;                         // unscaled
    Csr Gs, Gts;                       // scaled values, shared structure
    SpmvPlan pG, pGt;
    std::unique_ptr<DevMem> planmem[2];   // arrays of pG, pGt (replaced with the plan)
    int tuned = 0;                     // 1 once the plans are chosen (autotuner or caller)
    ConePlan planX, planY;
    // l, u: length n, -inf/+inf outside the box entries of each instance
    double *c, *h, *l, *u, *ones_n, *ones_m;
    double *e, *f, *cs, *hs, *ls, *us, *dx, *dy;
    double *x, *y, *xa, *ya, *xh, *yh, *aty, *gx, *aty0, *gx0, *atyh, *gxh, *xsum, *ysum;
    double *xc[2], *yc[2], *gxc[2], *atyc[2], *tmp_n, *tmp_m;
    double *partX, *partY, *scal;
    KktRaw *kraw;                      // [3 B]: slot k of instance b at k B + b
    DevState *st;                      // [B]
    int *flag;
    // batch maps (null for a single problem)
    int32_t *x_inst = nullptr, *y_inst = nullptr;
    int64_t *x_off = nullptr, *y_off = nullptr, *k_off = nullptr;   // [B+1]
    int32_t *rcode = nullptr;          // [B] restart codes of a check
    double *seg = nullptr;             // [5 B] per-instance reductions
    // host copy of a batch's concatenated data, for handing an instance to a
    // problem of its own (empty for a single problem)
    std::vector<int64_t> h_rp;
    std::vector<int32_t> h_ci;
    std::vector<double> h_val, h_c, h_h, h_l, h_u;
    std::vector<double> cinf, hinf, gmax, cs_norm, hs_norm;
    int scaled_ruiz = -1, scaled_pc = -1;
    // a captured batch of step attempts, replayed on a library stream
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};   // [precision mode]
    // timing events of settings.time_kernels: (PDCS_K_COUNT + 1) per attempt
    std::vector<hipEvent_t> tev;
    // mixed-precision form: FP32 copies of the scaled values (Gs.v32, Gts.v32)
    // and of the products' inputs x^, y^, allocated on first use
    float *xh32 = nullptr, *yh32 = nullptr;
    float *x32 = nullptr;   // input of pdcs_spmv32
    // rotated SOC blocks of the caller's problem (mapped to SOC at creation):
    // the caller's index of each block's first entry, in x and in the rows,
    // [B+1] bounds per instance, device copies and an (n + m) work buffer
    std::vector<int64_t> rx, ry, rx_b, ry_b;
    int64_t *rx_dev = nullptr, *ry_dev = nullptr;
    double *rtmp = nullptr;
    int64_t snaps_written = 0;         // snapshots of the last solve's trace
    ~pdcs_problem() {
        for (hipEvent_t e : tev) (void)hipEventDestroy(e);
        for (hipGraphExec_t g : gexec)
            if (g) (void)hipGraphExecDestroy(g);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (gstream) (void)hipStreamDestroy(gstream);
    }
};

struct pdcs_batch {
    pdcs_problem *p;
};

// The warm-start network: FP32 master parameters in one flat array laid out
// [W1 (hid x in), b1, W2 (hid x hid), b2, W3 (out x hid), b3] (weights row-major
// by output), their gradient and Adam moments, a BF16 copy for the GEMMs, and
// the activations of one batch.
struct pdcs_mlp {
    int64_t in = 0, hid = 0, out = 0, cap = 0, np = 0, step = 0;
    int64_t off[6] = {};
    hipStream_t stream = nullptr;
    DevMem mem;
    float *p, *g, *m1, *m2;
    uint16_t *p16;
    uint16_t *xb, *h1b, *h2b, *d16;
    float *h1, *h2, *o, *d32, *dh;
    double *part;
    // transposed operands of the backward GEMMs (all read along k) and the
    // padded leading dimension of the output gradient (a multiple of 8)
    uint16_t *ta, *tb, *wt;
    int64_t ldo = 0;
    // split-K partial products of dH2 = dO W3 (M = batch, K = the outputs)
    float *ws = nullptr;
    int64_t ws_elems = 0;
};

constexpr int kGraphBatch = 64;   // step attempts per captured graph
// the least a step attempt of one instance costs on its own (five launches)
constexpr double kAloneAttemptS = 25e-6;

static void validate_cones(int64_t nblk, const int32_t *t, const int64_t *d, int64_t expect,
                           const char *what, std::vector<int32_t> &ot, std::vector<int64_t> &od) {
    if (nblk < 0 || (nblk > 0 && (!t || !d))) fail(PDCS_ERR_INVALID_ARG, std::string(what) + ": bad cone list");
    int64_t sum = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        if (t[b] < kZero || t[b] > kRsoc) fail(PDCS_ERR_INVALID_ARG, std::string(what) + ": unknown cone type");
        if (d[b] < 1) fail(PDCS_ERR_DIMENSION, std::string(what) + ": cone of dimension < 1");
        if (t[b] == kRsoc && d[b] < 2) fail(PDCS_ERR_DIMENSION, std::string(what) + ": rotated SOC of dimension < 2");
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

static void check_desc(const pdcs_problem_desc *D) {
    if (!D) fail(PDCS_ERR_INVALID_ARG, "desc is NULL");
    if (D->n < 1 || D->m < 0 || D->nnz < 0 || D->n_box < 0 || D->n_box > D->n)
        fail(PDCS_ERR_INVALID_ARG, "bad sizes");
    if (!D->row_ptr || (D->nnz > 0 && (!D->col || !D->val)) || !D->c || (D->m > 0 && !D->h) ||
        (D->n_box > 0 && (!D->l || !D->u)))
        fail(PDCS_ERR_INVALID_ARG, "NULL array");
}

// Values of each matrix in the slab order of the plan it is used with (G and
// G~ with pG, G^T and G~^T with pGt); plans without slabs need none.  Called
// whenever a plan or the values change.
static void sync_slab_values(pdcs_problem *P) {
    hipStream_t s = P->stream;
    auto one = [&](Csr &A, const SpmvPlan &pl) {
        if (pl.n_slabs == 0 || !A.v) return;
        if (!A.sv) A.sv = P->mem.alloc<double>(A.nnz);
        if (A.v32 && !A.sv32) A.sv32 = P->mem.alloc<float>(A.nnz);
        slab_values(A, pl, s);
    };
    one(P->G, P->pG);
    one(P->Gs, P->pG);
    one(P->Gt, P->pGt);
    one(P->Gts, P->pGt);
}

static void set_plan(pdcs_problem *P, int side, int code);

// ------------------------------------------------------------ rotated SOC
// A rotated SOC block (2 u v >= ||w||^2, u, v >= 0) is an SOC block under the
// orthogonal, self-inverse map T(u, v, w) = ((u + v)/sqrt 2, (u - v)/sqrt 2, w):
//   row block: (G x - h) in RSOC  <=>  T (G x - h) in SOC, so the block's first
//              two rows of G and entries of h become their sum and difference
//              over sqrt 2, and the caller's dual variable is y = T y';
//   x block:   x in RSOC  <=>  x = T x' with x' in SOC, so the block's first
//              two columns of G and entries of c are combined the same way.
// The objective is unchanged; starting points and solutions are mapped by T.
struct RsocMap {
    std::vector<pdcs_problem_desc> d;
    std::vector<std::vector<int64_t>> rp, xd, rd;
    std::vector<std::vector<int32_t>> ci, xt, rt;
    std::vector<std::vector<double>> val, c, h;
    // caller's index of the first entry of each rotated block, over the whole
    // batch (instance b's x block at x0_b + offset), and [B+1] bounds per instance
    std::vector<int64_t> xpair, ypair, xpair_b, ypair_b;
};

static bool has_rsoc(int64_t nblk, const int32_t *t) {
    for (int64_t b = 0; t && b < nblk; ++b)
        if (t[b] == kRsoc) return true;
    return false;
}

// Host CSR checks needed before the arrays are read on the host.
static void check_csr_host(const pdcs_problem_desc *D) {
    if (D->row_ptr[0] != 0 || D->row_ptr[D->m] != D->nnz)
        fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
    for (int64_t r = 0; r < D->m; ++r)
        if (D->row_ptr[r] > D->row_ptr[r + 1]) fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
    for (int64_t k = 0; k < D->nnz; ++k)
        if (D->col[k] < 0 || D->col[k] >= D->n) fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
}

// Fills R with the descriptors of Ds[0, count) with every rotated block
// mapped to SOC; false (R untouched) when there is none.
static bool map_rsoc(const pdcs_problem_desc *Ds, int64_t count, RsocMap &R) {
    bool any = false;
    for (int64_t b = 0; b < count; ++b) {
        check_desc(Ds + b);
        any = any || has_rsoc(Ds[b].n_xcones, Ds[b].xcone_type) || has_rsoc(Ds[b].n_rcones, Ds[b].rcone_type);
    }
    if (!any) return false;
    const double r2 = 1.0 / std::sqrt(2.0);
    R.d.assign(Ds, Ds + count);
    R.rp.resize(count), R.xd.resize(count), R.rd.resize(count), R.ci.resize(count);
    R.xt.resize(count), R.rt.resize(count), R.val.resize(count), R.c.resize(count), R.h.resize(count);
    R.xpair_b.assign(1, 0), R.ypair_b.assign(1, 0);
    int64_t x0 = 0, y0 = 0;
    for (int64_t b = 0; b < count; ++b) {
        const pdcs_problem_desc &D = Ds[b];
        std::vector<int32_t> vt;
        std::vector<int64_t> vd;
        validate_cones(D.n_xcones, D.xcone_type, D.xcone_dim, D.n - D.n_box, "x cones", vt, vd);
        validate_cones(D.n_rcones, D.rcone_type, D.rcone_dim, D.m, "row cones", vt, vd);
        check_csr_host(&D);
        // pair[j] = 0: column j untouched, 1: first, 2: second entry of a rotated x block
        std::vector<int8_t> xpair(D.n, 0);
        std::vector<int64_t> rows_first;   // first rows of the rotated row blocks
        R.c[b].assign(D.c, D.c + D.n);
        R.h[b].assign(D.h, D.h + D.m);
        R.xt[b].assign(D.xcone_type, D.xcone_type + D.n_xcones);
        R.xd[b].assign(D.xcone_dim, D.xcone_dim + D.n_xcones);
        R.rt[b].assign(D.rcone_type, D.rcone_type + D.n_rcones);
        R.rd[b].assign(D.rcone_dim, D.rcone_dim + D.n_rcones);
        for (int64_t k = 0, o = D.n_box; k < D.n_xcones; o += D.xcone_dim[k], ++k) {
            if (D.xcone_type[k] != kRsoc) continue;
            R.xt[b][k] = kSoc;
            xpair[o] = 1, xpair[o + 1] = 2;
            R.xpair.push_back(x0 + o);
            const double a = D.c[o], e = D.c[o + 1];
            R.c[b][o] = (a + e) * r2, R.c[b][o + 1] = (a - e) * r2;
        }
        for (int64_t k = 0, o = 0; k < D.n_rcones; o += D.rcone_dim[k], ++k) {
            if (D.rcone_type[k] != kRsoc) continue;
            R.rt[b][k] = kSoc;
            rows_first.push_back(o);
            R.ypair.push_back(y0 + o);
            const double a = D.h[o], e = D.h[o + 1];
            R.h[b][o] = (a + e) * r2, R.h[b][o + 1] = (a - e) * r2;
        }
        // Merges entries (key, side, value) by key and appends the sums and
        // differences over sqrt 2 of sides 0 and 1 (exact zeros dropped).
        struct Ent { int32_t key; int side; double v; };
        auto merge = [&](std::vector<Ent> &ents, std::vector<std::pair<int32_t, double>> &o0,
                         std::vector<std::pair<int32_t, double>> &o1, int32_t key1_shift) {
            std::stable_sort(ents.begin(), ents.end(), [](const Ent &p, const Ent &q) { return p.key < q.key; });
            for (size_t i = 0; i < ents.size();) {
                double s0 = 0.0, s1 = 0.0;
                size_t j = i;
                for (; j < ents.size() && ents[j].key == ents[i].key; ++j) (ents[j].side ? s1 : s0) += ents[j].v;
                const double p = (s0 + s1) * r2, q = (s0 - s1) * r2;
                if (p != 0.0) o0.push_back({ents[i].key, p});
                if (q != 0.0) o1.push_back({ents[i].key + key1_shift, q});
                i = j;
            }
        };
        // columns: in each row, the entries of a rotated pair of columns
        std::vector<std::vector<std::pair<int32_t, double>>> rows(D.m);
        std::vector<Ent> ents;
        for (int64_t r = 0; r < D.m; ++r) {
            auto &out = rows[r];
            ents.clear();
            for (int64_t k = D.row_ptr[r]; k < D.row_ptr[r + 1]; ++k) {
                const int32_t j = D.col[k];
                if (!xpair[j]) out.push_back({j, D.val[k]});
                else ents.push_back({xpair[j] == 1 ? j : j - 1, xpair[j] - 1, D.val[k]});
            }
            merge(ents, out, out, 1);
        }
        // rows: the first two rows of each rotated row block, merged by column
        for (int64_t o : rows_first) {
            ents.clear();
            for (int w = 0; w < 2; ++w)
                for (const auto &e : rows[o + w]) ents.push_back({e.first, w, e.second});
            rows[o].clear(), rows[o + 1].clear();
            merge(ents, rows[o], rows[o + 1], 0);
        }
        auto &rp = R.rp[b];
        rp.assign(D.m + 1, 0);
        for (int64_t r = 0; r < D.m; ++r) rp[r + 1] = rp[r] + (int64_t)rows[r].size();
        R.ci[b].reserve(rp[D.m]), R.val[b].reserve(rp[D.m]);
        for (const auto &row : rows)
            for (const auto &e : row) R.ci[b].push_back(e.first), R.val[b].push_back(e.second);
        pdcs_problem_desc &M = R.d[b];
        M.nnz = rp[D.m];
        M.row_ptr = rp.data(), M.col = R.ci[b].data(), M.val = R.val[b].data();
        M.c = R.c[b].data(), M.h = R.h[b].data();
        M.xcone_type = R.xt[b].data(), M.xcone_dim = R.xd[b].data();
        M.rcone_type = R.rt[b].data(), M.rcone_dim = R.rd[b].data();
        R.xpair_b.push_back((int64_t)R.xpair.size()), R.ypair_b.push_back((int64_t)R.ypair.size());
        x0 += D.n, y0 += D.m;
    }
    return true;
}

static void rotate_host(double *v, const int64_t *offs, int64_t count, int64_t base) {
    const double r2 = 1.0 / std::sqrt(2.0);
    for (int64_t t = 0; t < count; ++t) {
        double *p = v + (offs[t] - base);
        const double a = p[0], e = p[1];
        p[0] = (a + e) * r2, p[1] = (a - e) * r2;
    }
}

// A problem, or a batch of `count` independent problems laid out block-
// diagonally: instance b owns entries [x0, x0 + n) of x, rows [y0, y0 + m) and
// nonzeros [k0, k0 + nnz); its columns are shifted by x0.  A batch needs host
// arrays; one problem may also come from device arrays.
// G^T of a problem or batch, instance by instance (the transpose of a
// block-diagonal matrix is block-diagonal).
static void transpose_blocks(pdcs_problem *P, hipStream_t s) {
    std::vector<TBlock> blk;
    for (const InstDims &I : P->inst) blk.push_back(TBlock{I.y0, I.m, I.x0, I.n, I.k0, I.nnz});
    transpose_csr(P->G, P->Gt, blk.data(), (int64_t)blk.size(), s);
}

// Stage lines of problem and batch creation on stderr when the environment
// sets PDCS_LOG (setting up a batch of billions of entries takes minutes).
static void create_log(const char *stage, std::chrono::steady_clock::time_point t0) {
    static const bool on = std::getenv("PDCS_LOG") != nullptr;
    if (!on) return;
    std::fprintf(stderr, "pdcs: create: %s at %.1f s\n", stage,
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    std::fflush(stderr);
}

static pdcs_problem *create_impl(const pdcs_problem_desc *Ds, int64_t count, void *stream,
                                 bool on_device) {
    const auto t_create = std::chrono::steady_clock::now();
    if (!Ds) fail(PDCS_ERR_INVALID_ARG, "desc is NULL");
    if (count < 1) fail(PDCS_ERR_INVALID_ARG, "no problem in the batch");
    if (on_device && count != 1) fail(PDCS_ERR_NOT_SUPPORTED, "a batch takes host arrays");
    RsocMap R;
    if (on_device) {
        check_desc(Ds);
        if (has_rsoc(Ds->n_xcones, Ds->xcone_type) || has_rsoc(Ds->n_rcones, Ds->rcone_type))
            fail(PDCS_ERR_NOT_SUPPORTED, "rotated SOC blocks need host arrays");
    } else if (map_rsoc(Ds, count, R)) {
        Ds = R.d.data();
    }
    auto P = std::make_unique<pdcs_problem>();
    P->B = count;
    P->stream = (hipStream_t)stream;
    P->xblk.push_back(0), P->rblk.push_back(0);
    int64_t n = 0, m = 0, nnz = 0;
    for (int64_t b = 0; b < count; ++b) {
        const pdcs_problem_desc *D = Ds + b;
        check_desc(D);
        InstDims I;
        I.x0 = n, I.n = D->n, I.y0 = m, I.m = D->m, I.nb = D->n_box, I.k0 = nnz, I.nnz = D->nnz;
        validate_cones(D->n_xcones, D->xcone_type, D->xcone_dim, D->n - D->n_box, "x cones", P->xt, P->xd);
        validate_cones(D->n_rcones, D->rcone_type, D->rcone_dim, D->m, "row cones", P->rt, P->rd);
        P->xblk.push_back((int64_t)P->xt.size()), P->rblk.push_back((int64_t)P->rt.size());
        n += D->n, m += D->m, nnz += D->nnz;
        P->inst.push_back(I);
    }
    for (const InstDims &I : P->inst)
        if (I.nnz >= ((int64_t)1 << 31))
            fail(PDCS_ERR_NOT_SUPPORTED, "each instance's nnz must be below 2^31");
    if (n >= ((int64_t)1 << 31) || m >= ((int64_t)1 << 31))
        fail(PDCS_ERR_NOT_SUPPORTED, "n and m must be below 2^31");
    P->n = n, P->m = m, P->nnz = nnz;
    const int64_t B = count;
    hipStream_t s = P->stream;
    DevMem &M = P->mem;
    P->G = Csr{m, n, nnz, M.alloc<int64_t>(m + 1), M.alloc<int32_t>(nnz), M.alloc<double>(nnz)};
    P->Gt = Csr{n, m, nnz, M.alloc<int64_t>(n + 1), M.alloc<int32_t>(nnz), M.alloc<double>(nnz)};
    P->c = M.alloc<double>(n);
    P->h = M.alloc<double>(m);
    P->l = M.alloc<double>(n);
    P->u = M.alloc<double>(n);
    fill(P->l, n, -INFINITY, s);
    fill(P->u, n, INFINITY, s);
    if (B == 1) {
        const pdcs_problem_desc *D = Ds;
        const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        auto cp = [&](void *dst, const void *src, size_t bytes) {
            if (bytes) PDCS_HIP(hipMemcpyAsync(dst, src, bytes, kind, s));
        };
        cp(P->G.rp, D->row_ptr, sizeof(int64_t) * (m + 1));
        cp(P->G.ci, D->col, sizeof(int32_t) * nnz);
        cp(P->G.v, D->val, sizeof(double) * nnz);
        cp(P->c, D->c, sizeof(double) * n);
        cp(P->h, D->h, sizeof(double) * m);
        cp(P->l, D->l, sizeof(double) * D->n_box);
        cp(P->u, D->u, sizeof(double) * D->n_box);
    } else {
        std::vector<int64_t> rp(m + 1);
        std::vector<int32_t> ci(nnz), xi(n), yi(m);
        std::vector<double> val(nnz), c(n), h(m), l(n, -INFINITY), u(n, INFINITY);
        std::vector<int64_t> xo(B + 1), yo(B + 1), ko(B + 1);
        rp[0] = 0;
        for (int64_t b = 0; b < B; ++b) {
            const pdcs_problem_desc *D = Ds + b;
            const InstDims &I = P->inst[b];
            if (D->row_ptr[0] != 0 || D->row_ptr[D->m] != D->nnz)
                fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
            for (int64_t r = 0; r < D->m; ++r) {
                if (D->row_ptr[r] > D->row_ptr[r + 1])
                    fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
                rp[I.y0 + r + 1] = I.k0 + D->row_ptr[r + 1];
            }
            for (int64_t k = 0; k < D->nnz; ++k) {
                if (D->col[k] < 0 || D->col[k] >= D->n)
                    fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
                ci[I.k0 + k] = (int32_t)(I.x0 + D->col[k]);
                val[I.k0 + k] = D->val[k];
            }
            std::copy(D->c, D->c + D->n, c.begin() + I.x0);
            if (D->m) std::copy(D->h, D->h + D->m, h.begin() + I.y0);
            std::copy(D->l, D->l + D->n_box, l.begin() + I.x0);
            std::copy(D->u, D->u + D->n_box, u.begin() + I.x0);
            std::fill(xi.begin() + I.x0, xi.begin() + I.x0 + I.n, (int32_t)b);
            std::fill(yi.begin() + I.y0, yi.begin() + I.y0 + I.m, (int32_t)b);
            xo[b] = I.x0, yo[b] = I.y0, ko[b] = I.k0;
        }
        xo[B] = n, yo[B] = m, ko[B] = nnz;
        h2d(P->G.rp, rp.data(), m + 1, s);
        h2d(P->G.ci, ci.data(), nnz, s);
        h2d(P->G.v, val.data(), nnz, s);
        h2d(P->c, c.data(), n, s);
        h2d(P->h, h.data(), m, s);
        h2d(P->l, l.data(), n, s);
        h2d(P->u, u.data(), n, s);
        P->x_inst = M.alloc<int32_t>(n), P->y_inst = M.alloc<int32_t>(m);
        P->x_off = M.alloc<int64_t>(B + 1), P->y_off = M.alloc<int64_t>(B + 1);
        P->k_off = M.alloc<int64_t>(B + 1);
        h2d(P->x_inst, xi.data(), n, s);
        h2d(P->y_inst, yi.data(), m, s);
        h2d(P->x_off, xo.data(), B + 1, s);
        h2d(P->y_off, yo.data(), B + 1, s);
        h2d(P->k_off, ko.data(), B + 1, s);
        PDCS_HIP(hipStreamSynchronize(s));
        P->h_rp = std::move(rp), P->h_ci = std::move(ci), P->h_val = std::move(val);
        P->h_c = std::move(c), P->h_h = std::move(h), P->h_l = std::move(l), P->h_u = std::move(u);
    }
    P->flag = M.alloc<int>(4);
    PDCS_HIP(hipMemsetAsync(P->flag, 0, sizeof(int) * 4, s));
    const int64_t vk = std::max(m + 1, nnz);
    hipLaunchKernelGGL(validate_csr_kernel, dim3((unsigned)((vk + 255) / 256)), dim3(256), 0, s,
                       P->G.rp, m, P->G.ci, nnz, n, P->flag);
    hipLaunchKernelGGL(validate_bounds_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       P->l, P->u, n, P->flag);
    check_finite(P->G.v, nnz, P->flag, s);
    check_finite(P->c, n, P->flag, s);
    check_finite(P->h, m, P->flag, s);
    int flag = 0;
    d2h(&flag, P->flag, 1, s);
    PDCS_HIP(hipStreamSynchronize(s));
    if (flag & 2) fail(PDCS_ERR_INVALID_ARG, "malformed CSR (row_ptr or column index)");
    if (flag & 4) fail(PDCS_ERR_INVALID_ARG, "bounds: NaN, l > u, l = +inf or u = -inf");
    if (flag & 1) fail(PDCS_ERR_NONFINITE, "non-finite value in G, c or h");

    if (!R.d.empty()) {
        P->rx = std::move(R.xpair), P->ry = std::move(R.ypair);
        P->rx_b = std::move(R.xpair_b), P->ry_b = std::move(R.ypair_b);
        P->rx_dev = M.alloc<int64_t>((int64_t)P->rx.size());
        P->ry_dev = M.alloc<int64_t>((int64_t)P->ry.size());
        P->rtmp = M.alloc<double>(n + m);
        h2d(P->rx_dev, P->rx.data(), (int64_t)P->rx.size(), s);
        h2d(P->ry_dev, P->ry.data(), (int64_t)P->ry.size(), s);
        PDCS_HIP(hipStreamSynchronize(s));
    }
    create_log("uploaded", t_create);
    transpose_blocks(P.get(), s);
    create_log("transposed", t_create);
    std::vector<int64_t> hrp(m + 1), hrpt(n + 1);
    d2h(hrp.data(), P->G.rp, m + 1, s);
    d2h(hrpt.data(), P->Gt.rp, n + 1, s);
    PDCS_HIP(hipStreamSynchronize(s));

    // Internal order of x.  The gathers of x^ in G~x^ follow column popularity
    // (power-law degrees put most of the accesses on few columns), so in each
    // instance the hottest columns are renumbered to the front: first the
    // entries of the elementwise sets (box; zero, free and nonnegative cones,
    // all held as bounds [l, u]), then the SOC and exponential blocks, each
    // kept whole and rated by its largest degree.  Hot columns then share cache
    // lines.
    //   Columns with the same rows (the parts x1 - x2 of a split free
    // variable, say) are gathered by the same rows of G~: placed side by side
    // they share cache lines in G~x^, and their rows of G~^T read the same
    // entries of y^.  Outside the hottest units, columns of degree >= 2 are
    // grouped by a hash of their row lists (a collision only costs locality).
    {
        std::vector<double> ul(n), uu(n);   // the caller's bounds, caller's order
        d2h(ul.data(), P->l, n, s);
        d2h(uu.data(), P->u, n, s);
        std::vector<int32_t> hci(nnz);      // rows of each column, ascending
        d2h(hci.data(), P->Gt.ci, nnz, s);
        PDCS_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> perm(n), pos(n);
        std::vector<double> il(n), iu(n);
        P->ixblk.assign(1, 0);
        for (int64_t b = 0; b < B; ++b) {
            InstDims &I = P->inst[b];
            auto deg = [&](int64_t j) { return hrpt[I.x0 + j + 1] - hrpt[I.x0 + j]; };
            struct Unit { int64_t start, dim, heat; int32_t type; };
            std::vector<Unit> elem, blk;
            for (int64_t j = 0; j < I.nb; ++j) elem.push_back({j, 1, deg(j), -1});
            int64_t o = I.nb;
            for (int64_t k = P->xblk[b]; k < P->xblk[b + 1]; ++k) {
                const int32_t t = P->xt[k];
                const int64_t d = P->xd[k];
                if (t == kZero || t == kFree || t == kNonneg) {
                    for (int64_t j = 0; j < d; ++j) elem.push_back({o + j, 1, deg(o + j), t});
                } else {
                    int64_t h = 0;
                    for (int64_t j = 0; j < d; ++j) h = std::max(h, deg(o + j));
                    blk.push_back({o, d, h, t});
                }
                o += d;
            }
            auto hotter = [](const Unit &a, const Unit &c) { return a.heat > c.heat; };
// the hottest 1% of units move to the front, by degree; the others keep
            // their order (sorting them all clusters the long rows of G~^T, which
            // cost the transposed product more than the gathers gained: measured)
            auto front = [&](std::vector<Unit> &v) -> size_t {
                if (v.empty()) return 0;
                std::vector<int64_t> hs;
                for (auto &u : v) hs.push_back(u.heat);
                const size_t k = hs.size() / 100;
                std::nth_element(hs.begin(), hs.begin() + k, hs.end(), std::greater<int64_t>());
                const int64_t thr = hs[k];
                auto mid = std::stable_partition(v.begin(), v.end(),
                                                 [&](const Unit &u) { return u.heat > thr; });
                std::stable_sort(v.begin(), mid, hotter);
                return (size_t)(mid - v.begin());
            };
            auto twins = [&](std::vector<Unit> &v, size_t from) {
                const size_t cnt = v.size() - from;
                std::vector<std::pair<uint64_t, uint32_t>> hv;
                for (size_t i = 0; i < cnt; ++i) {
                    const Unit &u = v[from + i];
                    if (u.heat < 2) continue;
                    const int64_t g = I.x0 + u.start;
                    uint64_t h = 0x9E3779B97F4A7C15ull ^ (uint64_t)u.heat;
                    for (int64_t k = hrpt[g]; k < hrpt[g + 1]; ++k) {
                        h ^= (uint64_t)(uint32_t)hci[k] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
                        h *= 0xBF58476D1CE4E5B9ull;
                    }
                    hv.push_back({h, (uint32_t)i});
                }
                if (hv.empty()) return;
                std::sort(hv.begin(), hv.end());
                std::vector<int64_t> next(cnt, -1);
                bool any = false;
                for (size_t a = 0; a + 1 < hv.size(); ++a)
                    if (hv[a].first == hv[a + 1].first) next[hv[a].second] = hv[a + 1].second, any = true;
                if (!any) return;
                std::vector<Unit> out;
                out.reserve(cnt);
                std::vector<char> placed(cnt, 0);
                for (size_t i = 0; i < cnt; ++i) {
                    if (placed[i]) continue;
                    for (int64_t j = (int64_t)i; j >= 0; j = next[j])
                        if (!placed[j]) out.push_back(v[from + j]), placed[j] = 1;
                }
                std::copy(out.begin(), out.end(), v.begin() + from);
            };
            twins(elem, front(elem));
            front(blk);
            int64_t q = 0;
            for (const Unit &u : elem) {
                const int64_t g = I.x0 + u.start, p = I.x0 + q++;
                perm[p] = (int32_t)g;
                il[p] = u.type < 0 ? ul[g] : (u.type == kFree ? -INFINITY : 0.0);
                iu[p] = u.type < 0 ? uu[g] : (u.type == kZero ? 0.0 : INFINITY);
            }
            I.nb_in = q;
            for (const Unit &u : blk) {
                for (int64_t j = 0; j < u.dim; ++j) {
                    const int64_t p = I.x0 + q++;
                    perm[p] = (int32_t)(I.x0 + u.start + j);
                    il[p] = -INFINITY, iu[p] = INFINITY;
                }
                P->ixt.push_back(u.type), P->ixd.push_back(u.dim);
            }
            P->ixblk.push_back((int64_t)P->ixt.size());
        }
        for (int64_t p = 0; p < n; ++p) pos[perm[p]] = (int32_t)p;
        P->xperm = M.alloc<int32_t>(n), P->xpos = M.alloc<int32_t>(n);
        h2d(P->xperm, perm.data(), n, s);
        h2d(P->xpos, pos.data(), n, s);
        h2d(P->l, il.data(), n, s);
        h2d(P->u, iu.data(), n, s);
        create_log("column order chosen", t_create);
        relabel(P->G.ci, nnz, P->xpos, s);
        double *cu = M.alloc<double>(n);
        copy_vec(P->c, cu, n, s);
        gather(P->c, cu, P->xperm, n, s);
        transpose_blocks(P.get(), s);
        d2h(hrpt.data(), P->Gt.rp, n + 1, s);
        PDCS_HIP(hipStreamSynchronize(s));   // the host vectors die at the end of this block
    }
    create_log("transposed in the column order", t_create);
    set_plan(P.get(), 0, 0);
    set_plan(P.get(), 1, 0);
    create_log("product plans built", t_create);
    HostPlan hx, hy;
    for (int64_t b = 0; b < B; ++b) {
        const InstDims &I = P->inst[b];
        append_plan(hx, (int32_t)b, I.x0, I.nb_in, I.x0 + I.nb_in, P->ixt.data() + P->ixblk[b],
                    P->ixd.data() + P->ixblk[b], P->ixblk[b + 1] - P->ixblk[b]);
        append_plan(hy, (int32_t)b, I.y0, 0, I.y0, P->rt.data() + P->rblk[b], P->rd.data() + P->rblk[b],
                    P->rblk[b + 1] - P->rblk[b]);
    }
    P->planX = upload_plan(M, hx, s);
    P->planY = upload_plan(M, hy, s);

    P->Gs = Csr{m, n, nnz, P->G.rp, P->G.ci, M.alloc<double>(nnz)};
    P->Gts = Csr{n, m, nnz, P->Gt.rp, P->Gt.ci, M.alloc<double>(nnz)};
    P->ones_n = M.alloc<double>(n);
    P->ones_m = M.alloc<double>(m);
    fill(P->ones_n, n, 1.0, s);
    fill(P->ones_m, m, 1.0, s);
    P->e = M.alloc<double>(m), P->f = M.alloc<double>(n);
    P->cs = M.alloc<double>(n), P->hs = M.alloc<double>(m);
    P->ls = M.alloc<double>(n), P->us = M.alloc<double>(n);
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
    P->seg = M.alloc<double>(5 * B);
    P->rcode = M.alloc<int32_t>(B);
    P->kraw = M.alloc<KktRaw>(3 * B);
    P->st = M.alloc<DevState>(B);
    std::vector<double> r(2 * B, 0.0);
    if (B == 1) {
        reduce_absmax(P->c, n, P->seg + 0, s);
        reduce_absmax(P->h, m, P->seg + 1, s);
    } else {
        reduce_segments(1, P->c, P->x_off, B, P->seg, s);
        reduce_segments(1, P->h, P->y_off, B, P->seg + B, s);
    }
    d2h(r.data(), P->seg, 2 * B, s);
    PDCS_HIP(hipStreamSynchronize(s));
    P->cinf.assign(r.begin(), r.begin() + B);
    P->hinf.assign(r.begin() + B, r.end());
    for (int64_t b = 0; b < B; ++b)
        if (P->inst[b].m == 0) P->hinf[b] = 0.0;
    sync_slab_values(P.get());
    create_log("ready", t_create);
    return P.release();
}

// Rescaling of Section 3 (reading: Ruiz passes + one Pock-Chambolle pass),
// cached for the parameters it was computed with.  The row and column passes
// of a block-diagonal batch touch one instance each, so a batch is rescaled
// instance by instance.
static void ensure_scaling(pdcs_problem *P, int ruiz, int pc) {
    if (P->scaled_ruiz == ruiz && P->scaled_pc == pc) return;
    hipStream_t s = P->stream;
    const int64_t n = P->n, m = P->m, B = P->B;
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
    if (P->Gs.v32) {   // keep the FP32 copies in step with the scaling
        to_float(P->Gs.v, P->Gs.v32, P->nnz, s);
        to_float(P->Gts.v, P->Gts.v32, P->nnz, s);
    }
    sync_slab_values(P);
    scale_problem_vectors(n, m, n, P->c, P->h, P->l, P->u, P->e, P->f, P->cs, P->hs, P->ls,
                          P->us, P->dx, P->dy, s);
    std::vector<double> r(3 * B, 0.0);
    if (B == 1) {
        reduce_absmax(P->Gs.v, P->nnz, P->seg + 0, s);
        reduce_sumsq(P->cs, n, P->seg + 1, s);
        reduce_sumsq(P->hs, m, P->seg + 2, s);
    } else {
        reduce_segments(1, P->Gs.v, P->k_off, B, P->seg, s);
        reduce_segments(0, P->cs, P->x_off, B, P->seg + B, s);
        reduce_segments(0, P->hs, P->y_off, B, P->seg + 2 * B, s);
    }
    d2h(r.data(), P->seg, 3 * B, s);
    PDCS_HIP(hipStreamSynchronize(s));
    P->gmax.resize(B), P->cs_norm.resize(B), P->hs_norm.resize(B);
    for (int64_t b = 0; b < B; ++b) {
        P->gmax[b] = P->inst[b].nnz > 0 ? r[b] : 0.0;
        P->cs_norm[b] = std::sqrt(r[B + b]);
        P->hs_norm[b] = P->inst[b].m > 0 ? std::sqrt(r[2 * B + b]) : 0.0;
    }
    P->scaled_ruiz = ruiz, P->scaled_pc = pc;
}

// FP32 copies for the mixed-precision form, made once per problem (and kept in
// step with the scaling by ensure_scaling).
static void ensure_fp32(pdcs_problem *P) {
    if (P->Gs.v32) return;
    hipStream_t s = P->stream;
    P->xh32 = P->mem.alloc<float>(P->n);
    P->yh32 = P->mem.alloc<float>(P->m);
    float *g32 = P->mem.alloc<float>(P->nnz), *gt32 = P->mem.alloc<float>(P->nnz);
    to_float(P->Gs.v, g32, P->nnz, s);
    to_float(P->Gts.v, gt32, P->nnz, s);
    P->Gs.v32 = g32, P->Gts.v32 = gt32;
    sync_slab_values(P);
}

// Host copies of G's (or G^T's) column indices and the running column counts.
static void slab_source(pdcs_problem *P, bool transposed, std::vector<int32_t> &ci,
                        std::vector<int64_t> &cc) {
    const Csr &A = transposed ? P->Gt : P->G;
    const Csr &At = transposed ? P->G : P->Gt;
    ci.resize(A.nnz), cc.resize(At.rows + 1);
    d2h(ci.data(), A.ci, A.nnz, P->stream);
    d2h(cc.data(), At.rp, At.rows + 1, P->stream);
    PDCS_HIP(hipStreamSynchronize(P->stream));
}

// The layout code of a plan (see pdcs_set_layout).
static int layout_code(const SpmvPlan &pl) {
    return pl.n_slabs > 0 ? slab_code(pl.n_slabs - (pl.hot_cols > 0)) : pl.stream ? -1 : pl.lanes;
}

static bool valid_layout(int code) {
    if (code == 0 || code == -1) return true;
    for (int L = 2; L <= 64; L <<= 1)
        if (code == L) return true;
    const int S = slabs_of(code);
    return S == 1 || S == 2 || S == 4 || S == 8;
}

// The default layout of a product: column slabs when the gathered vector
// passes half an XCD's L2 (one slab per 2 MB of it, 2 to 8 slabs), so each
// XCD keeps its slab cached beside the streamed entries; else 0 (CSR-stream for rows averaging fewer than 12
// entries, row-split otherwise).  Batches keep the latter (their instances'
// vectors are small; the autotuner can still pick slabs).
static int default_layout(const pdcs_problem *P, int side) {
    const Csr &A = side == 0 ? P->G : P->Gt;
    const double bytes = 8.0 * (double)A.cols;
    if (P->B != 1 || bytes <= kXcdL2Bytes / 2 || A.nnz >= INT32_MAX || A.rows >= INT32_MAX) return 0;
    int S = 2;
    while (S < kMaxSlabs && bytes > S * (kXcdL2Bytes / 2.0)) S <<= 1;
    return slab_code(S);
}

// Rebuilds the plan of G x (side 0) or G^T y (side 1) in layout `code`, frees
// the old plan's arrays once the device is idle, and drops the captured graphs
// (they hold the old plan).  The caller refreshes the slab values.
static void set_plan(pdcs_problem *P, int side, int code) {
    hipStream_t s = P->stream;
    if (code == 0) code = default_layout(P, side);
    const Csr &A = side == 0 ? P->G : P->Gt;
    std::vector<int64_t> rp(A.rows + 1);
    d2h(rp.data(), A.rp, A.rows + 1, s);
    PDCS_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> ci;
    std::vector<int64_t> cc;
    if (slabs_of(code)) {
        if (P->nnz >= INT32_MAX || A.rows >= INT32_MAX)
            fail(PDCS_ERR_NOT_SUPPORTED, "column slabs need fewer than 2^31 rows and entries");
        slab_source(P, side == 1, ci, cc);
    }
    auto mem = std::make_unique<DevMem>();
    const SpmvPlan pl = build_spmv_plan(*mem, rp, s, code, SlabSource{&ci, &cc});
    PDCS_HIP(hipDeviceSynchronize());   // no launch in flight still reads the old plan
    for (hipGraphExec_t &g : P->gexec)
        if (g) (void)hipGraphExecDestroy(g), g = nullptr;
    (side == 0 ? P->pG : P->pGt) = pl;
    P->planmem[side] = std::move(mem);
}

// Autotuner of the product plans: times each candidate layout (CSR-stream,
// row-split with 2..64 lanes per row, 2, 4 or 8 column slabs) of G~ and G~^T
// on the problem's own matrices with HIP events and keeps the fastest.  Runs
// once per problem, before the first graph capture.
static void autotune_spmv(pdcs_problem *P) {
    if (P->tuned) return;
    hipStream_t s = P->stream;
    std::vector<int64_t> hrp(P->m + 1), hrpt(P->n + 1);
    d2h(hrp.data(), P->G.rp, P->m + 1, s);
    d2h(hrpt.data(), P->Gt.rp, P->n + 1, s);
    PDCS_HIP(hipStreamSynchronize(s));
    hipEvent_t a, b;
    PDCS_HIP(hipEventCreate(&a));
    PDCS_HIP(hipEventCreate(&b));
    const bool slab_ok = P->nnz < INT32_MAX && P->m < INT32_MAX && P->n < INT32_MAX;
    std::vector<int> cands{-1, 2, 4, 8, 16, 32, 64};
    if (slab_ok)
        for (int S : {2, 4, 8}) cands.push_back(slab_code(S));
    for (int side = 0; side < 2; ++side) {
        Csr A = side == 0 ? P->Gs : P->Gts;
        const std::vector<int64_t> &rp = side == 0 ? hrp : hrpt;
        std::vector<int32_t> hci;
        std::vector<int64_t> hcc;
        if (slab_ok) slab_source(P, side == 1, hci, hcc);
        const SlabSource src{&hci, &hcc};
        double *in = side == 0 ? P->ones_n : P->ones_m;
        double *out = side == 0 ? P->tmp_m : P->tmp_n;
        DevMem vals;
        A.sv = slab_ok ? vals.alloc<double>(A.nnz) : nullptr;
        A.sv32 = nullptr;
        float best = INFINITY;
        int best_c = 0;
        for (int c : cands) {
            DevMem tmp;
            const SpmvPlan plan = build_spmv_plan(tmp, rp, s, c, src);
            // a plan whose launch would exceed 2^31 work-items (a workgroup per
            // long-row chunk when most rows count as long) is not a candidate
            if (spmv_blocks(A, plan) + 64 > kMaxLaunchBlocks) continue;
            slab_values(A, plan, s);
            spmv(A, plan, in, out, SpmvSkip{}, s);   // warm
            PDCS_HIP(hipEventRecord(a, s));
            for (int r = 0; r < 5; ++r) spmv(A, plan, in, out, SpmvSkip{}, s);
            PDCS_HIP(hipEventRecord(b, s));
            PDCS_HIP(hipEventSynchronize(b));
            float ms = 0.0f;
            PDCS_HIP(hipEventElapsedTime(&ms, a, b));
            if (ms < best) best = ms, best_c = c;
        }
        set_plan(P, side, best_c);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    sync_slab_values(P);
    P->tuned = 1;
}

// Fixed step step_fixed / ||G~_b||_2 per instance, the norm by power iteration
// on G~^T G~ from the normalised all-ones vector (the plain-PDHG step of the
// ablation); the blocks of a batch are iterated together, each normalised on
// its own.
static std::vector<double> fixed_step(pdcs_problem *P, const pdcs_settings *S) {
    hipStream_t s = P->stream;
    const int64_t n = P->n, B = P->B;
    std::vector<double> v(B);
    for (int64_t b = 0; b < B; ++b) v[b] = 1.0 / std::sqrt((double)P->inst[b].n);
    h2d(P->seg, v.data(), B, s);
    fill_by_inst(P->tmp_n, P->x_inst, P->seg, n, s);
    double *sums = P->seg + B;
    for (int it = 0; it < S->power_iters; ++it) {
        spmv(P->Gs, P->pG, P->tmp_n, P->tmp_m, SpmvSkip{}, s);
        spmv(P->Gts, P->pGt, P->tmp_m, P->atyh, SpmvSkip{}, s);
        if (B == 1)
            reduce_sumsq(P->atyh, n, sums, s);
        else
            reduce_segments(0, P->atyh, P->x_off, B, sums, s);
        scale_by_inv_sqrt(P->atyh, sums, P->x_inst, P->tmp_n, n, s);
    }
    d2h(v.data(), sums, B, s);
    PDCS_HIP(hipStreamSynchronize(s));
    for (int64_t b = 0; b < B; ++b) {
        const double lam = std::sqrt(v[b]);
        v[b] = (S->power_iters > 0 && lam > 0.0) ? S->step_fixed / std::sqrt(lam) : 1.0;
    }
    return v;
}

struct Kkt {
    double err_p, err_d, err_gap, pobj, dobj, dx2, dy2;
    double avg() const { return (err_p + err_d + err_gap) / 3.0; }
    double mx() const { return std::max(err_p, std::max(err_d, err_gap)); }
};

static Kkt kkt_from_raw(const pdcs_problem *P, int64_t b, const KktRaw &r) {
    Kkt k;
    k.err_p = r.rows_max[0] / (1.0 + std::max(P->hinf[b], std::max(r.rows_max[1], r.rows_max[2])));
    k.err_d = r.cols_max[0] / (1.0 + std::max(P->cinf[b], r.cols_max[1]));
    k.pobj = r.cols_sum[0];
    k.dobj = r.rows_sum[0] + r.cols_sum[1];
    k.err_gap = std::fabs(k.pobj - k.dobj) / (1.0 + std::max(std::fabs(k.pobj), std::fabs(k.dobj)));
    k.dx2 = r.cols_sum[2];
    k.dy2 = r.rows_sum[1];
    return k;
}

// Enqueue the termination measures of the scaled points (xc, yc) of every
// instance with products gxc = G~xc and atyc = G~^T yc into kraw[slot B + b];
// distances are to (xa, ya).
static void enqueue_kkt(pdcs_problem *P, const double *xc, const double *yc, const double *gxc,
                        const double *atyc, const double *xa, const double *ya, const double *e,
                        const double *f, int slot) {
    hipStream_t s = P->stream;
    pass_kkt_rows(P->planY, KktRowsArgs{gxc, P->h, e, yc, ya, P->tmp_m}, P->partY, s);
    pass_kkt_cols(P->planX, KktColsArgs{atyc, P->c, f, P->l, P->u, xc, xa, P->tmp_n}, P->partX, s);
    reduce_kkt(P->B, P->partY, P->planY.inst_tiles, P->planY.ntiles, P->partX, P->planX.inst_tiles,
               P->planX.ntiles, P->kraw + slot * P->B, s);
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
    info->polish_iter = 0;
}

// One step attempt of Algorithm 1 (see the file header) for every instance,
// `batch` times.  With `ev`, event ev[(PDCS_K_COUNT + 1) b + j] is recorded
// before kernel j of attempt b and ev[(PDCS_K_COUNT + 1) b + PDCS_K_COUNT]
// after its last kernel.
static void enqueue_attempts(pdcs_problem *P, long long batch, int mode, hipStream_t s,
                             const hipEvent_t *ev = nullptr) {
    const bool mixed = mode > 0;
    const PrimalArgs pa{P->x, P->aty, P->cs, P->ls, P->us, P->dx, P->xh, P->st,
                        mixed ? P->xh32 : nullptr, mode == 2 ? 1 : 0};
    // each product is one launch: its finishing sums are taken by the dual
    // pass (G~x^) and the Halpern step (G~^T y^)
    DualArgs da{P->y, P->gxh, P->gx, P->hs, P->dy, P->yh, P->st, mixed ? P->yh32 : nullptr};
    da.fp32proj = mode == 2 ? 1 : 0;
    da.gt = tail_of(P->pG, P->m);
    da.gxh_out = P->gxh;
    HalpernArgs ha{P->x,  P->aty, P->xsum, P->xh, P->atyh, P->xa, P->aty0, P->y, P->gx,
                   P->ysum, P->yh, P->gxh, P->ya, P->gx0,  P->n,    P->m,  P->st,
                   P->x_inst, P->y_inst};
    ha.at = tail_of(P->pGt, P->n);
    // the step decision runs in the G~^T launch, so that product cannot wait
    // for it: it is formed for every running instance (and unused after a
    // rejected attempt); the decision's halt takes effect in the next attempt
    ha.promote = P->st;
    ha.n_inst = P->B;
    DecideArgs dec;
    dec.st = P->st, dec.B = P->B;
    dec.px = P->partX, dec.tx = P->planX.inst_tiles, dec.ntx = P->planX.ntiles;
    dec.py = P->partY, dec.ty = P->planY.inst_tiles, dec.nty = P->planY.ntiles;
    const SpmvSkip on_halt{P->st, P->y_inst, SkipHalt};       // rows of G~: y entries
    const SpmvSkip on_halt_t{P->st, P->x_inst, SkipHalt};     // rows of G~^T: x entries
    constexpr int E = PDCS_K_COUNT + 1;
    auto mark = [&](long long b, int j) {
        if (ev) PDCS_HIP(hipEventRecord(ev[E * b + j], s));
    };
    for (long long b = 0; b < batch; ++b) {
        mark(b, PDCS_K_PRIMAL);
        pass_primal(P->planX, pa, P->partX, s);
        mark(b, PDCS_K_SPMV_G);
        if (mixed)
            spmv32_head(P->Gs, P->pG, P->xh32, P->gxh, on_halt, s);
        else
            spmv_head(P->Gs, P->pG, P->xh, P->gxh, on_halt, s);
        mark(b, PDCS_K_DUAL);
        pass_dual(P->planY, da, P->partY, s);
        mark(b, PDCS_K_DECIDE);   // no launch of its own: inside the next one
        mark(b, PDCS_K_SPMV_GT);
        if (mixed)
            spmv32_head(P->Gts, P->pGt, P->yh32, P->atyh, on_halt_t, s, dec);
        else
            spmv_head(P->Gts, P->pGt, P->yh, P->atyh, on_halt_t, s, dec);
        mark(b, PDCS_K_HALPERN);
        halpern(ha, s);
        mark(b, PDCS_K_COUNT);
    }
}

// Captures kGraphBatch attempts once per problem on a library-owned stream
// (the caller's stream may be the null stream, which cannot be captured).
static void ensure_graph(pdcs_problem *P, int mode) {
    if (P->gexec[mode]) return;
    if (!P->gstream) PDCS_HIP(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
    if (!P->ev_in) PDCS_HIP(hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming));
    if (!P->ev_out) PDCS_HIP(hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming));
    hipGraph_t g = nullptr;
    PDCS_HIP(hipStreamBeginCapture(P->gstream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_attempts(P, kGraphBatch, mode, P->gstream);
    } catch (...) {
        (void)hipStreamEndCapture(P->gstream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    PDCS_HIP(hipStreamEndCapture(P->gstream, &g));
    hipError_t e = hipGraphInstantiate(&P->gexec[mode], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    PDCS_HIP(e);
}

static void run_graph(pdcs_problem *P, int mode, hipStream_t s) {
    PDCS_HIP(hipEventRecord(P->ev_in, s));
    PDCS_HIP(hipStreamWaitEvent(P->gstream, P->ev_in, 0));
    PDCS_HIP(hipGraphLaunch(P->gexec[mode], P->gstream));
    PDCS_HIP(hipEventRecord(P->ev_out, P->gstream));
    PDCS_HIP(hipStreamWaitEvent(s, P->ev_out, 0));
}

// A problem of its own for instance b of a batch, from the batch's host copy.
static pdcs_problem *extract_instance(const pdcs_problem *P, int64_t b) {
    const InstDims &I = P->inst[b];
    std::vector<int64_t> rp(I.m + 1);
    std::vector<int32_t> ci(I.nnz);
    for (int64_t r = 0; r <= I.m; ++r) rp[r] = P->h_rp[I.y0 + r] - I.k0;
    for (int64_t k = 0; k < I.nnz; ++k) ci[k] = P->h_ci[I.k0 + k] - (int32_t)I.x0;
    pdcs_problem_desc D{};
    D.n = I.n, D.m = I.m, D.nnz = I.nnz, D.n_box = I.nb;
    D.row_ptr = rp.data(), D.col = ci.data(), D.val = P->h_val.data() + I.k0;
    D.c = P->h_c.data() + I.x0, D.h = P->h_h.data() + I.y0;
    D.l = P->h_l.data() + I.x0, D.u = P->h_u.data() + I.x0;
    D.n_xcones = P->xblk[b + 1] - P->xblk[b];
    D.xcone_type = P->xt.data() + P->xblk[b], D.xcone_dim = P->xd.data() + P->xblk[b];
    D.n_rcones = P->rblk[b + 1] - P->rblk[b];
    D.rcone_type = P->rt.data() + P->rblk[b], D.rcone_dim = P->rd.data() + P->rblk[b];
    return create_impl(&D, 1, P->stream, false);
}

// Algorithm 1 on every instance of P at once.  x0/y0/omega0/xo/yo/infos are
// per instance (x0[b], y0[b] nullable: cold start; omega0 <= 0: default);
// a trace is only for a single problem.
static void solve_batch(pdcs_problem *P, const pdcs_settings *S, const double *const *x0,
                        const double *const *y0, const double *omega0, double *const *xo,
                        double *const *yo, pdcs_info *infos, pdcs_trace *tr) {
    using clk = std::chrono::steady_clock;
    const int64_t B = P->B;
    if (!S || !xo || !yo) fail(PDCS_ERR_INVALID_ARG, "settings, x_out and y_out are required");
    for (int64_t b = 0; b < B; ++b)
        if (!xo[b] || !yo[b]) fail(PDCS_ERR_INVALID_ARG, "settings, x_out and y_out are required");
    if (S->check_every < 1 || S->ruiz_iters < 0 || S->max_attempts < 1 || !(S->tol >= 0.0) ||
        S->step_mode < 0 || S->step_mode > 1 || (S->step_mode == 1 && !(S->step_fixed > 0.0)) ||
        S->precision < 0 || S->precision > 2 || !(S->polish_tol >= 0.0) || S->polish_stall < 1 ||
        S->plain_pdhg < 0 || S->plain_pdhg > 1 || (S->plain_pdhg == 1 && !(S->step_fixed > 0.0)) ||
        S->batch_dropout < 0 || S->batch_dropout > 2)
        fail(PDCS_ERR_INVALID_ARG, "bad settings");
    if (tr && B != 1) fail(PDCS_ERR_INVALID_ARG, "a trace is for a single problem");
    if (tr && (tr->cap < 0 || tr->n_snap < 0 || (tr->n_snap > 0 && (!tr->snap_iter || !tr->snap_x || !tr->snap_y)) ||
               (tr->cap > 0 && (!tr->attempts || !tr->eta_used || !tr->beta || !tr->omega ||
                                !tr->check_code || !tr->check_kkt)) ||
               tr->replay_count < 0 ||
               (tr->replay_count > 0 && (!tr->replay_attempts || !tr->replay_beta || !tr->replay_check_code))))
        fail(PDCS_ERR_INVALID_ARG, "bad trace");
    const int64_t n_replay = tr ? tr->replay_count : 0;
    for (int64_t k = 0; k < n_replay; ++k)
        if (tr->replay_attempts[k] < 1 || tr->replay_check_code[k] < 0 || tr->replay_check_code[k] > 16)
            fail(PDCS_ERR_INVALID_ARG, "bad replay log");
    const auto t_start = clk::now();
    hipStream_t s = P->stream;
    const int64_t n = P->n, m = P->m;
    ensure_scaling(P, S->ruiz_iters, S->pock_chambolle ? 1 : 0);
    if (S->autotune && !P->tuned) autotune_spmv(P);   // drops graphs of the old plans
    // precision mode: 0 FP64; 1 FP32 products; 2 FP32 products and projections
    int mode = S->precision;
    bool mixed = mode > 0;
    if (mixed) ensure_fp32(P);
    int64_t polish_iter = mixed ? -1 : 0;
    std::vector<double> best_mixed(B, INFINITY);
    std::vector<int> stall(B, 0);

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
    int *rp_att = tmem.alloc<int>(n_replay);
    double *rp_beta = tmem.alloc<double>(n_replay);
    if (n_replay > 0) {
        static_assert(sizeof(int) == sizeof(int32_t), "replay log layout");
        h2d(rp_att, (const int *)tr->replay_attempts, n_replay, P->stream);
        h2d(rp_beta, tr->replay_beta, n_replay, P->stream);
    }

    // no root guesses yet: every solve starts from the same state; barrier
    // counters and the timeout flag of grid-level blocks start from zero (a
    // timed-out earlier solve leaves them out of step)
    for (ConePlan *pl : {&P->planX, &P->planY}) {
        fill(pl->soc_root, pl->n_soc, NAN, s);
        fill(pl->exp_root, pl->n_exp, NAN, s);
        clear_grid(*pl, s);
    }

    // z^{0,0}: the mapped starting point projected onto X x Y (reading)
    fill(P->xc[1], n, 0.0, s);   // the caller's order, gathered into the internal one
    fill(P->tmp_m, m, 0.0, s);
    for (int64_t b = 0; b < B; ++b) {
        const InstDims &I = P->inst[b];
        if (x0 && x0[b]) h2d(P->xc[1] + I.x0, x0[b], I.n, s);
        if (y0 && y0[b]) h2d(P->tmp_m + I.y0, y0[b], I.m, s);
    }
    gather(P->tmp_n, P->xc[1], P->xperm, n, s);
    scale_in(P->tmp_n, P->f, P->x, n, s);
    scale_in(P->tmp_m, P->e, P->y, m, s);
    pass_candidate(P->planX, false, CandArgs{P->x, P->ls, P->us, P->dx, P->st, 0, P->xa}, P->partX, s);
    pass_candidate(P->planY, true, CandArgs{P->y, P->ls, P->us, P->dy, P->st, 0, P->ya}, P->partY, s);
    spmv(P->Gs, P->pG, P->xa, P->gx0, SpmvSkip{}, s);
    spmv(P->Gts, P->pGt, P->ya, P->aty0, SpmvSkip{}, s);
    RestartArgs ra{n, m, {P->xa, P->xc[1]}, {P->ya, P->yc[1]}, {P->gx0, P->gxc[1]},
                   {P->aty0, P->atyc[1]}, nullptr, P->x_inst, P->y_inst,
                   P->x, P->y, P->xa, P->ya, P->gx, P->aty, P->gx0, P->aty0, P->xsum, P->ysum};
    restart_copy(ra, s);
    enqueue_kkt(P, P->xa, P->ya, P->gx0, P->aty0, P->xa, P->ya, P->e, P->f, 2);
    std::vector<KktRaw> raw(3 * B);
    d2h(raw.data() + 2 * B, P->kraw + 2 * B, B, s);

    std::vector<double> eta0(B);
    const bool plain = S->plain_pdhg == 1;
    if (S->step_mode == 1 || plain) eta0 = fixed_step(P, S);
    std::vector<DevState> hs(B);
    std::vector<Kkt> k_anchor(B), kout(B);
    std::vector<int> status(B, -1), out_src(B, -2);   // -2: not written yet
    // writes instance b's unscaled output from the anchor (src -1) or a
    // candidate (0, 1); enqueued on s before any later pass reuses the buffers
    auto emit = [&](int64_t b, int src) {
        const InstDims &I = P->inst[b];
        const double *sx = src < 0 ? P->xa : P->xc[src];
        const double *sy = src < 0 ? P->ya : P->yc[src];
        // x: unscaled, then back to the caller's order (atyh is free between attempts)
        unscale(sx + I.x0, P->f + I.x0, P->tmp_n + I.x0, I.n, s);
        if (S->out_on_device) {
            scatter(xo[b], P->tmp_n + I.x0, P->xperm + I.x0, I.n, I.x0, s);
            unscale(sy + I.y0, P->e + I.y0, yo[b], I.m, s);
        } else {
            scatter(P->atyh + I.x0, P->tmp_n + I.x0, P->xperm + I.x0, I.n, I.x0, s);
            unscale(sy + I.y0, P->e + I.y0, P->tmp_m + I.y0, I.m, s);
            d2h(xo[b], P->atyh + I.x0, I.n, s);
            d2h(yo[b], P->tmp_m + I.y0, I.m, s);
        }
        out_src[b] = src;
    };
    std::vector<double> kprev_avg(B, INFINITY);
    std::vector<long long> restarts(B, 0), checks(B, 0);
    PDCS_HIP(hipStreamSynchronize(s));
    for (int64_t b = 0; b < B; ++b) {
        DevState &h = hs[b];
        h = DevState{};
        h.eta = S->step_mode == 1 || plain ? eta0[b] : (P->gmax[b] > 0.0 ? 1.0 / P->gmax[b] : 1.0);
        h.omega = (P->cs_norm[b] > 1e-10 && P->hs_norm[b] > 1e-10) ? P->cs_norm[b] / P->hs_norm[b] : 1.0;
        if (plain) h.omega = 1.0;   // the baseline takes the same step on both sides
        if (omega0 && omega0[b] > 0.0) h.omega = omega0[b];
        h.tau = h.eta / h.omega, h.sigma = h.eta * h.omega;
        h.beta_prev = 1.0, h.r_prev = INFINITY;
        h.max_iter = S->max_iter, h.check_every = S->check_every, h.max_attempts = S->max_attempts;
        h.beta_mode = S->beta_mode, h.beta_const = S->beta_const, h.beta_grow = S->beta_grow;
        h.step_mode = plain ? 1 : S->step_mode;
        h.plain = plain ? 1 : 0;
        if (plain) h.beta_mode = 1, h.beta_const = 0.0;
        h.beta_shrink = S->beta_shrink, h.step_reduce_exp = S->step_reduce_exp;
        h.step_grow_exp = S->step_grow_exp;
        h.log_cap = cap, h.log_attempts = log_att, h.log_eta = log_eta, h.log_beta = log_beta,
        h.log_omega = log_om;
        h.rp_count = n_replay, h.rp_attempts = rp_att, h.rp_beta = rp_beta;
        h.skip_update = 1, h.status = -1;
        k_anchor[b] = kout[b] = kkt_from_raw(P, b, raw[2 * B + b]);
        if (k_anchor[b].mx() <= S->tol) status[b] = PDCS_SOLVE_OPTIMAL;
        if (!(k_anchor[b].mx() == k_anchor[b].mx())) status[b] = PDCS_SOLVE_NUMERICAL;
        if (status[b] < 0 && S->max_iter <= 0) status[b] = PDCS_SOLVE_ITER_LIMIT;
        h.halt = h.halt_next = status[b] >= 0 ? 1 : 0;
    }
    h2d(P->st, hs.data(), B, s);
    const auto t_iter = clk::now();
    double last_log = 0.0;   // progress lines (settings.log_every)
    const double setup_s = std::chrono::duration<double>(t_iter - t_start).count();

    auto active = [&](int64_t b) { return status[b] < 0; };
    auto any_running = [&]() {
        for (int64_t b = 0; b < B; ++b)
            if (active(b) && !hs[b].halt) return true;
        return false;
    };
    auto any_active = [&]() {
        for (int64_t b = 0; b < B; ++b)
            if (active(b)) return true;
        return false;
    };
    int64_t snap = 0;
    const bool stepwise = tr && (tr->cap > 0 || tr->n_snap > 0);
    std::vector<long long> prev_att(B, 0);
    constexpr int E = PDCS_K_COUNT + 1;
    double kms[PDCS_K_COUNT] = {};
    int64_t klaunch[PDCS_K_COUNT] = {};
    if (S->time_kernels && P->tev.empty()) {
        P->tev.resize(E * kGraphBatch, nullptr);
        for (hipEvent_t &e : P->tev) PDCS_HIP(hipEventCreate(&e));
    }
    std::vector<int32_t> code(B, 0), last_src(B, -1);
    std::vector<pdcs_info> handed(B);     // results of instances finished on their own
    std::vector<double> done(B, -1.0);    // seconds until each instance stopped
    std::vector<char> was_handed(B, 0);
    // seconds per attempt over the batch: at the first check (the whole batch
    // running) and since the last check, for the hand-over rule of dropout 2
    double full_att_s = -1.0, t_last_check = 0.0;
    long long att_since = 0;
    while (any_active()) {
        // ---- step attempts until every running instance asks for a check ----
        while (any_running()) {
            long long todo = kGraphBatch;
            for (int64_t b = 0; b < B; ++b)
                if (active(b) && !hs[b].halt)
                    todo = std::min<long long>(todo, S->check_every - hs[b].kin % S->check_every);
            const long long batch = stepwise ? 1 : std::max<long long>(1, todo);
            att_since += batch;
            if (S->time_kernels) {
                enqueue_attempts(P, batch, mode, s, P->tev.data());
            } else if (S->use_graph && batch == kGraphBatch) {
                ensure_graph(P, mode);
                run_graph(P, mode, s);
            } else {
                enqueue_attempts(P, batch, mode, s);
            }
            const long long it_before = hs[0].n_iter;
            std::vector<long long> att_before(B), acc_before(B);
            for (int64_t b = 0; b < B; ++b)
                att_before[b] = hs[b].attempts_total + hs[b].attempts_cur, acc_before[b] = hs[b].n_iter;
            d2h(hs.data(), P->st, B, s);
            PDCS_HIP(hipStreamSynchronize(s));
            if (S->time_kernels) {
                // attempts run in order and an instance halts only at the end of
                // a batch, so the first `worked` attempts did work somewhere
                long long worked = 0, acc = 0;
                for (int64_t b = 0; b < B; ++b) {
                    worked = std::max(worked, hs[b].attempts_total + hs[b].attempts_cur - att_before[b]);
                    acc = std::max(acc, hs[b].n_iter - acc_before[b]);
                }
                for (long long a = 0; a < worked && a < batch; ++a)
                    for (int j = 0; j < PDCS_K_COUNT; ++j) {
                        float ms = 0.0f;
                        PDCS_HIP(hipEventElapsedTime(&ms, P->tev[E * a + j], P->tev[E * a + j + 1]));
                        kms[j] += ms;
                    }
                klaunch[PDCS_K_PRIMAL] += worked, klaunch[PDCS_K_SPMV_G] += worked;
                klaunch[PDCS_K_DUAL] += worked, klaunch[PDCS_K_DECIDE] += worked;
                klaunch[PDCS_K_SPMV_GT] += acc, klaunch[PDCS_K_HALPERN] += acc;
            }
            if (tr && snap < tr->n_snap && hs[0].n_iter > it_before && tr->snap_iter[snap] == hs[0].n_iter) {
                unscale(P->x, P->f, P->tmp_n, n, s);
                scatter(P->atyh, P->tmp_n, P->xperm, n, 0, s);
                unscale(P->y, P->e, P->tmp_m, m, s);
                d2h(tr->snap_x + snap * n, P->atyh, n, s);
                d2h(tr->snap_y + snap * m, P->tmp_m, m, s);
                PDCS_HIP(hipStreamSynchronize(s));
                ++snap;
            }
        }
        for (int64_t b = 0; b < B; ++b)
            if (active(b) && hs[b].status == PDCS_SOLVE_NUMERICAL) status[b] = PDCS_SOLVE_NUMERICAL;
        if (!any_active()) break;
        // ---- check: candidates P(z^{t,k}) and P(z_bar^{t,k}) of every instance ----
        pass_candidate(P->planX, false, CandArgs{P->x, P->ls, P->us, P->dx, P->st, 0, P->xc[0]}, P->partX, s);
        pass_candidate(P->planY, true, CandArgs{P->y, P->ls, P->us, P->dy, P->st, 0, P->yc[0]}, P->partY, s);
        pass_candidate(P->planX, false, CandArgs{P->xsum, P->ls, P->us, P->dx, P->st, 1, P->xc[1]}, P->partX, s);
        pass_candidate(P->planY, true, CandArgs{P->ysum, P->ls, P->us, P->dy, P->st, 1, P->yc[1]}, P->partY, s);
        for (int cnd = 0; cnd < 2; ++cnd) {
            spmv(P->Gs, P->pG, P->xc[cnd], P->gxc[cnd], SpmvSkip{}, s);
            spmv(P->Gts, P->pGt, P->yc[cnd], P->atyc[cnd], SpmvSkip{}, s);
            enqueue_kkt(P, P->xc[cnd], P->yc[cnd], P->gxc[cnd], P->atyc[cnd], P->xa, P->ya, P->e, P->f, cnd);
        }
        d2h(raw.data(), P->kraw, 2 * B, s);
        int gerr[2] = {0, 0};
        if (P->planX.n_grid > 0) d2h(gerr, P->planX.grid_err, 1, s);
        if (P->planY.n_grid > 0) d2h(gerr + 1, P->planY.grid_err, 1, s);
        PDCS_HIP(hipStreamSynchronize(s));
        if (gerr[0] || gerr[1])
            fail(PDCS_ERR_HIP, "a grid-level SOC projection timed out waiting for its workgroups");
        const double elapsed = std::chrono::duration<double>(clk::now() - t_iter).count();
        // the products are one launch over the batch, so the batch switches to
        // FP64 together: as soon as any instance meets the rule (waiting for
        // all of them kept the instances that were ready in FP32 products,
        // short of the tolerance, until the slowest one caught up)
        bool any_restart = false, switch_ok = false;
        int64_t log_running = 0, log_iter = 0;
        double log_kkt = 0.0;
        for (int64_t b = 0; b < B; ++b) {
            code[b] = 0;
            if (!active(b)) continue;
            DevState &h = hs[b];
            ++checks[b];
            ++log_running;
            log_iter = std::max<int64_t>(log_iter, h.n_iter);
            const Kkt k1 = kkt_from_raw(P, b, raw[b]), k2 = kkt_from_raw(P, b, raw[B + b]);
            int chosen = !plain && k2.avg() < k1.avg() ? 1 : 0;
            last_src[b] = chosen;
            Kkt kc = chosen ? k2 : k1;
            double kcv = kc.avg();
            log_kkt = std::max(log_kkt, kc.mx());
            const double kav = k_anchor[b].avg();
            int reason = 0, stop = 0;
            if (!(kcv == kcv)) {
                status[b] = PDCS_SOLVE_NUMERICAL, stop = 1;
            } else if (kc.mx() <= S->tol) {
                status[b] = PDCS_SOLVE_OPTIMAL, stop = 1;
            } else if (h.n_iter >= S->max_iter) {
                status[b] = PDCS_SOLVE_ITER_LIMIT, stop = 1;
            } else if (S->time_limit > 0.0 && elapsed >= S->time_limit) {
                status[b] = PDCS_SOLVE_TIME_LIMIT, stop = 1;
            }
            if (!stop && !plain) {
                if (kcv <= S->restart_sufficient * kav)
                    reason = 1;
                else if (kcv <= S->restart_necessary * kav && kcv > kprev_avg[b])
                    reason = 2;
                else if ((double)h.kin >= S->restart_artificial * (double)h.n_iter)
                    reason = 3;
            }
            const int64_t rec = h.n_iter - 1;
            if (rec >= 0 && rec < n_replay && tr->replay_check_code[rec] > 0) {
                // replay: the other run's candidate, restart reason and stop
                const int rc = tr->replay_check_code[rec] - 1;
                chosen = rc & 1;
                last_src[b] = chosen;
                kc = chosen ? k2 : k1;
                kcv = kc.avg();
                reason = (rc >> 1) & 3;
                stop = (rc >> 3) & 1;
                status[b] = !stop ? -1
                            : (h.n_iter >= S->max_iter && !(kc.mx() <= S->tol)) ? PDCS_SOLVE_ITER_LIMIT
                                                                                : PDCS_SOLVE_OPTIMAL;
            }
            if (tr && rec >= 0 && rec < cap) {
                tr->check_code[rec] = 1 + chosen + 2 * reason + 8 * stop;
                tr->check_kkt[rec] = kcv;
            }
            if (stop) {
                kout[b] = kc;
                done[b] = elapsed;
                h.halt = 1;   // finished: its tiles and rows stay idle
                emit(b, chosen);
                continue;
            }
            if (reason) {
                // PrimalWeightUpdate (reading: PDLP's smoothed log-ratio rule)
                const double ddx = std::sqrt(kc.dx2), ddy = std::sqrt(kc.dy2);
                if (ddx > 1e-10 && ddy > 1e-10)
                    h.omega = std::exp(0.5 * std::log(ddy / ddx) + 0.5 * std::log(h.omega));
                code[b] = 1 + chosen;
                any_restart = true;
                k_anchor[b] = kc;
                kprev_avg[b] = INFINITY;
                h.kin = 0;
                h.eta_sum = 0.0;
                h.beta_prev = 1.0;
                h.r_prev = INFINITY;
                h.tau = h.eta / h.omega, h.sigma = h.eta * h.omega;
                ++restarts[b];
            } else {
                kprev_avg[b] = kcv;
            }
            if (mixed) {
                if (kc.mx() < best_mixed[b]) best_mixed[b] = kc.mx(), stall[b] = 0;
                else ++stall[b];
                if (kc.mx() <= S->polish_tol || stall[b] >= S->polish_stall) switch_ok = true;
            }
        }
        if (S->log_every > 0.0 && elapsed - last_log >= S->log_every) {
            last_log = elapsed;
            std::fprintf(stderr, "pdcs: %9.2f s  %lld of %lld instance(s) at this check, up to %lld iterations, "
                                 "worst max-KKT %.3e\n",
                         elapsed, (long long)log_running, (long long)B, (long long)log_iter, log_kkt);
            std::fflush(stderr);
        }
        if (any_restart) {
            h2d(P->rcode, code.data(), B, s);
            RestartArgs rc{n, m, {P->xc[0], P->xc[1]}, {P->yc[0], P->yc[1]}, {P->gxc[0], P->gxc[1]},
                           {P->atyc[0], P->atyc[1]}, P->rcode, P->x_inst, P->y_inst,
                           P->x, P->y, P->xa, P->ya, P->gx, P->aty, P->gx0, P->aty0, P->xsum, P->ysum};
            restart_copy(rc, s);
        }
        if (mixed && switch_ok && any_active()) {
            // polish phase: FP64 products from here on (reading: the switch rule);
            // the kept products are recomputed in FP64 (a restart brought them
            // with its candidate already; recomputing gives the same bits)
            mixed = false;
            mode = 0;
            for (int64_t b = 0; b < B; ++b)
                if (active(b)) { polish_iter = hs[b].n_iter; break; }
            spmv(P->Gs, P->pG, P->x, P->gx, SpmvSkip{}, s);
            spmv(P->Gts, P->pGt, P->y, P->aty, SpmvSkip{}, s);
            spmv(P->Gs, P->pG, P->xa, P->gx0, SpmvSkip{}, s);
            spmv(P->Gts, P->pGt, P->ya, P->aty0, SpmvSkip{}, s);
            for (int64_t b = 0; b < B; ++b) checks[b] += 1;   // four more products each
        }
        // Stragglers (reading, not in the paper): once the instances still
        // running hold at most 1/8 of the batch's nonzeros, every launch over
        // the batch costs more than their own work.  Each is handed to a problem
        // of its own, restarted at its chosen candidate with its primal weight
        // (a restart, as Algorithm 1 may take at any check), with the rest of
        // the iteration and time budget.
        // dropout 1: at that share.  dropout 2: also only once an attempt over
        // the batch costs more than 4x what the running instances' own
        // attempts would (their share of the first check's cost per attempt,
        // at least kAloneAttemptS each): the launches then mostly dispatch
        // workgroups of finished instances, which return at once.
        const double att_s = att_since > 0 ? (elapsed - t_last_check) / (double)att_since : 0.0;
        if (full_att_s < 0.0) full_att_s = att_s;
        t_last_check = elapsed, att_since = 0;
        if (B > 1 && S->batch_dropout && any_active()) {
            int64_t act_nnz = 0, act_cnt = 0;
            for (int64_t b = 0; b < B; ++b)
                if (active(b)) act_nnz += P->inst[b].nnz, ++act_cnt;
            const double own_s = std::max(full_att_s * (double)act_nnz / (double)std::max<int64_t>(P->nnz, 1),
                                          kAloneAttemptS * (double)act_cnt);
            const bool costly = S->batch_dropout != 2 || att_s > 4.0 * own_s;
            if (8 * act_nnz <= P->nnz && costly) {
                for (int64_t b = 0; b < B; ++b) {
                    if (!active(b)) continue;
                    const InstDims &I = P->inst[b];
                    const int src = last_src[b];
                    std::vector<double> hx(I.n), hy(I.m);
                    unscale((src < 0 ? P->xa : P->xc[src]) + I.x0, P->f + I.x0, P->tmp_n + I.x0, I.n, s);
                    scatter(P->atyh + I.x0, P->tmp_n + I.x0, P->xperm + I.x0, I.n, I.x0, s);
                    unscale((src < 0 ? P->ya : P->yc[src]) + I.y0, P->e + I.y0, P->tmp_m + I.y0, I.m, s);
                    d2h(hx.data(), P->atyh + I.x0, I.n, s);
                    d2h(hy.data(), P->tmp_m + I.y0, I.m, s);
                    PDCS_HIP(hipStreamSynchronize(s));
                    std::unique_ptr<pdcs_problem> sub(extract_instance(P, b));
                    pdcs_settings S2 = *S;
                    S2.max_iter = std::max<int64_t>(0, S->max_iter - hs[b].n_iter);
                    const double used = std::chrono::duration<double>(clk::now() - t_iter).count();
                    if (S->time_limit > 0.0) S2.time_limit = std::max(1e-9, S->time_limit - used);
                    const double *px = hx.data(), *py = hy.data();
                    const double om = hs[b].omega;
                    pdcs_info si{};
                    solve_batch(sub.get(), &S2, &px, &py, &om, &xo[b], &yo[b], &si, nullptr);
                    si.iterations += hs[b].n_iter;
                    si.attempts += hs[b].attempts_total;
                    si.restarts += restarts[b] + 1;
                    si.spmv += hs[b].attempts_total + hs[b].attempts_cur + hs[b].n_iter + 2 + 4 * checks[b];
                    handed[b] = si;
                    was_handed[b] = 1;
                    done[b] = std::chrono::duration<double>(clk::now() - t_iter).count();
                    status[b] = si.status;
                    out_src[b] = src;   // written by the problem of its own
                    hs[b].halt = 1;
                }
            }
        }
        for (int64_t b = 0; b < B; ++b) {
            if (active(b)) hs[b].halt = 0;
            hs[b].halt_next = hs[b].halt;
        }
        h2d(P->st, hs.data(), B, s);
    }

    // ---- outputs of the instances that ended without a final check: the anchor ----
    for (int64_t b = 0; b < B; ++b)
        if (out_src[b] == -2) emit(b, -1);
    if (tr && cap > 0) {
        const int64_t cnt = std::min<int64_t>(cap, hs[0].n_iter);
        d2h(tr->attempts, log_att, cnt, s);
        d2h(tr->eta_used, log_eta, cnt, s);
        d2h(tr->beta, log_beta, cnt, s);
        d2h(tr->omega, log_om, cnt, s);
        tr->count = cnt;
    }
    PDCS_HIP(hipStreamSynchronize(s));
    check_grid(P->planX, s);
    check_grid(P->planY, s);
    P->snaps_written = snap;
    const double solve_s = std::chrono::duration<double>(clk::now() - t_iter).count();
    for (int64_t b = 0; b < B; ++b) {
        if (!infos) break;
        // products: one with G~ per attempt, one with G~^T per accepted
        // iteration, two at the start and four per check
        const long long spmv_count = hs[b].attempts_total + hs[b].attempts_cur + hs[b].n_iter + 2 + 4 * checks[b];
        if (was_handed[b]) {
            infos[b] = handed[b];
            infos[b].setup_s = setup_s, infos[b].solve_s = solve_s;
            infos[b].done_s = done[b];
            continue;
        }
        fill_info(infos + b, status[b], hs[b], restarts[b], spmv_count, kout[b], setup_s, solve_s);
        infos[b].done_s = done[b] >= 0.0 ? done[b] : solve_s;
        for (int j = 0; j < PDCS_K_COUNT; ++j)
            infos[b].kernel_ms[j] = kms[j], infos[b].kernel_launches[j] = klaunch[j];
        infos[b].polish_iter = polish_iter;
    }
}

// The caller's point (x [n] or y [m], device) in the solver's formulation: a
// copy with each rotated pair mapped by T, or v itself when there is none.
static const double *to_solver(pdcs_problem *P, bool is_y, const double *v, hipStream_t s) {
    const std::vector<int64_t> &o = is_y ? P->ry : P->rx;
    if (o.empty()) return v;
    double *t = is_y ? P->rtmp + P->n : P->rtmp;
    d2d(t, v, is_y ? P->m : P->n, s);
    rotate_pairs(t, is_y ? P->ry_dev : P->rx_dev, (int64_t)o.size(), 0, s);
    return t;
}
// Maps a result of the solver's formulation (device) back to the caller's.
static void to_caller(pdcs_problem *P, bool is_y, double *v, hipStream_t s) {
    const std::vector<int64_t> &o = is_y ? P->ry : P->rx;
    if (!o.empty()) rotate_pairs(v, is_y ? P->ry_dev : P->rx_dev, (int64_t)o.size(), 0, s);
}

// solve_batch in the caller's formulation: the rotated pairs of the starting
// points, the solutions and the snapshots are mapped by T.
static void solve_caller(pdcs_problem *P, const pdcs_settings *S, const double *const *x0,
                         const double *const *y0, const double *omega0, double *const *xo,
                         double *const *yo, pdcs_info *infos, pdcs_trace *tr) {
    if (P->rx.empty() && P->ry.empty()) return solve_batch(P, S, x0, y0, omega0, xo, yo, infos, tr);
    const int64_t B = P->B;
    auto span = [&](bool is_y, int64_t b) {
        const std::vector<int64_t> &o = is_y ? P->ry : P->rx, &ob = is_y ? P->ry_b : P->rx_b;
        return std::make_pair(o.data() + ob[b], ob[b + 1] - ob[b]);
    };
    std::vector<std::vector<double>> hx(B), hy(B);
    std::vector<const double *> px(B, nullptr), py(B, nullptr);
    for (int64_t b = 0; b < B; ++b) {
        const InstDims &I = P->inst[b];
        if (x0 && x0[b]) {
            hx[b].assign(x0[b], x0[b] + I.n);
            const auto o = span(false, b);
            rotate_host(hx[b].data(), o.first, o.second, I.x0);
            px[b] = hx[b].data();
        }
        if (y0 && y0[b]) {
            hy[b].assign(y0[b], y0[b] + I.m);
            const auto o = span(true, b);
            rotate_host(hy[b].data(), o.first, o.second, I.y0);
            py[b] = hy[b].data();
        }
    }
    solve_batch(P, S, px.data(), py.data(), omega0, xo, yo, infos, tr);
    for (int64_t b = 0; b < B; ++b) {
        const InstDims &I = P->inst[b];
        const auto ox = span(false, b), oy = span(true, b);
        if (S->out_on_device) {
            rotate_pairs(xo[b], P->rx_dev + P->rx_b[b], ox.second, I.x0, P->stream);
            rotate_pairs(yo[b], P->ry_dev + P->ry_b[b], oy.second, I.y0, P->stream);
        } else {
            rotate_host(xo[b], ox.first, ox.second, I.x0);
            rotate_host(yo[b], oy.first, oy.second, I.y0);
        }
    }
    if (S->out_on_device) PDCS_HIP(hipStreamSynchronize(P->stream));
    for (int64_t i = 0; tr && i < P->snaps_written; ++i) {
        rotate_host(tr->snap_x + i * P->n, P->rx.data(), (int64_t)P->rx.size(), 0);
        rotate_host(tr->snap_y + i * P->m, P->ry.data(), (int64_t)P->ry.size(), 0);
    }
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
    s->precision = 0;
    s->polish_tol = 1e-5;
    s->polish_stall = 8;
    s->autotune = 0;
    s->batch_dropout = 0;
    s->plain_pdhg = 0;
    s->log_every = 0.0;
    return PDCS_OK;
}

pdcs_status pdcs_problem_create(const pdcs_problem_desc *desc, void *hip_stream, pdcs_problem **out) {
    if (!out) {
        g_last_error = "out is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    return guarded([&] { *out = create_impl(desc, 1, hip_stream, false); });
}

pdcs_status pdcs_problem_create_device(const pdcs_problem_desc *desc, void *hip_stream,
                                       pdcs_problem **out) {
    if (!out) {
        g_last_error = "out is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    return guarded([&] { *out = create_impl(desc, 1, hip_stream, true); });
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
        solve_caller(p, settings, &x0, &y0, &omega0, &x_out, &y_out, info, trace);
    });
}

pdcs_status pdcs_scaling(pdcs_problem *p, const pdcs_settings *settings, double *e_out,
                         double *f_out) {
    return guarded([&] {
        if (!p || !settings || !e_out || !f_out) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        ensure_scaling(p, settings->ruiz_iters, settings->pock_chambolle ? 1 : 0);
        d2h(e_out, p->e, p->m, p->stream);
        scatter(p->tmp_n, p->f, p->xperm, p->n, 0, p->stream);
        d2h(f_out, p->tmp_n, p->n, p->stream);
        PDCS_HIP(hipStreamSynchronize(p->stream));
    });
}

pdcs_status pdcs_spmv(pdcs_problem *p, int transpose, const double *x_dev, double *y_dev,
                      void *hip_stream) {
    return guarded([&] {
        if (!p || !x_dev || !y_dev) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        x_dev = to_solver(p, transpose != 0, x_dev, s);
        // columns are held in the internal order of x
        if (transpose) {
            spmv(p->Gt, p->pGt, x_dev, p->tmp_n, SpmvSkip{}, s);
            scatter(y_dev, p->tmp_n, p->xperm, p->n, 0, s);
        } else {
            gather(p->tmp_n, x_dev, p->xperm, p->n, s);
            spmv(p->G, p->pG, p->tmp_n, y_dev, SpmvSkip{}, s);
        }
        to_caller(p, transpose == 0, y_dev, s);
    });
}

pdcs_status pdcs_spmv32(pdcs_problem *p, int transpose, const double *x_dev, double *y_dev,
                        void *hip_stream) {
    return guarded([&] {
        if (!p || !x_dev || !y_dev) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : p->stream;
        if (!p->G.v32) {   // FP32 copies of the unscaled values, made on first use
            float *g32 = p->mem.alloc<float>(p->nnz), *gt32 = p->mem.alloc<float>(p->nnz);
            to_float(p->G.v, g32, p->nnz, s);
            to_float(p->Gt.v, gt32, p->nnz, s);
            p->x32 = p->mem.alloc<float>(std::max(p->n, p->m));
            p->G.v32 = g32, p->Gt.v32 = gt32;
            sync_slab_values(p);
        }
        x_dev = to_solver(p, transpose != 0, x_dev, s);
        // columns are held in the internal order of x
        if (transpose) {
            to_float(x_dev, p->x32, p->m, s);
            spmv32(p->Gt, p->pGt, p->x32, p->tmp_n, SpmvSkip{}, s);
            scatter(y_dev, p->tmp_n, p->xperm, p->n, 0, s);
        } else {
            gather(p->tmp_n, x_dev, p->xperm, p->n, s);
            to_float(p->tmp_n, p->x32, p->n, s);
            spmv32(p->G, p->pG, p->x32, y_dev, SpmvSkip{}, s);
        }
        to_caller(p, transpose == 0, y_dev, s);
    });
}

pdcs_status pdcs_set_layout(pdcs_problem *p, int layout_g, int layout_gt) {
    return guarded([&] {
        if (!p) fail(PDCS_ERR_INVALID_ARG, "NULL problem");
        if (!valid_layout(layout_g) || !valid_layout(layout_gt))
            fail(PDCS_ERR_INVALID_ARG, "unknown layout code");
        set_plan(p, 0, layout_g);
        set_plan(p, 1, layout_gt);
        sync_slab_values(p);
        PDCS_HIP(hipStreamSynchronize(p->stream));
        p->tuned = 1;
    });
}

pdcs_status pdcs_get_layout(const pdcs_problem *p, int *layout_g, int *layout_gt) {
    return guarded([&] {
        if (!p || !layout_g || !layout_gt) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        *layout_g = layout_code(p->pG);
        *layout_gt = layout_code(p->pGt);
    });
}

pdcs_status pdcs_kkt(pdcs_problem *p, const double *x_dev, const double *y_dev, double *out) {
    return guarded([&] {
        if (!p || !x_dev || !y_dev || !out) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        hipStream_t s = p->stream;
        x_dev = to_solver(p, false, x_dev, s);
        y_dev = to_solver(p, true, y_dev, s);
        double *xi = p->xc[1];   // x in the internal order
        gather(xi, x_dev, p->xperm, p->n, s);
        spmv(p->G, p->pG, xi, p->gxc[0], SpmvSkip{}, s);
        spmv(p->Gt, p->pGt, y_dev, p->atyc[0], SpmvSkip{}, s);
        enqueue_kkt(p, xi, y_dev, p->gxc[0], p->atyc[0], xi, y_dev, p->ones_m, p->ones_n, 0);
        KktRaw r;
        d2h(&r, p->kraw, 1, s);
        PDCS_HIP(hipStreamSynchronize(s));
        const Kkt k = kkt_from_raw(p, 0, r);
        out[0] = k.err_p, out[1] = k.err_d, out[2] = k.err_gap, out[3] = k.pobj, out[4] = k.dobj;
    });
}

// Rotated SOC blocks of a cone list become SOC blocks; returns their first
// entries.  T maps the rotated cone onto the SOC, so the projection onto the
// rotated cone is T P_SOC(T v); under a scaling D != I this no longer holds.
static std::vector<int64_t> rsoc_to_soc(std::vector<int32_t> &t, const std::vector<int64_t> &d,
                                        const double *d_dev) {
    std::vector<int64_t> rot;
    for (size_t b = 0, o = 0; b < t.size(); o += d[b], ++b)
        if (t[b] == kRsoc) t[b] = kSoc, rot.push_back((int64_t)o);
    if (!rot.empty() && d_dev) fail(PDCS_ERR_NOT_SUPPORTED, "rotated SOC blocks are projected with D = I");
    return rot;
}

static pdcs_status project_impl(int64_t nblocks, const int32_t *types, const int64_t *dims,
                                int dual, const double *d_dev, double *v_dev, void *hip_stream,
                                int fp32proj) {
    return guarded([&] {
        if (nblocks < 0 || (nblocks > 0 && (!types || !dims || !v_dev)))
            fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        int64_t len = 0;
        for (int64_t b = 0; b < nblocks; ++b) len += dims[b];
        std::vector<int32_t> t;
        std::vector<int64_t> d;
        validate_cones(nblocks, types, dims, len, "cones", t, d);
        const std::vector<int64_t> rot = rsoc_to_soc(t, d, d_dev);
        hipStream_t s = (hipStream_t)hip_stream;
        DevMem mem;
        ConePlan plan = upload_plan(mem, build_plan(0, 0, t, d), s);
        double *part = mem.alloc<double>(plan.ntiles * kPartials);
        int64_t *rot_dev = mem.alloc<int64_t>((int64_t)rot.size());
        h2d(rot_dev, rot.data(), (int64_t)rot.size(), s);
        rotate_pairs(v_dev, rot_dev, (int64_t)rot.size(), 0, s);
        pass_project(plan, dual != 0, ProjArgs{v_dev, d_dev, fp32proj}, part, s);
        rotate_pairs(v_dev, rot_dev, (int64_t)rot.size(), 0, s);
        PDCS_HIP(hipStreamSynchronize(s));
        check_grid(plan, s);
    });
}

pdcs_status pdcs_project(int64_t nblocks, const int32_t *types, const int64_t *dims, int dual,
                         const double *d_dev, double *v_dev, void *hip_stream) {
    return project_impl(nblocks, types, dims, dual, d_dev, v_dev, hip_stream, 0);
}

pdcs_status pdcs_project_fp32(int64_t nblocks, const int32_t *types, const int64_t *dims, int dual,
                              const double *d_dev, double *v_dev, void *hip_stream) {
    return project_impl(nblocks, types, dims, dual, d_dev, v_dev, hip_stream, 1);
}

}  // extern "C"

// Device scratch of pdcs_project_noalloc: the tile plan, the per-tile partial
// sums, the grid-level blocks' barrier state and the rotated blocks' offsets,
// carved per call.  Every GPU holds its own copy; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[PDCS_PROJECT_NOALLOC_SCRATCH_BYTES];

static void *scratch_address() {
    static std::mutex mu;
    static std::vector<void *> addr;   // per device ordinal, filled once each
    int dev = 0;
    PDCS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)addr.size() <= dev) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        PDCS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        addr[dev] = p;
    }
    return addr[dev];
}

// Bump placement of typed arrays in the scratch, 256-byte aligned.
struct ScratchCarve {
    uintptr_t base;
    size_t used = 0;
    template <class T>
    T *take(int64_t n) {
        T *p = reinterpret_cast<T *>(base + used);
        used += (sizeof(T) * (size_t)std::max<int64_t>(n, 1) + 255) & ~(size_t)255;
        return p;
    }
};

extern "C" {

pdcs_status pdcs_project_noalloc(int64_t nblocks, const int32_t *types, const int64_t *dims,
                                 int dual, const double *d_dev, double *v_dev, void *hip_stream) {
    return guarded([&] {
        if (nblocks < 0 || (nblocks > 0 && (!types || !dims || !v_dev)))
            fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        int64_t len = 0;
        for (int64_t b = 0; b < nblocks; ++b) len += dims[b];
        std::vector<int32_t> t;
        std::vector<int64_t> d;
        validate_cones(nblocks, types, dims, len, "cones", t, d);
        const std::vector<int64_t> rot = rsoc_to_soc(t, d, d_dev);
        const HostPlan H = build_plan(0, 0, t, d);
        const int64_t ntiles = (int64_t)H.tiles.size(), n_rot = (int64_t)rot.size();
        // sizes first (the carve only adds offsets to a null base here)
        ScratchCarve probe{0};
        probe.take<Tile>(ntiles);
        probe.take<int64_t>((int64_t)H.soc_off.size());
        probe.take<int32_t>((int64_t)H.soc_dim.size());
        probe.take<int64_t>((int64_t)H.exp_off.size());
        probe.take<unsigned long long>(H.n_grid);
        probe.take<double>(H.n_grid * 2 * kSocGridMaxParts * kSocGridSlot);
        probe.take<int>(1);
        probe.take<double>(ntiles * kPartials);
        probe.take<int64_t>(n_rot);
        if (probe.used > (size_t)PDCS_PROJECT_NOALLOC_SCRATCH_BYTES)
            fail(PDCS_ERR_NOT_SUPPORTED,
                 "pdcs_project_noalloc: this cone list needs " + std::to_string(probe.used) +
                     " bytes of device scratch, more than its fixed " +
                     std::to_string((size_t)PDCS_PROJECT_NOALLOC_SCRATCH_BYTES) +
                     " bytes; use pdcs_project or pdcs_cones_create");
        if (ntiles == 0) return;
        hipStream_t s = (hipStream_t)hip_stream;
        ScratchCarve c{reinterpret_cast<uintptr_t>(scratch_address())};
        ConePlan P;
        P.ntiles = ntiles;
        P.tiles = c.take<Tile>(ntiles);
        P.soc_off = c.take<int64_t>((int64_t)H.soc_off.size());
        P.soc_dim = c.take<int32_t>((int64_t)H.soc_dim.size());
        P.exp_off = c.take<int64_t>((int64_t)H.exp_off.size());
        P.n_soc = (int64_t)H.soc_off.size();
        P.n_exp = (int64_t)H.exp_off.size();
        P.n_grid = H.n_grid;
        P.grid_ctr = c.take<unsigned long long>(P.n_grid);
        P.grid_part = c.take<double>(P.n_grid * 2 * kSocGridMaxParts * kSocGridSlot);
        P.grid_err = c.take<int>(1);
        double *part = c.take<double>(ntiles * kPartials);
        int64_t *rot_dev = c.take<int64_t>(n_rot);
        h2d(P.tiles, H.tiles.data(), ntiles, s);
        h2d(P.soc_off, H.soc_off.data(), P.n_soc, s);
        h2d(P.soc_dim, H.soc_dim.data(), P.n_soc, s);
        h2d(P.exp_off, H.exp_off.data(), P.n_exp, s);
        h2d(rot_dev, rot.data(), n_rot, s);
        // the barrier counters must start at zero; a kernel clears them (the
        // scratch keeps whatever the last call on this GPU left)
        clear_grid(P, s);
        rotate_pairs(v_dev, rot_dev, n_rot, 0, s);
        pass_project(P, dual != 0, ProjArgs{v_dev, d_dev, 0}, part, s);
        rotate_pairs(v_dev, rot_dev, n_rot, 0, s);
        PDCS_HIP(hipStreamSynchronize(s));   // also keeps the host plan alive for the copies
        check_grid(P, s);
    });
}

struct pdcs_cones {
    DevMem mem;
    ConePlan plan;
    double *part = nullptr;
    int64_t len = 0;
    int64_t n_rot = 0;          // rotated SOC blocks, projected as T P_SOC(T v)
    int64_t *rot = nullptr;     // [n_rot] their first entries
};

pdcs_status pdcs_cones_create(int64_t nblocks, const int32_t *types, const int64_t *dims,
                              void *hip_stream, pdcs_cones **out) {
    if (!out) {
        g_last_error = "out is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    return guarded([&] {
        if (nblocks < 0 || (nblocks > 0 && (!types || !dims))) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        int64_t len = 0;
        for (int64_t b = 0; b < nblocks; ++b) len += dims[b];
        std::vector<int32_t> t;
        std::vector<int64_t> d;
        validate_cones(nblocks, types, dims, len, "cones", t, d);
        const std::vector<int64_t> rot = rsoc_to_soc(t, d, nullptr);
        auto c = std::make_unique<pdcs_cones>();
        hipStream_t s = (hipStream_t)hip_stream;
        c->plan = upload_plan(c->mem, build_plan(0, 0, t, d), s);
        c->part = c->mem.alloc<double>(c->plan.ntiles * kPartials);
        c->len = len;
        c->n_rot = (int64_t)rot.size();
        c->rot = c->mem.alloc<int64_t>(c->n_rot);
        h2d(c->rot, rot.data(), c->n_rot, s);
        PDCS_HIP(hipStreamSynchronize(s));
        *out = c.release();
    });
}

pdcs_status pdcs_cones_project(pdcs_cones *c, int dual, const double *d_dev, double *v_dev,
                               void *hip_stream) {
    return guarded([&] {
        if (!c || (c->len > 0 && !v_dev)) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        if (c->n_rot > 0 && d_dev) fail(PDCS_ERR_NOT_SUPPORTED, "rotated SOC blocks are projected with D = I");
        hipStream_t s = (hipStream_t)hip_stream;
        clear_grid(c->plan, s);   // an earlier call that timed out leaves the counters out of step
        rotate_pairs(v_dev, c->rot, c->n_rot, 0, s);
        pass_project(c->plan, dual != 0, ProjArgs{v_dev, d_dev}, c->part, s);
        rotate_pairs(v_dev, c->rot, c->n_rot, 0, s);
    });
}

void pdcs_cones_destroy(pdcs_cones *c) { delete c; }

pdcs_status pdcs_batch_create(const pdcs_problem_desc *descs, int64_t count, void *hip_stream,
                              pdcs_batch **out) {
    if (!out) {
        g_last_error = "out is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    return guarded([&] {
        std::unique_ptr<pdcs_problem> p(create_impl(descs, count, hip_stream, false));
        *out = new pdcs_batch{p.release()};
    });
}

pdcs_status pdcs_batch_solve(pdcs_batch *b, const pdcs_settings *settings, const double *const *x0,
                             const double *const *y0, const double *omega0, double *const *x_out,
                             double *const *y_out, pdcs_info *infos) {
    return guarded([&] {
        if (!b || !b->p) fail(PDCS_ERR_INVALID_ARG, "batch is NULL");
        solve_caller(b->p, settings, x0, y0, omega0, x_out, y_out, infos, nullptr);
    });
}

int64_t pdcs_batch_size(const pdcs_batch *b) { return b && b->p ? b->p->B : 0; }

void pdcs_batch_destroy(pdcs_batch *b) {
    if (!b) return;
    if (b->p) {
        (void)hipStreamSynchronize(b->p->stream);
        delete b->p;
    }
    delete b;
}

pdcs_status pdcs_gemm_bf16(int ta, int tb, int64_t M, int64_t N, int64_t K, const uint16_t *a,
                           int64_t lda, const uint16_t *b, int64_t ldb, const float *bias, int relu,
                           float *c32, uint16_t *c16, int64_t ldc, void *hip_stream) {
    return guarded([&] {
        if (M < 0 || N < 0 || K < 0 || (M && N && K && (!a || !b)) || (!c32 && !c16))
            fail(PDCS_ERR_INVALID_ARG, "bad GEMM arguments");
        if (lda < (ta ? M : K) || ldb < (tb ? K : N) || ldc < N)
            fail(PDCS_ERR_INVALID_ARG, "leading dimension too small");
        gemm_bf16(ta, tb, M, N, K, a, lda, b, ldb, bias, relu, c32, c16, ldc, (hipStream_t)hip_stream);
    });
}

pdcs_status pdcs_mlp_create(int64_t in, int64_t hid, int64_t out, int64_t max_batch,
                            const float *params, void *hip_stream, pdcs_mlp **mlp) {
    if (!mlp) {
        g_last_error = "out is NULL";
        return PDCS_ERR_INVALID_ARG;
    }
    *mlp = nullptr;
    return guarded([&] {
        if (in < 1 || hid < 1 || out < 1 || max_batch < 1 || !params) fail(PDCS_ERR_INVALID_ARG, "bad sizes");
        auto M = std::make_unique<pdcs_mlp>();
        M->in = in, M->hid = hid, M->out = out, M->cap = max_batch;
        M->stream = (hipStream_t)hip_stream;
        M->off[0] = 0;
        M->off[1] = M->off[0] + hid * in;
        M->off[2] = M->off[1] + hid;
        M->off[3] = M->off[2] + hid * hid;
        M->off[4] = M->off[3] + hid;
        M->off[5] = M->off[4] + out * hid;
        M->np = M->off[5] + out;
        DevMem &D = M->mem;
        hipStream_t s = M->stream;
        M->p = D.alloc<float>(M->np), M->g = D.alloc<float>(M->np);
        M->m1 = D.alloc<float>(M->np), M->m2 = D.alloc<float>(M->np);
        M->p16 = D.alloc<uint16_t>(M->np);
        h2d(M->p, params, M->np, s);
        to_bf16(M->p, M->p16, M->np, s);
        PDCS_HIP(hipMemsetAsync(M->m1, 0, sizeof(float) * M->np, s));
        PDCS_HIP(hipMemsetAsync(M->m2, 0, sizeof(float) * M->np, s));
        const int64_t B = max_batch;
        M->xb = D.alloc<uint16_t>(B * in);
        M->h1 = D.alloc<float>(B * hid), M->h1b = D.alloc<uint16_t>(B * hid);
        M->h2 = D.alloc<float>(B * hid), M->h2b = D.alloc<uint16_t>(B * hid);
        M->o = D.alloc<float>(B * out);
        M->ldo = (out + 7) / 8 * 8;
        M->d32 = D.alloc<float>(B * std::max(out, hid));
        M->d16 = D.alloc<uint16_t>(B * std::max(M->ldo, hid));
        M->ta = D.alloc<uint16_t>(std::max(out, hid) * B);
        M->tb = D.alloc<uint16_t>(std::max(hid, in) * B);
        M->wt = D.alloc<uint16_t>(hid * std::max(M->ldo, hid));
        M->dh = D.alloc<float>(B * hid);
        M->ws_elems = 32 * B * hid;
        M->ws = D.alloc<float>(M->ws_elems);
        M->part = D.alloc<double>((B * std::max(out, hid) + 255) / 256);
        PDCS_HIP(hipStreamSynchronize(s));
        *mlp = M.release();
    });
}

int64_t pdcs_mlp_num_params(const pdcs_mlp *m) { return m ? m->np : 0; }

static void mlp_forward(pdcs_mlp *M, const float *theta, int64_t B, float *out) {
    hipStream_t s = M->stream;
    const int64_t in = M->in, hid = M->hid, O = M->out;
    if (!mlp_hidden(B, in, hid, theta, M->p16 + M->off[0], M->p + M->off[1], M->p16 + M->off[2],
                    M->p + M->off[3], M->xb, M->h1, M->h1b, M->h2, M->h2b, s)) {
        to_bf16(theta, M->xb, B * in, s);
        gemm_bf16(0, 1, B, hid, in, M->xb, in, M->p16 + M->off[0], in, M->p + M->off[1], 1, M->h1, M->h1b, hid, s);
        gemm_bf16(0, 1, B, hid, hid, M->h1b, hid, M->p16 + M->off[2], hid, M->p + M->off[3], 1, M->h2, M->h2b, hid, s);
    }
    gemm_bf16(0, 1, B, O, hid, M->h2b, hid, M->p16 + M->off[4], hid, M->p + M->off[5], 0, out, nullptr, O, s);
}

// Gradient of L = (1 / (2 B out)) sum (o - target)^2 into M->g; returns L.
static double mlp_gradient(pdcs_mlp *M, const float *theta, const float *target, int64_t B) {
    hipStream_t s = M->stream;
    const int64_t in = M->in, hid = M->hid, O = M->out;
    mlp_forward(M, theta, B, M->o);
    const int64_t n = B * O, nblk = (n + 255) / 256;
    const int64_t ldo = M->ldo;
    mse_grad(M->o, target, n, O, ldo, (float)(1.0 / (double)n), M->d32, M->d16, M->part, s);
    float *g = M->g;
    // Every GEMM reads both operands along k: transposed copies of the
    // activations (k = the batch) and of the weights (k = the output units).
    // layer 3: dW3 = dO^T H2, db3 = colsum(dO), dH2 = dO W3
    transpose_bf16(M->d16, B, O, ldo, M->ta, B, s);
    transpose_bf16(M->h2b, B, hid, hid, M->tb, B, s);
    gemm_bf16(0, 1, O, hid, B, M->ta, B, M->tb, B, nullptr, 0, g + M->off[4], nullptr, hid, s);
    colsum(M->d32, B, O, g + M->off[5], s);
    transpose_bf16(M->p16 + M->off[4], O, hid, hid, M->wt, ldo, s);
    if (!gemm_bf16_split(B, hid, O, M->d16, ldo, M->wt, ldo, nullptr, 0, M->dh, nullptr, hid, M->ws,
                         M->ws_elems, s))
        gemm_bf16(0, 1, B, hid, O, M->d16, ldo, M->wt, ldo, nullptr, 0, M->dh, nullptr, hid, s);
    // layer 2
    relu_back(M->dh, M->h2, B * hid, M->d32, M->d16, s);
    transpose_bf16(M->d16, B, hid, hid, M->ta, B, s);
    transpose_bf16(M->h1b, B, hid, hid, M->tb, B, s);
    gemm_bf16(0, 1, hid, hid, B, M->ta, B, M->tb, B, nullptr, 0, g + M->off[2], nullptr, hid, s);
    colsum(M->d32, B, hid, g + M->off[3], s);
    transpose_bf16(M->p16 + M->off[2], hid, hid, hid, M->wt, hid, s);
    gemm_bf16(0, 1, B, hid, hid, M->d16, hid, M->wt, hid, nullptr, 0, M->dh, nullptr, hid, s);
    // layer 1
    relu_back(M->dh, M->h1, B * hid, M->d32, M->d16, s);
    transpose_bf16(M->d16, B, hid, hid, M->ta, B, s);
    transpose_bf16(M->xb, B, in, in, M->tb, B, s);
    gemm_bf16(0, 1, hid, in, B, M->ta, B, M->tb, B, nullptr, 0, g + M->off[0], nullptr, in, s);
    colsum(M->d32, B, hid, g + M->off[1], s);
    std::vector<double> part(nblk);
    d2h(part.data(), M->part, nblk, s);
    PDCS_HIP(hipStreamSynchronize(s));
    double loss = 0.0;
    for (double v : part) loss += v;
    return loss / (2.0 * (double)n);
}

pdcs_status pdcs_mlp_forward(pdcs_mlp *m, const float *theta_dev, int64_t batch, float *out_dev) {
    return guarded([&] {
        if (!m || !theta_dev || !out_dev || batch < 1 || batch > m->cap) fail(PDCS_ERR_INVALID_ARG, "bad arguments");
        mlp_forward(m, theta_dev, batch, out_dev);
    });
}

pdcs_status pdcs_mlp_gradient(pdcs_mlp *m, const float *theta_dev, const float *target_dev,
                              int64_t batch, float *grad_host, double *loss) {
    return guarded([&] {
        if (!m || !theta_dev || !target_dev || batch < 1 || batch > m->cap) fail(PDCS_ERR_INVALID_ARG, "bad arguments");
        const double l = mlp_gradient(m, theta_dev, target_dev, batch);
        if (loss) *loss = l;
        if (grad_host) {
            d2h(grad_host, m->g, m->np, m->stream);
            PDCS_HIP(hipStreamSynchronize(m->stream));
        }
    });
}

pdcs_status pdcs_mlp_train_step(pdcs_mlp *m, const float *theta_dev, const float *target_dev,
                                int64_t batch, float lr, double *loss) {
    return guarded([&] {
        if (!m || !theta_dev || !target_dev || batch < 1 || batch > m->cap || !(lr > 0.0f))
            fail(PDCS_ERR_INVALID_ARG, "bad arguments");
        const double l = mlp_gradient(m, theta_dev, target_dev, batch);
        if (loss) *loss = l;
        m->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, (float)m->step), c2 = 1.0f - std::pow(b2, (float)m->step);
        adam(m->p, m->g, m->m1, m->m2, m->np, lr, b1, b2, 1e-8f, c1, c2, m->p16, m->stream);
    });
}

pdcs_status pdcs_mlp_get_params(const pdcs_mlp *m, float *params_host) {
    return guarded([&] {
        if (!m || !params_host) fail(PDCS_ERR_INVALID_ARG, "NULL argument");
        d2h(params_host, m->p, m->np, m->stream);
        PDCS_HIP(hipStreamSynchronize(m->stream));
    });
}

void pdcs_mlp_destroy(pdcs_mlp *m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    delete m;
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
