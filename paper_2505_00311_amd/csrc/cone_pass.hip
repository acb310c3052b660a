// cone_pass.hip -- one launch projects a whole vector onto a product of cones
// (eq. (6)) and fuses what the solver does around the projection: the primal
// and dual updates of eq. (5) with their step-size reductions, the projection
// of restart candidates, and the termination measures of eq.
// (PDCS_terminate_tolerance).
//
// Each workgroup reads one tile of the side's cone plan: a run of elementwise
// entries (box / zero / free / nonnegative, thread per entry), SOC blocks of
// one size class (an aligned group of 8, 16, 32 or 64 lanes per block, up to
// 256 entries), one larger SOC block (whole workgroup), or up to 64
// exponential cones (one thread each) -- the thread-, block- and grid-level
// strategies of Section 4 mapped to CDNA wavefronts.
#include "cones_device.hpp"

namespace pdcs {

__device__ __forceinline__ int dual_kind(int k) {
    switch (k) {
    case kTileZero: return kTileFree;
    case kTileFree: return kTileZero;
    case kTileExp: return kTileExpDual;
    case kTileExpDual: return kTileExp;
    default: return k;
    }
}

// ---------------------------------------------------------------- ops
// An op supplies: skip(), load(j) -> value before projection, scale(j) ->
// diagonal of D (1 when unscaled), box(j, v) -> projection of a box entry,
// store(j, v, p, acc) / store_box(...), and scratch() for the workgroup SOC path.
// kWarm: the op runs once per step attempt on slowly changing inputs, so the
// roots of the SOC and exponential cases are kept per block between launches
// and start the next root search.

struct OpPrimal {  // x^ = Proj_X(x - tau (c~ - G~^T y)), acc.s0 += (x^ - x)^2
    static constexpr bool kWarm = true;
    PrimalArgs a;
    double tau;
    const DevState *st;
    __device__ void begin(int inst) {
        st = a.st + inst;
        tau = st->tau;
    }
    __device__ bool skip() const { return st->halt != 0; }
    __device__ double load(int64_t j) const { return a.x[j] - tau * (a.cs[j] - a.aty[j]); }
    __device__ double scale(int64_t j) const { return a.dx[j]; }
    __device__ double box(int64_t j, double v) const { return fmin(fmax(v, a.ls[j]), a.us[j]); }
    __device__ void store(int64_t j, double, double p, Acc &acc) const {
        a.xh[j] = p;
        if (a.xh32) a.xh32[j] = (float)p;
        const double d = p - a.x[j];
        acc.s[0] += d * d;
    }
    __device__ void store_box(int64_t j, double v, double p, Acc &acc) const { store(j, v, p, acc); }
    __device__ double *scratch() const { return a.xh; }
};

struct OpDual {  // y^ = Proj_Y(y + sigma (h~ - 2 G~x^ + G~x)), acc: |dy|^2, <dy, G~dx>
    static constexpr bool kWarm = true;
    DualArgs a;
    double sigma;
    const DevState *st;
    __device__ void begin(int inst) {
        st = a.st + inst;
        sigma = st->sigma;
    }
    __device__ bool skip() const { return st->halt != 0; }
    // G~x^ at row i (finished here when the product left its last sums);
    // load and store of a row run on the same thread
    __device__ double gxh(int64_t i) const { return a.gt.active() ? a.gt.value(a.gxh, i) : a.gxh[i]; }
    __device__ double load(int64_t i) const {
        const double g = gxh(i);
        if (a.gt.active()) a.gxh_out[i] = g;
        return a.y[i] + sigma * (a.hs[i] - 2.0 * g + a.gx[i]);
    }
    __device__ double scale(int64_t i) const { return a.dy[i]; }
    __device__ double box(int64_t, double v) const { return v; }
    __device__ void store(int64_t i, double, double p, Acc &acc) const {
        a.yh[i] = p;
        if (a.yh32) a.yh32[i] = (float)p;
        const double d = p - a.y[i];
        acc.s[0] += d * d;
        acc.s[1] += d * (gxh(i) - a.gx[i]);
    }
    __device__ void store_box(int64_t i, double v, double p, Acc &acc) const { store(i, v, p, acc); }
    __device__ double *scratch() const { return a.yh; }
};

struct OpCand {  // dst = Proj(src / div), div = 1 or the sum of step weights
    static constexpr bool kWarm = false;
    CandArgs a;
    double div;
    __device__ void begin(int inst) { div = a.use_avg ? a.st[inst].eta_sum : 1.0; }
    __device__ bool skip() const { return false; }
    __device__ double load(int64_t j) const { return a.use_avg ? a.src[j] / div : a.src[j]; }
    __device__ double scale(int64_t j) const { return a.d[j]; }
    __device__ double box(int64_t j, double v) const { return fmin(fmax(v, a.ls[j]), a.us[j]); }
    __device__ void store(int64_t j, double, double p, Acc &) const { a.dst[j] = p; }
    __device__ void store_box(int64_t j, double v, double p, Acc &acc) const { store(j, v, p, acc); }
    __device__ double *scratch() const { return a.dst; }
};

// rows of eq. (PDCS_terminate_tolerance): r = G x - h (unscaled), P(r) onto K_d^*
struct OpKktRows {
    static constexpr bool kWarm = false;
    KktRowsArgs a;
    __device__ void begin(int) {}
    __device__ bool skip() const { return false; }
    __device__ double load(int64_t i) const { return a.gxc[i] / a.e[i] - a.h[i]; }
    __device__ double scale(int64_t) const { return 1.0; }
    __device__ double box(int64_t, double v) const { return v; }
    __device__ void store(int64_t i, double r, double p, Acc &acc) const {
        acc.mx[0] = fmax(acc.mx[0], fabs(r - p));
        acc.mx[1] = fmax(acc.mx[1], fabs(a.gxc[i] / a.e[i]));
        acc.mx[2] = fmax(acc.mx[2], fabs(p));
        acc.s[0] += (a.e[i] * a.yc[i]) * a.h[i];
        const double d = a.yc[i] - a.ya[i];
        acc.s[1] += d * d;
    }
    __device__ void store_box(int64_t i, double v, double p, Acc &acc) const { store(i, v, p, acc); }
    __device__ double *scratch() const { return a.tmp; }
};

// columns: lambda = c - G^T y (unscaled); box entries measured against Lambda
// of eq. (defn_Lambda1), cone entries against K_p^*
struct OpKktCols {
    static constexpr bool kWarm = false;
    KktColsArgs a;
    __device__ void begin(int) {}
    __device__ bool skip() const { return false; }
    __device__ double load(int64_t j) const { return a.c[j] - a.atyc[j] / a.f[j]; }
    __device__ double scale(int64_t) const { return 1.0; }
    __device__ double box(int64_t j, double lam) const {
        const bool lf = isfinite(a.l[j]), uf = isfinite(a.u[j]);
        if (!lf && !uf) return 0.0;
        if (!lf) return lam < 0.0 ? lam : 0.0;
        if (!uf) return lam > 0.0 ? lam : 0.0;
        return lam;
    }
    __device__ void common(int64_t j, double lam, double p, Acc &acc) const {
        acc.mx[0] = fmax(acc.mx[0], fabs(lam - p));
        acc.mx[1] = fmax(acc.mx[1], fabs(a.atyc[j] / a.f[j]));
        acc.s[0] += a.c[j] * (a.f[j] * a.xc[j]);
        const double d = a.xc[j] - a.xa[j];
        acc.s[2] += d * d;
    }
    __device__ void store(int64_t j, double lam, double p, Acc &acc) const { common(j, lam, p, acc); }
    __device__ void store_box(int64_t j, double lam, double p, Acc &acc) const {
        common(j, lam, p, acc);
        if (p > 0.0) acc.s[1] += a.l[j] * p;
        if (p < 0.0) acc.s[1] -= a.u[j] * (-p);
    }
    __device__ double *scratch() const { return a.tmp; }
};

struct OpProject {
    static constexpr bool kWarm = false;
    ProjArgs a;
    __device__ void begin(int) {}
    __device__ bool skip() const { return false; }
    __device__ double load(int64_t j) const { return a.v[j]; }
    __device__ double scale(int64_t j) const { return a.d ? a.d[j] : 1.0; }
    __device__ double box(int64_t, double v) const { return v; }
    __device__ void store(int64_t j, double, double p, Acc &) const { a.v[j] = p; }
    __device__ void store_box(int64_t j, double v, double p, Acc &acc) const { store(j, v, p, acc); }
    __device__ double *scratch() const { return a.v; }
};

// ------------------------------------------------- workgroup-per-SOC block
template <class Op>
__device__ void soc_block(Op &op, int64_t off, int dim, Acc &acc, double *root) {
    double *buf = op.scratch();
    const int tid = threadIdx.x;
    for (int e = tid; e < dim; e += kBlock) buf[off + e] = op.load(off + e);
    __syncthreads();
    const double t = buf[off];
    const double d0 = op.scale(off);
    double sums[3] = {0.0, 0.0, 0.0};
    for (int e = 1 + tid; e < dim; e += kBlock) {
        const double x = buf[off + e], dh = op.scale(off + e) / d0;
        sums[0] += (dh * x) * (dh * x);
        sums[1] += (x / dh) * (x / dh);
        sums[2] += x * x;
    }
    block_sum_all<3>(sums);
    const double nd = sqrt(sums[0]), ndi = sqrt(sums[1]), nx2 = sums[2];
    int cs;
    double s = 0.0;
    if (t <= 0.0 && nd <= -t) {
        cs = 1;
    } else if (ndi <= t) {
        cs = 2;
    } else if (t == 0.0) {
        cs = 3;
        double q2[1] = {0.0};
        for (int e = 1 + tid; e < dim; e += kBlock) {
            const double x = buf[off + e], dh = op.scale(off + e) / d0;
            const double q = x / (dh + 1.0 / dh);
            q2[0] += q * q;
        }
        block_sum_all<1>(q2);
        s = sqrt(q2[0]);
    } else {
        cs = 4;
        const double lo = t > 0.0 ? t : 0.0, hi = sqrt(t * t + nx2);
        double xpos = lo, xneg = hi;
        s = 0.5 * (t + sqrt(nx2));
        if (!(s > lo && s < hi)) s = 0.5 * (lo + hi);
        if (root) {
            const double g = *root;   // root of an earlier, nearby input
            if (g > lo && g < hi) s = g;
        }
        double dxold = hi - lo, dx = dxold;
        auto eval = [&](double ss, double &f, double &df) {
            const double a = 1.0 - t / ss;
            double g[2] = {0.0, 0.0};
            for (int e = 1 + tid; e < dim; e += kBlock) {
                const double x = buf[off + e], dh = op.scale(off + e) / d0;
                const double xd = x * dh;
                const double iq = 1.0 / (dh * dh + a);
                const double u = xd * xd * iq * iq;
                g[0] += u;
                g[1] += u * iq;
            }
            block_sum_all<2>(g);
            f = g[0] - ss * ss;
            df = -2.0 * (t / (ss * ss)) * g[1] - 2.0 * ss;
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
                dx = f / df;
                s -= dx;
            }
            if (fabs(dx) <= 4.0 * kEps * s) break;
            eval(s, f, df);
        }
    }
    __syncthreads();  // every thread has read buf[off] (t) and *root before they change
    if (root && cs == 4 && tid == 0) *root = s;
    const double a = 1.0 - t / s;
    for (int e = tid; e < dim; e += kBlock) {
        const int64_t j = off + e;
        const double v = buf[j];
        double p;
        if (cs == 1) {
            p = 0.0;
        } else if (cs == 2) {
            p = v;
        } else if (e == 0) {
            p = s;
        } else {
            const double dh = op.scale(j) / d0;
            p = cs == 3 ? v / (1.0 + 1.0 / (dh * dh)) : v / (1.0 + a / (dh * dh));
        }
        op.store(j, v, p, acc);
    }
}

// --------------------------------------- lane-group-per-SOC block (dim <= 256)
template <class Op, int LPB, int R>
__device__ __forceinline__ void soc_tile(Op &op, const Tile &tl, const int64_t *__restrict__ soc_off,
                                         const int32_t *__restrict__ soc_dim, double *soc_root,
                                         Acc &acc) {
    const int gi = threadIdx.x / LPB, g = threadIdx.x % LPB;
    if (gi >= tl.count) return;
    const int64_t b = tl.start + gi;
    const int64_t off = soc_off[b];
    const int dim = soc_dim[b];
    double v[R], d[R], p[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = g + LPB * r;
        v[r] = e < dim ? op.load(off + e) : 0.0;
        d[r] = e < dim ? op.scale(off + e) : 1.0;
    }
    double s_new;
    soc_project_group<LPB, R>(dim, v, d, p, soc_root ? soc_root[b] : __builtin_nan(""), s_new);
    if (soc_root && g == 0 && s_new == s_new) soc_root[b] = s_new;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = g + LPB * r;
        if (e < dim) op.store(off + e, v[r], p[r], acc);
    }
}

// ------------------------------------------------------------------ kernel
template <class Op, bool DUAL>
__global__ __launch_bounds__(kBlock) void cone_pass_kernel(Op op, const Tile *__restrict__ tiles,
                                                           const int64_t *__restrict__ soc_off,
                                                           const int32_t *__restrict__ soc_dim,
                                                           const int64_t *__restrict__ exp_off,
                                                           double *__restrict__ partials,
                                                           double *__restrict__ soc_root,
                                                           double *__restrict__ exp_root) {
    const Tile tl = tiles[blockIdx.x];
    op.begin(tl.inst);
    if (op.skip()) return;
    const int kind = DUAL ? dual_kind(tl.kind) : tl.kind;
    const int tid = threadIdx.x;
    Acc acc;
    switch (kind) {
    case kTileBox:
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store_box(j, v, op.box(j, v), acc);
        }
        break;
    case kTileZero:
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store(j, v, 0.0, acc);
        }
        break;
    case kTileFree:
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store(j, v, v, acc);
        }
        break;
    case kTileNonneg:
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store(j, v, v > 0.0 ? v : 0.0, acc);
        }
        break;
    case kTileSoc8: soc_tile<Op, 8, 1>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc16: soc_tile<Op, 16, 1>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc32: soc_tile<Op, 32, 1>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc64: soc_tile<Op, 64, 1>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc128: soc_tile<Op, 64, 2>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc256: soc_tile<Op, 64, 4>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSocBlock:
        soc_block(op, soc_off[tl.start], soc_dim[tl.start], acc,
                  soc_root ? soc_root + tl.start : nullptr);
        break;
    case kTileExp:
    case kTileExpDual:
        if (tid < tl.count) {
            const int64_t off = exp_off[tl.start + tid];
            const double r0 = op.load(off), s0 = op.load(off + 1), t0 = op.load(off + 2);
            const double dr = op.scale(off), ds = op.scale(off + 1), dt = op.scale(off + 2);
            double pr, ps, pt, rho;
            const double guess = exp_root ? exp_root[tl.start + tid] : __builtin_nan("");
            if (kind == kTileExp)
                exp_project(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho);
            else
                exp_dual_project(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho);
            if (exp_root && rho == rho) exp_root[tl.start + tid] = rho;
            op.store(off, r0, pr, acc);
            op.store(off + 1, s0, ps, acc);
            op.store(off + 2, t0, pt, acc);
        }
        break;
    }
    write_partials(acc, partials, blockIdx.x);
}

template <class Op, bool DUAL>
static void launch(const ConePlan &p, const Op &op, double *partials, hipStream_t s) {
    if (p.ntiles == 0) return;
    hipLaunchKernelGGL((cone_pass_kernel<Op, DUAL>), dim3((unsigned)p.ntiles), dim3(kBlock), 0, s,
                       op, p.tiles, p.soc_off, p.soc_dim, p.exp_off, partials,
                       Op::kWarm ? p.soc_root : nullptr, Op::kWarm ? p.exp_root : nullptr);
    PDCS_HIP(hipGetLastError());
}

void pass_primal(const ConePlan &p, const PrimalArgs &a, double *partials, hipStream_t s) {
    launch<OpPrimal, false>(p, OpPrimal{a, 0.0}, partials, s);
}
void pass_dual(const ConePlan &p, const DualArgs &a, double *partials, hipStream_t s) {
    launch<OpDual, true>(p, OpDual{a, 0.0}, partials, s);
}
void pass_candidate(const ConePlan &p, bool y_side, const CandArgs &a, double *partials,
                    hipStream_t s) {
    if (y_side)
        launch<OpCand, true>(p, OpCand{a, 1.0}, partials, s);
    else
        launch<OpCand, false>(p, OpCand{a, 1.0}, partials, s);
}
void pass_kkt_rows(const ConePlan &p, const KktRowsArgs &a, double *partials, hipStream_t s) {
    launch<OpKktRows, false>(p, OpKktRows{a}, partials, s);
}
void pass_kkt_cols(const ConePlan &p, const KktColsArgs &a, double *partials, hipStream_t s) {
    launch<OpKktCols, true>(p, OpKktCols{a}, partials, s);
}
void pass_project(const ConePlan &p, bool dual, const ProjArgs &a, double *partials,
                  hipStream_t s) {
    if (dual)
        launch<OpProject, true>(p, OpProject{a}, partials, s);
    else
        launch<OpProject, false>(p, OpProject{a}, partials, s);
}

}  // namespace pdcs
