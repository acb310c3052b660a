// cone_pass.hip -- one launch projects a whole vector onto a product of cones
// (eq. (6)) and fuses what the solver does around the projection: the primal
// and dual updates of eq. (5) with their step-size reductions, the projection
// of restart candidates, and the termination measures of eq.
// (PDCS_terminate_tolerance).
//
// Each workgroup reads one tile of the side's cone plan: a run of elementwise
// entries (box / zero / free / nonnegative, thread per entry), SOC blocks of
// one size class (an aligned group of 8, 16, 32 or 64 lanes per block, up to
// 256 entries), one larger SOC block (whole workgroup), or up to 256
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

// Projection of one elementwise entry of kind k (box: [lo, hi]).
__device__ __forceinline__ double elem_proj(int k, double v, double lo, double hi) {
    switch (k) {
    case kTileBox: return fmin(fmax(v, lo), hi);
    case kTileZero: return 0.0;
    case kTileFree: return v;
    default: return v > 0.0 ? v : 0.0;
    }
}

// Elementwise tiles of the two step passes.  A thread's entries are taken
// kElemRound at a time with all of their loads issued first (clamped indices;
// the arrays are restrict-qualified so that the compiler may move loads ahead
// of the previous entries' stores), then projected and stored in entry order,
// so the partial sums are those of the one-entry-at-a-time loop.
constexpr int kElemRound = 4;

__device__ __forceinline__ void primal_elem(int kind, int64_t start, int64_t end, double tau,
                                            const double *__restrict__ x,
                                            const double *__restrict__ cs,
                                            const double *__restrict__ aty,
                                            const double *__restrict__ ls,
                                            const double *__restrict__ us,
                                            double *__restrict__ xh, float *__restrict__ xh32,
                                            Acc &acc) {
    constexpr int U = kElemRound;
    const bool box = kind == kTileBox;
    for (int64_t j0 = start + threadIdx.x; j0 < end; j0 += U * kBlock) {
        double xv[U], cv[U], av[U], lv[U], uv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = min(j0 + (int64_t)u * kBlock, end - 1);
            xv[u] = x[j], cv[u] = cs[j], av[u] = aty[j];
            lv[u] = box ? ls[j] : 0.0;
            uv[u] = box ? us[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + (int64_t)u * kBlock;
            if (j >= end) break;
            const double p = elem_proj(kind, xv[u] - tau * (cv[u] - av[u]), lv[u], uv[u]);
            xh[j] = p;
            if (xh32) xh32[j] = (float)p;
            const double d = p - xv[u];
            acc.s[0] += d * d;
        }
    }
}

__device__ __forceinline__ void dual_elem(int kind, int64_t start, int64_t end, double sigma,
                                          const ProductTail &gt, const double *__restrict__ y,
                                          const double *__restrict__ gxh_in,
                                          const double *__restrict__ gx,
                                          const double *__restrict__ hs,
                                          double *__restrict__ yh, float *__restrict__ yh32,
                                          double *__restrict__ gxh_out, Acc &acc) {
    constexpr int U = kElemRound;
    const bool tail = gt.active();
    for (int64_t i0 = start + threadIdx.x; i0 < end; i0 += U * kBlock) {
        double yv[U], gv[U], xv[U], hv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = min(i0 + (int64_t)u * kBlock, end - 1);
            yv[u] = y[i], xv[u] = gx[i], hv[u] = hs[i];
            gv[u] = tail ? gt.value(gxh_in, i) : gxh_in[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            if (i >= end) break;
            const double p = elem_proj(kind, yv[u] + sigma * (hv[u] - 2.0 * gv[u] + xv[u]), 0.0, 0.0);
            if (tail) gxh_out[i] = gv[u];
            yh[i] = p;
            if (yh32) yh32[i] = (float)p;
            const double d = p - yv[u];
            acc.s[0] += d * d;
            acc.s[1] += d * (gv[u] - xv[u]);
        }
    }
}

// What a load hands to the store of the same entry: the value before the
// projection (v) and, for the step passes, the inputs the store needs again
// (so the store does not re-read them after the writes of earlier entries,
// which the compiler cannot reorder and each of which waits a memory latency).
struct Ld {
    double v, u, w, z;
};

// ---------------------------------------------------------------- ops
// An op supplies: skip(), load(j) -> value before projection, scale(j) ->
// diagonal of D (1 when unscaled), box(j, v) -> projection of a box entry,
// store(j, v, p, acc) / store_box(...), and scratch() for the workgroup SOC path.
// kWarm: the op runs once per step attempt on slowly changing inputs, so the
// roots of the SOC and exponential cases are kept per block between launches
// and start the next root search.
// kUnit: D = I is known when the kernel is built (scale(j) is the constant 1),
// and the SOC blocks take the closed form of that case.
// kInPlace: load(j) returns scratch()[j] unchanged, so the workgroup SOC path
// reads its input where it lies instead of copying it to the scratch first.

struct OpPrimal {  // x^ = Proj_X(x - tau (c~ - G~^T y)), acc.s0 += (x^ - x)^2
    static constexpr bool kWarm = true;
    static constexpr bool kUnit = false;
    static constexpr bool kInPlace = false;
    PrimalArgs a;
    double tau;
    const DevState *st;
    __device__ void begin(int inst) {
        st = a.st + inst;
        tau = st->tau;
    }
    __host__ __device__ bool fp32() const { return a.fp32proj != 0; }
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
    // kCarry: elem() is the pipelined elementwise tile, load_ld/store_ld carry
    // x from the load to the store
    static constexpr bool kCarry = true;
    __device__ void elem(int kind, int64_t start, int64_t end, Acc &acc) const {
        primal_elem(kind, start, end, tau, a.x, a.cs, a.aty, a.ls, a.us, a.xh, a.xh32, acc);
    }
    __device__ Ld load_ld(int64_t j) const {
        const double x = a.x[j];
        return Ld{x - tau * (a.cs[j] - a.aty[j]), x, 0.0, 0.0};
    }
    __device__ void store_ld(int64_t j, const Ld &l, double p, Acc &acc) const {
        a.xh[j] = p;
        if (a.xh32) a.xh32[j] = (float)p;
        const double d = p - l.u;
        acc.s[0] += d * d;
    }
};

struct OpDual {  // y^ = Proj_Y(y + sigma (h~ - 2 G~x^ + G~x)), acc: |dy|^2, <dy, G~dx>
    static constexpr bool kWarm = true;
    static constexpr bool kUnit = false;
    static constexpr bool kInPlace = false;
    DualArgs a;
    double sigma;
    const DevState *st;
    __device__ void begin(int inst) {
        st = a.st + inst;
        sigma = st->sigma;
    }
    __host__ __device__ bool fp32() const { return a.fp32proj != 0; }
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
    static constexpr bool kCarry = true;
    __device__ void elem(int kind, int64_t start, int64_t end, Acc &acc) const {
        dual_elem(kind, start, end, sigma, a.gt, a.y, a.gxh, a.gx, a.hs, a.yh, a.yh32, a.gxh_out, acc);
    }
    // carries y, G~x^ and G~x; G~x^ is stored (when finished here) with y^
    __device__ Ld load_ld(int64_t i) const {
        const double y = a.y[i], g = gxh(i), gx = a.gx[i];
        return Ld{y + sigma * (a.hs[i] - 2.0 * g + gx), y, g, gx};
    }
    __device__ void store_ld(int64_t i, const Ld &l, double p, Acc &acc) const {
        if (a.gt.active()) a.gxh_out[i] = l.w;
        a.yh[i] = p;
        if (a.yh32) a.yh32[i] = (float)p;
        const double d = p - l.u;
        acc.s[0] += d * d;
        acc.s[1] += d * (l.w - l.z);
    }
};

struct OpCand {  // dst = Proj(src / div), div = 1 or the sum of step weights
    static constexpr bool kWarm = false;
    static constexpr bool kUnit = false;
    static constexpr bool kInPlace = false;
    static constexpr bool kCarry = false;
    CandArgs a;
    double div;
    __device__ void begin(int inst) { div = a.use_avg ? a.st[inst].eta_sum : 1.0; }
    __host__ __device__ bool fp32() const { return false; }
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
    static constexpr bool kUnit = false;
    static constexpr bool kInPlace = false;
    static constexpr bool kCarry = false;
    KktRowsArgs a;
    __device__ void begin(int) {}
    __host__ __device__ bool fp32() const { return false; }
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
    static constexpr bool kUnit = false;
    static constexpr bool kInPlace = false;
    static constexpr bool kCarry = false;
    KktColsArgs a;
    __device__ void begin(int) {}
    __host__ __device__ bool fp32() const { return false; }
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
    static constexpr bool kUnit = false;
    static constexpr bool kInPlace = true;
    static constexpr bool kCarry = false;
    ProjArgs a;
    __device__ void begin(int) {}
    __host__ __device__ bool fp32() const { return a.fp32proj != 0; }
    __device__ bool skip() const { return false; }
    __device__ double load(int64_t j) const { return a.v[j]; }
    __device__ double scale(int64_t j) const { return a.d ? a.d[j] : 1.0; }
    __device__ double box(int64_t, double v) const { return v; }
    __device__ void store(int64_t j, double, double p, Acc &) const { a.v[j] = p; }
    __device__ void store_box(int64_t j, double v, double p, Acc &acc) const { store(j, v, p, acc); }
    __device__ double *scratch() const { return a.v; }
};

// A projection call without scaling vector (d == nullptr).
struct OpProjectUnit : OpProject {
    static constexpr bool kUnit = true;
    __device__ double scale(int64_t) const { return 1.0; }
};

template <class Op>
__device__ __forceinline__ Ld load_ld(const Op &op, int64_t j) {
    if constexpr (Op::kCarry)
        return op.load_ld(j);
    else
        return Ld{op.load(j), 0.0, 0.0, 0.0};
}
template <class Op>
__device__ __forceinline__ void store_ld(const Op &op, int64_t j, const Ld &l, double p, Acc &acc) {
    if constexpr (Op::kCarry)
        op.store_ld(j, l, p, acc);
    else
        op.store(j, l.v, p, acc);
}

// ------------------------------------------------- workgroup-per-SOC block
// D = I: the equation of the root-finding case of Theorem 1 becomes
// ||x|| = 2s - t, so s = (t + ||x||)/2 and x is scaled by s/||x||.  One
// reduction (||x||^2 over entries [lo, hi) of the block) and one store pass;
// blocks inside the cone are left as they are.  Every part has read t before
// part 0 stores the new t: the reduction's barrier lies between the two.
template <class Op, class Red>
__device__ void soc_block_range_unit(Op &op, int64_t off, int lo, int hi, Acc &acc, Red &red) {
    static_assert(Op::kInPlace, "the closed form reads its input in place");
    // A thread takes its entries U at a time (kBlock apart) and issues the U
    // loads, predicated on the range, before it uses any of them, so that
    // enough bytes are in flight per workgroup.  When the range fits in one
    // such batch (at most U kBlock entries), the store pass reuses the values
    // the norm pass loaded instead of reading them again.
    constexpr int U = 8;
    const int tid = threadIdx.x;
    const bool one = hi - lo <= U * kBlock;
    const double t = op.load(off);
    double sq[1] = {0.0};
    double x[U];
    for (int64_t e = lo + tid; e < hi; e += U * kBlock) {
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = e + u * kBlock < hi ? op.load(off + e + u * kBlock) : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) sq[0] += e + u * kBlock == 0 ? 0.0 : x[u] * x[u];
    }
    red.sum(sq);
    const double nx = sqrt(sq[0]);
    if (nx <= t) return;                                  // case 2: inside
    const bool polar = t <= 0.0 && nx <= -t;              // case 1: polar -> 0
    const double s = polar ? 0.0 : 0.5 * (t + nx), c = polar ? 0.0 : s / nx;
    for (int64_t e = lo + tid; e < hi; e += U * kBlock) {
        if (!one) {
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = e + u * kBlock < hi ? op.load(off + e + u * kBlock) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t eu = e + u * kBlock;
            if (eu < hi) op.store(off + eu, x[u], eu == 0 ? s : x[u] * c, acc);
        }
    }
}

// The workgroup projects entries [lo, hi) of the block at `off` (the whole
// block for the workgroup class, one part for the grid class); every sum over
// the block goes through red.sum, which returns the block total to every
// thread.  The reductions over the block (read-only loops) are unrolled by 4
// so that a thread's loads of the scratch and scale vectors are issued
// together.
template <class Op, class Red>
__device__ void soc_block_range(Op &op, int64_t off, int dim, int lo, int hi, Acc &acc,
                                double *root, Red &red) {
    if constexpr (Op::kUnit) {
        soc_block_range_unit(op, off, lo, hi, acc, red);
        return;
    }
    double *buf = op.scratch();
    const int tid = threadIdx.x;
    if constexpr (!Op::kInPlace) {
        for (int e = lo + tid; e < hi; e += kBlock) buf[off + e] = op.load(off + e);
        __syncthreads();
    }
    const double t = lo == 0 ? buf[off] : op.load(off);
    const double d0 = op.scale(off);
    const int e0 = (lo == 0 ? 1 : lo) + tid;
    // With the root of an earlier, nearby input, the first root-finding
    // evaluation at it is summed in this same pass (the arithmetic of eval
    // below, one reduction fewer); it is used when that root is in bracket.
    // Only passes that keep roots (Op::kWarm) have one; the others reduce the
    // three norms alone.
    constexpr int K = Op::kWarm ? 5 : 3;
    const double g0 = root ? *root : 0.0;
    const bool fuse = K == 5 && g0 > 0.0 && isfinite(g0);
    const double a0 = fuse ? 1.0 - t / g0 : 0.0;
    double sums[K] = {};
#pragma unroll 4
    for (int e = e0; e < hi; e += kBlock) {
        const double x = buf[off + e], dh = op.scale(off + e) / d0;
        sums[0] += (dh * x) * (dh * x);
        sums[1] += (x / dh) * (x / dh);
        sums[2] += x * x;
        if constexpr (K == 5) {
            if (fuse) {
                const double xd = x * dh;
                const double iq = 1.0 / (dh * dh + a0);
                const double u = xd * xd * iq * iq;
                sums[3] += u;
                sums[4] += u * iq;
            }
        }
    }
    red.sum(sums);
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
#pragma unroll 4
        for (int e = e0; e < hi; e += kBlock) {
            const double x = buf[off + e], dh = op.scale(off + e) / d0;
            const double q = x / (dh + 1.0 / dh);
            q2[0] += q * q;
        }
        red.sum(q2);
        s = sqrt(q2[0]);
    } else {
        cs = 4;
        const double lo_s = t > 0.0 ? t : 0.0, hi_s = sqrt(t * t + nx2);
        double xpos = lo_s, xneg = hi_s;
        s = 0.5 * (t + sqrt(nx2));
        if (!(s > lo_s && s < hi_s)) s = 0.5 * (lo_s + hi_s);
        const bool warm = fuse && g0 > lo_s && g0 < hi_s;
        if (warm) s = g0;
        double dxold = hi_s - lo_s, dx = dxold;
        auto eval = [&](double ss, double &f, double &df) {
            const double a = 1.0 - t / ss;
            double g[2] = {0.0, 0.0};
#pragma unroll 4
            for (int e = e0; e < hi; e += kBlock) {
                const double x = buf[off + e], dh = op.scale(off + e) / d0;
                const double xd = x * dh;
                const double iq = 1.0 / (dh * dh + a);
                const double u = xd * xd * iq * iq;
                g[0] += u;
                g[1] += u * iq;
            }
            red.sum(g);
            f = g[0] - ss * ss;
            df = -2.0 * (t / (ss * ss)) * g[1] - 2.0 * ss;
        };
        double f, df;
        if constexpr (K == 5) {
            if (warm) {
                f = sums[3] - s * s;
                df = -2.0 * (t / (s * s)) * sums[4] - 2.0 * s;
            } else {
                eval(s, f, df);
            }
        } else {
            eval(s, f, df);
        }
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
    // every thread of every part has read buf[off] (t) and *root before they
    // change: the workgroup barrier here, and for the grid class the barrier
    // of the first reduction, which the other parts pass only after reading
    __syncthreads();
    if (root && cs == 4 && tid == 0 && lo == 0) *root = s;
    const double a = 1.0 - t / s;
    for (int e = lo + tid; e < hi; e += kBlock) {
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

struct BlockRed {
    template <int K>
    __device__ void sum(double (&v)[K]) { block_sum_all<K>(v); }
};

template <class Op>
__device__ void soc_block(Op &op, int64_t off, int dim, Acc &acc, double *root) {
    BlockRed red;
    soc_block_range(op, off, dim, 0, dim, acc, root, red);
}

// ------------------------------------ grid level: several workgroups per block
// The grid-level strategy of Section 4 for the largest SOC blocks, inside the
// pass launch: a block of dim >= kSocGridMin is cut into G parts of
// consecutive entries, one workgroup each.  Each sum over the block becomes: block sums per part,
// written to the part's slot; a barrier of the G workgroups; then every part
// adds the G slots in part order, so all parts hold the same bits and take
// the same decisions.  The slots alternate between two rounds: a part writes
// round r + 2 only after the barrier of round r + 1, which every part passes
// only after reading round r.
struct GridSync {
    unsigned long long *ctr;
    double *part;
    int *err;
};

// about one second of the 100 MHz wall clock
constexpr long long kGridWaitTicks = 100000000;

// Barrier of the G workgroups of one block.  The counter only grows: the
// arrivals of a round are the next G values, so the round is complete when
// the counter reaches the next multiple of G.  A wait past kGridWaitTicks (a
// part that never arrives) sets the error flag and returns false; the caller
// then stops waiting.
__device__ bool grid_barrier(unsigned long long *ctr, int G, int *err) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // this part's slot before its arrival
        const unsigned long long a = atomicAdd(ctr, 1ull);
        const unsigned long long target = (a / (unsigned long long)G + 1ull) * (unsigned long long)G;
        const long long t0 = wall_clock64();
        int good = 1;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (wall_clock64() - t0 > kGridWaitTicks) {
                atomicOr(err, 1);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();   // the other parts' slots after their arrivals
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

struct GridRed {
    GridSync g;
    int slot, part, parts, round;
    bool ok;
    template <int K>
    __device__ void sum(double (&v)[K]) {
        static_assert(K <= kSocGridSlot, "a reduction round holds kSocGridSlot values per part");
        block_sum_all<K>(v);
        double *buf = g.part + ((int64_t)slot * 2 + (round & 1)) * (kSocGridMaxParts * kSocGridSlot);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                __hip_atomic_store(buf + part * kSocGridSlot + k, v[k], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (ok) ok = grid_barrier(g.ctr + slot, parts, g.err);
        // thread t adds the slots of parts t, t + kBlock, ... in order, then the
        // workgroup sums those in a fixed order: every part forms the same bits
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = 0.0;
        for (int q = threadIdx.x; q < parts; q += kBlock)
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[k] += __hip_atomic_load(buf + q * kSocGridSlot + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        block_sum_all<K>(v);
        ++round;
    }
};

template <class Op>
__device__ void soc_grid_part(Op &op, const Tile &tl, const int64_t *__restrict__ soc_off,
                              const int32_t *__restrict__ soc_dim, double *soc_root,
                              const GridSync &gs, Acc &acc) {
    const int part = tl.count % kSocGridPartCode, parts = tl.count / kSocGridPartCode;
    const int64_t b = tl.start;
    const int dim = soc_dim[b];
    const int chunk = (dim + parts - 1) / parts;
    const int lo = part * chunk, hi = lo + chunk < dim ? lo + chunk : dim;
    // after a timed-out barrier anywhere, no part waits again
    const bool ok = __hip_atomic_load(gs.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    GridRed red{gs, tl.pad, part, parts, 0, ok};
    soc_block_range(op, soc_off[b], dim, lo, hi, acc, soc_root ? soc_root + b : nullptr, red);
}

// --------------------------------------- lane-group-per-SOC block (dim <= 256)
template <class Op, int LPB, int R, bool F32>
__device__ __forceinline__ void soc_tile(Op &op, const Tile &tl, const int64_t *__restrict__ soc_off,
                                         const int32_t *__restrict__ soc_dim, double *soc_root,
                                         Acc &acc) {
    const int gi = threadIdx.x / LPB, g = threadIdx.x % LPB;
    if (gi >= tl.count) return;
    const int64_t b = tl.start + gi;
    const int64_t off = soc_off[b];
    const int dim = soc_dim[b];
    const double guess = soc_root ? soc_root[b] : __builtin_nan("");
    // loads at clamped indices, unconditional, so none waits behind a branch
    Ld l[R];
    double v[R], d[R], p[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = g + LPB * r;
        const int64_t j = off + (e < dim ? e : dim - 1);
        l[r] = load_ld(op, j);
        d[r] = op.scale(j);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool on = g + LPB * r < dim;
        v[r] = on ? l[r].v : 0.0;
        d[r] = on ? d[r] : 1.0;
    }
    double s_new;
    if constexpr (Op::kUnit)
        soc_project_group_unit<LPB, R>(dim, v, p, s_new);
    else if constexpr (F32)
        soc_project_group_f<LPB, R>(dim, v, d, p, guess, s_new);
    else
        soc_project_group<LPB, R>(dim, v, d, p, guess, s_new);
    if (soc_root && g == 0 && s_new == s_new) soc_root[b] = s_new;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = g + LPB * r;
        if (e < dim) store_ld(op, off + e, l[r], p[r], acc);
    }
}

// ------------------------------------------------------------------ kernel
// F32: the lane-group SOC and exponential projections in FP32 (the mixed
// form's; a kernel of its own so the FP64 kernels keep their registers).
template <class Op, bool DUAL, bool F32>
__global__ __launch_bounds__(kBlock) void cone_pass_kernel(Op op, const Tile *__restrict__ tiles,
                                                           const int64_t *__restrict__ soc_off,
                                                           const int32_t *__restrict__ soc_dim,
                                                           const int64_t *__restrict__ exp_off,
                                                           double *__restrict__ partials,
                                                           double *__restrict__ soc_root,
                                                           double *__restrict__ exp_root,
                                                           GridSync gs) {
    const Tile tl = tiles[blockIdx.x];
    op.begin(tl.inst);
    if (op.skip()) return;
    const int kind = DUAL ? dual_kind(tl.kind) : tl.kind;
    const int tid = threadIdx.x;
    Acc acc;
    switch (kind) {
    case kTileBox:
        if constexpr (Op::kCarry) {
            op.elem(kind, tl.start, tl.start + tl.count, acc);
            break;
        }
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store_box(j, v, op.box(j, v), acc);
        }
        break;
    case kTileZero:
        if constexpr (Op::kCarry) {
            op.elem(kind, tl.start, tl.start + tl.count, acc);
            break;
        }
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store(j, v, 0.0, acc);
        }
        break;
    case kTileFree:
        if constexpr (Op::kCarry) {
            op.elem(kind, tl.start, tl.start + tl.count, acc);
            break;
        }
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store(j, v, v, acc);
        }
        break;
    case kTileNonneg:
        if constexpr (Op::kCarry) {
            op.elem(kind, tl.start, tl.start + tl.count, acc);
            break;
        }
        for (int64_t j = tl.start + tid; j < tl.start + tl.count; j += kBlock) {
            const double v = op.load(j);
            op.store(j, v, v > 0.0 ? v : 0.0, acc);
        }
        break;
    case kTileSoc8: soc_tile<Op, 8, 1, F32>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc16: soc_tile<Op, 16, 1, F32>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc32: soc_tile<Op, 16, 2, F32>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc64: soc_tile<Op, 16, 4, F32>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc128: soc_tile<Op, 32, 4, F32>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSoc256: soc_tile<Op, 64, 4, F32>(op, tl, soc_off, soc_dim, soc_root, acc); break;
    case kTileSocBlock:
        soc_block(op, soc_off[tl.start], soc_dim[tl.start], acc,
                  soc_root ? soc_root + tl.start : nullptr);
        break;
    case kTileSocGrid:
        soc_grid_part(op, tl, soc_off, soc_dim, soc_root, gs, acc);
        break;
    case kTileExp:
    case kTileExpDual:
        if (tid < tl.count) {
            const int64_t off = exp_off[tl.start + tid];
            const Ld lr = load_ld(op, off), ls = load_ld(op, off + 1), lt = load_ld(op, off + 2);
            const double r0 = lr.v, s0 = ls.v, t0 = lt.v;
            const double dr = op.scale(off), ds = op.scale(off + 1), dt = op.scale(off + 2);
            double pr, ps, pt, rho;
            const double guess = exp_root ? exp_root[tl.start + tid] : __builtin_nan("");
            if constexpr (F32) {
                if (kind == kTileExp)
                    exp_project_f(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho);
                else
                    exp_dual_project_f(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho);
            } else if (kind == kTileExp) {
                exp_project(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho);
            } else {
                exp_dual_project(r0, s0, t0, dr, ds, dt, pr, ps, pt, guess, rho);
            }
            if (exp_root && rho == rho) exp_root[tl.start + tid] = rho;
            store_ld(op, off, lr, pr, acc);
            store_ld(op, off + 1, ls, ps, acc);
            store_ld(op, off + 2, lt, pt, acc);
        }
        break;
    }
    write_partials(acc, partials, blockIdx.x);
}

template <class Op, bool DUAL>
static void launch(const ConePlan &p, const Op &op, double *partials, hipStream_t s) {
    if (p.ntiles == 0) return;
    const GridSync gs{p.grid_ctr, p.grid_part, p.grid_err};
    double *sr = Op::kWarm ? p.soc_root : nullptr, *er = Op::kWarm ? p.exp_root : nullptr;
    if (op.fp32())
        hipLaunchKernelGGL((cone_pass_kernel<Op, DUAL, true>), dim3((unsigned)p.ntiles), dim3(kBlock), 0,
                           s, op, p.tiles, p.soc_off, p.soc_dim, p.exp_off, partials, sr, er, gs);
    else
        hipLaunchKernelGGL((cone_pass_kernel<Op, DUAL, false>), dim3((unsigned)p.ntiles), dim3(kBlock), 0,
                           s, op, p.tiles, p.soc_off, p.soc_dim, p.exp_off, partials, sr, er, gs);
    PDCS_HIP(hipGetLastError());
}

__global__ void clear_grid_kernel(unsigned long long *ctr, int64_t n, int *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ctr[i] = 0ull;
    if (i == 0) *err = 0;
}

void clear_grid(const ConePlan &p, hipStream_t s) {
    if (p.n_grid == 0) return;
    hipLaunchKernelGGL(clear_grid_kernel, dim3((unsigned)((p.n_grid + 255) / 256)), dim3(256), 0, s,
                       p.grid_ctr, p.n_grid, p.grid_err);
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
    if (!a.d) {
        OpProjectUnit op;
        op.a = a;
        if (dual)
            launch<OpProjectUnit, true>(p, op, partials, s);
        else
            launch<OpProjectUnit, false>(p, op, partials, s);
    } else if (dual) {
        launch<OpProject, true>(p, OpProject{a}, partials, s);
    } else {
        launch<OpProject, false>(p, OpProject{a}, partials, s);
    }
}

}  // namespace pdcs
