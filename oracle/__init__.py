"""Plain FP64 CPU oracle for PDCS (restarted, reflected-Halpern, adaptive-step
PDHG for conic programs; Lin, Xiong, Ge, Ye).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path (``paper_2505_00311_amd``) never imports it and shares no code with it.

The arithmetic lives in ``pdcs_oracle.c`` (C99, double precision, single
thread); this module only compiles it with gcc and marshals numpy arrays
through ctypes.  An instance is any object with the attributes
``n, m, n_box, row_ptr, col, val, c, h, l, u, xcone_type, xcone_dim,
rcone_type, rcone_dim``.

Rotated second-order cones (type RSOC: 2 u v >= ||w||^2 with u, v >= 0, the
cone of the appendix's Lasso form) are handled here, in Python: the problem
is rewritten with the orthogonal symmetric map T that is the identity except
for the 2x2 block [[1, 1], [1, -1]] / sqrt 2 on the first two entries of each
rotated block (T maps the rotated cone onto the second-order cone), and
points are mapped by T on the way in and out.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdcs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ZERO, FREE, NONNEG, SOC, EXP, EXP_DUAL, RSOC = range(7)
OPTIMAL, ITER_LIMIT, TIME_LIMIT, NUMERICAL = range(4)

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("n", _i64), ("m", _i64), ("nnz", _i64), ("n_box", _i64),
                ("row_ptr", _pi64), ("col", _pi32), ("val", _pd),
                ("c", _pd), ("h", _pd), ("l", _pd), ("u", _pd),
                ("n_xcones", _i64), ("xcone_type", _pi32), ("xcone_dim", _pi64),
                ("n_rcones", _i64), ("rcone_type", _pi32), ("rcone_dim", _pi64)]


class Settings(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i64), ("check_every", _i32),
                ("ruiz_iters", _i32), ("pock_chambolle", _i32), ("beta_mode", _i32),
                ("beta_const", _dbl), ("beta_grow", _dbl), ("beta_shrink", _dbl),
                ("step_reduce_exp", _dbl), ("step_grow_exp", _dbl),
                ("restart_sufficient", _dbl), ("restart_necessary", _dbl),
                ("restart_artificial", _dbl), ("max_attempts", _i32), ("step_mode", _i32),
                ("step_fixed", _dbl), ("power_iters", _i32), ("plain_pdhg", _i32)]


class _Info(ctypes.Structure):
    _fields_ = [("status", _i32), ("iterations", _i64), ("attempts", _i64),
                ("restarts", _i64), ("pobj", _dbl), ("dobj", _dbl), ("err_p", _dbl),
                ("err_d", _dbl), ("err_gap", _dbl), ("omega", _dbl), ("eta", _dbl)]


class _Trace(ctypes.Structure):
    _fields_ = [("cap", _i64), ("count", _i64), ("attempts", _pi32), ("eta_used", _pd),
                ("beta", _pd), ("omega", _pd), ("check_code", _pi32), ("check_kkt", _pd),
                ("n_snap", _i64), ("snap_iter", _pi64), ("snap_x", _pd), ("snap_y", _pd),
                ("replay_count", _i64), ("replay_attempts", _pi32), ("replay_beta", _pd),
                ("replay_check_code", _pi32), ("margin", _pd)]


_lib_handle = None


def _declare(L):
    L.orc_settings_default.argtypes = [ctypes.POINTER(Settings)]
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = None
    L.orc_get_threads.argtypes = []
    L.orc_proj_soc.argtypes = [_i64, _pd, _pd, _pd]
    L.orc_proj_exp.argtypes = [_pd, _pd, _pd]
    L.orc_proj_exp_dual.argtypes = [_pd, _pd, _pd]
    L.orc_proj_blocks.argtypes = [_i64, _pi32, _pi64, ctypes.c_int, _pd, _pd]
    L.orc_proj_blocks.restype = None
    L.orc_spmv.argtypes = [_i64, _pi64, _pi32, _pd, _pd, _pd]
    L.orc_spmv.restype = None
    L.orc_scaling.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(Settings), _pd, _pd]
    L.orc_kkt.argtypes = [ctypes.POINTER(_Problem), _pd, _pd, _pd, _pd, _pd, _pd, _pd]
    L.orc_onepdhg.argtypes = [ctypes.POINTER(_Problem), _pd, _pd, _dbl, _dbl, _pd, _pd]
    L.orc_solve.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(Settings), _pd, _pd,
                            _dbl, _pd, _pd, ctypes.POINTER(_Info), ctypes.POINTER(_Trace)]
    return L


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib_handle = _declare(ctypes.CDLL(_LIB))
    return _lib_handle


def build_variant(name: str, flags) -> ctypes.CDLL:
    """The same oracle source compiled with other floating-point flags (for
    example FMA contraction on) into liboracle_<name>.so: a second, equally
    valid rounding of the same arithmetic, for measuring how far two correct
    FP64 implementations drift apart.  Pass the handle as solve(..., lib=)."""
    out = os.path.join(_HERE, f"liboracle_{name}.so")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", *flags,
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return _declare(ctypes.CDLL(out))


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


class _Keep:
    """Holds the contiguous copies a ctypes struct points into."""

    def __init__(self):
        self.refs = []

    def arr(self, a, dtype):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        self.refs.append(a)
        return a


def _problem(inst, keep: _Keep) -> _Problem:
    rp = keep.arr(inst.row_ptr, np.int64)
    col = keep.arr(inst.col, np.int32)
    val = keep.arr(inst.val, np.float64)
    c = keep.arr(inst.c, np.float64)
    h = keep.arr(inst.h, np.float64)
    nb = int(inst.n_box)
    l = keep.arr(inst.l if nb else np.zeros(1), np.float64)
    u = keep.arr(inst.u if nb else np.zeros(1), np.float64)
    xt = keep.arr(inst.xcone_type, np.int32)
    xd = keep.arr(inst.xcone_dim, np.int64)
    rt = keep.arr(inst.rcone_type, np.int32)
    rd = keep.arr(inst.rcone_dim, np.int64)
    return _Problem(int(inst.n), int(inst.m), int(val.size), nb,
                    _ptr(rp, ctypes.c_int64), _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_double),
                    _ptr(c, ctypes.c_double), _ptr(h, ctypes.c_double),
                    _ptr(l, ctypes.c_double), _ptr(u, ctypes.c_double),
                    int(xt.size), _ptr(xt, ctypes.c_int32), _ptr(xd, ctypes.c_int64),
                    int(rt.size), _ptr(rt, ctypes.c_int32), _ptr(rd, ctypes.c_int64))


def _rotation(types, dims, start, size):
    """The map T over a vector of `size` entries whose cone blocks (types,
    dims) start at entry `start`: a sparse matrix, identity except
    [[1, 1], [1, -1]] / sqrt 2 on the first two entries of each rotated
    block.  T is symmetric and orthogonal, so T^-1 = T^T = T."""
    import scipy.sparse as sp
    r = 1.0 / np.sqrt(2.0)
    rows, cols, vals = [], [], []
    rotated = set()
    o = start
    for t, d in zip(np.asarray(types), np.asarray(dims)):
        if int(t) == RSOC:
            rotated.update((o, o + 1))
            rows += [o, o, o + 1, o + 1]
            cols += [o, o + 1, o, o + 1]
            vals += [r, r, r, -r]
        o += int(d)
    ident = [i for i in range(size) if i not in rotated]
    rows += ident
    cols += ident
    vals += [1.0] * len(ident)
    return sp.csr_matrix((vals, (rows, cols)), shape=(size, size))


def _has_rsoc(inst):
    return bool(np.any(np.asarray(inst.xcone_type) == RSOC) or
                np.any(np.asarray(inst.rcone_type) == RSOC))


def _as_soc(inst):
    """The problem with every rotated block replaced by an SOC block:
    G' = T_r G T_x, c' = T_x c, h' = T_r h (T_r over the rows, T_x over x);
    x = T_x x', y = T_r y'.  Returns (problem, T_x, T_r)."""
    import scipy.sparse as sp
    from types import SimpleNamespace
    n, m = int(inst.n), int(inst.m)
    Tx = _rotation(inst.xcone_type, inst.xcone_dim, int(inst.n_box), n)
    Tr = _rotation(inst.rcone_type, inst.rcone_dim, 0, m)
    G = sp.csr_matrix((np.asarray(inst.val, np.float64), np.asarray(inst.col, np.int64),
                       np.asarray(inst.row_ptr, np.int64)), shape=(m, n))
    G2 = sp.csr_matrix(Tr @ G @ Tx)
    G2.eliminate_zeros()
    G2.sort_indices()
    soc = lambda t: np.where(np.asarray(t) == RSOC, SOC, np.asarray(t)).astype(np.int32)
    return SimpleNamespace(
        n=n, m=m, n_box=int(inst.n_box), row_ptr=G2.indptr.astype(np.int64),
        col=G2.indices.astype(np.int32), val=G2.data.astype(np.float64),
        c=Tx @ np.asarray(inst.c, np.float64), h=Tr @ np.asarray(inst.h, np.float64),
        l=inst.l, u=inst.u, xcone_type=soc(inst.xcone_type), xcone_dim=inst.xcone_dim,
        rcone_type=soc(inst.rcone_type), rcone_dim=inst.rcone_dim), Tx, Tr


def set_threads(n: int) -> None:
    """Threads of the oracle's timing mode (1 = the deterministic default)."""
    _lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_lib().orc_get_threads())


def default_settings(**overrides) -> Settings:
    s = Settings()
    _lib().orc_settings_default(ctypes.byref(s))
    for k, v in overrides.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


# ---------------------------------------------------------------- projections
def proj_soc(v, d=None):
    """Projection onto D K_soc (Theorem 1). Returns (projection, case)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty_like(v)
    case = _lib().orc_proj_soc(v.size, _ptr(v, ctypes.c_double), _ptr(dd, ctypes.c_double),
                               _ptr(out, ctypes.c_double))
    return out, case


def proj_exp(v, d=None):
    """Projection onto D K_exp (Theorem 3). Returns (projection, case)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty(3)
    case = _lib().orc_proj_exp(_ptr(v, ctypes.c_double), _ptr(dd, ctypes.c_double),
                               _ptr(out, ctypes.c_double))
    return out, case


def proj_exp_dual(v, d=None):
    """Projection onto D K_exp^* (Remark of Appendix A.2). Returns (projection, case)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty(3)
    case = _lib().orc_proj_exp_dual(_ptr(v, ctypes.c_double), _ptr(dd, ctypes.c_double),
                                    _ptr(out, ctypes.c_double))
    return out, case


def proj_blocks(types, dims, v, d=None, dual=False):
    """Projection onto a product of (scaled) cones, eq. (6).  Rotated blocks:
    T P_SOC(T v), for D = I only (the rotated cone is self-dual)."""
    if np.any(np.asarray(types) == RSOC):
        if d is not None:
            raise ValueError("rotated SOC blocks are projected with D = I")
        T = _rotation(types, dims, 0, int(np.sum(dims)))
        st = np.where(np.asarray(types) == RSOC, SOC, np.asarray(types))
        return T @ proj_blocks(st, dims, T @ np.asarray(v, np.float64), None, dual)
    t = np.ascontiguousarray(types, dtype=np.int32)
    k = np.ascontiguousarray(dims, dtype=np.int64)
    out = np.array(v, dtype=np.float64, copy=True)
    dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
    _lib().orc_proj_blocks(t.size, _ptr(t, ctypes.c_int32), _ptr(k, ctypes.c_int64),
                           1 if dual else 0, _ptr(dd, ctypes.c_double), _ptr(out, ctypes.c_double))
    return out


def spmv(row_ptr, col, val, x):
    """y = A x for a CSR matrix (plain definition)."""
    rp = np.ascontiguousarray(row_ptr, np.int64)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    xx = np.ascontiguousarray(x, np.float64)
    y = np.empty(rp.size - 1)
    _lib().orc_spmv(rp.size - 1, _ptr(rp, ctypes.c_int64), _ptr(ci, ctypes.c_int32),
                    _ptr(v, ctypes.c_double), _ptr(xx, ctypes.c_double), _ptr(y, ctypes.c_double))
    return y


# ---------------------------------------------------------------- problem-level
def scaling(inst, settings: Settings | None = None):
    """Rescaling factors (E, F); of the rewritten problem when it has rotated blocks."""
    if _has_rsoc(inst):
        inst = _as_soc(inst)[0]
    keep = _Keep()
    P = _problem(inst, keep)
    s = settings or default_settings()
    e = np.empty(int(inst.m))
    f = np.empty(int(inst.n))
    _lib().orc_scaling(ctypes.byref(P), ctypes.byref(s), _ptr(e, ctypes.c_double),
                       _ptr(f, ctypes.c_double))
    return e, f


def kkt(inst, x, y):
    """eq. (PDCS_terminate_tolerance) at unscaled (x, y); with rotated
    blocks, the measures of the rewritten problem at (T_x x, T_r y)."""
    if _has_rsoc(inst):
        inst, Tx, Tr = _as_soc(inst)
        x, y = Tx @ np.asarray(x, np.float64), Tr @ np.asarray(y, np.float64)
    keep = _Keep()
    P = _problem(inst, keep)
    x = keep.arr(x, np.float64)
    y = keep.arr(y, np.float64)
    out = [ctypes.c_double() for _ in range(5)]
    _lib().orc_kkt(ctypes.byref(P), _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                   *[ctypes.byref(o) for o in out])
    ep, ed, eg, po, do = (o.value for o in out)
    return {"err_p": ep, "err_d": ed, "err_gap": eg, "pobj": po, "dobj": do}


def onepdhg(inst, x, y, tau, sigma):
    """One PDHG step, eq. (5), on the unscaled problem."""
    if _has_rsoc(inst):
        inst2, Tx, Tr = _as_soc(inst)
        xh, yh = onepdhg(inst2, Tx @ np.asarray(x, np.float64), Tr @ np.asarray(y, np.float64),
                         tau, sigma)
        return Tx @ xh, Tr @ yh
    keep = _Keep()
    P = _problem(inst, keep)
    x = keep.arr(x, np.float64)
    y = keep.arr(y, np.float64)
    xh = np.empty(int(inst.n))
    yh = np.empty(int(inst.m))
    _lib().orc_onepdhg(ctypes.byref(P), _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                       float(tau), float(sigma), _ptr(xh, ctypes.c_double),
                       _ptr(yh, ctypes.c_double))
    return xh, yh


def solve(inst, settings: Settings | None = None, x0=None, y0=None, omega0: float = 0.0,
          log_cap: int = 0, snap_iters=None, replay=None, lib=None):
    """Algorithm 1 with rescaling.  Returns a dict with x, y, info fields and,
    if requested, the decision log and iterate snapshots.  `replay` (a decision
    log: a dict with "attempts", "beta" and "check_code" arrays) forces those
    decisions for as many iterations as it holds.  `lib` is another build of
    the same source (build_variant) to run instead.  Rotated blocks: the
    rewritten problem is solved from (T_x x0, T_r y0) and its iterates are
    mapped back by T."""
    if _has_rsoc(inst):
        inst2, Tx, Tr = _as_soc(inst)
        fwd = lambda T, v: None if v is None else T @ np.asarray(v, np.float64)
        res = solve(inst2, settings, fwd(Tx, x0), fwd(Tr, y0), omega0, log_cap, snap_iters,
                    replay, lib)
        res["x"], res["y"] = Tx @ res["x"], Tr @ res["y"]
        if "log" in res:
            res["log"]["snap_x"] = np.array([Tx @ v for v in res["log"]["snap_x"]])
            res["log"]["snap_y"] = np.array([Tr @ v for v in res["log"]["snap_y"]])
        return res
    keep = _Keep()
    P = _problem(inst, keep)
    s = settings or default_settings()
    n, m = int(inst.n), int(inst.m)
    x0a = keep.arr(x0, np.float64)
    y0a = keep.arr(y0, np.float64)
    x = np.empty(n)
    y = np.empty(m)
    info = _Info()
    tr = None
    logs = None
    if log_cap or snap_iters is not None:
        cap = max(int(log_cap), 1)
        snaps = np.ascontiguousarray(snap_iters if snap_iters is not None else [], dtype=np.int64)
        logs = {"attempts": np.zeros(cap, np.int32), "eta_used": np.zeros(cap),
                "beta": np.zeros(cap), "omega": np.zeros(cap),
                "check_code": np.zeros(cap, np.int32), "check_kkt": np.zeros(cap),
                "margin": np.zeros(cap),
                "snap_iter": snaps, "snap_x": np.zeros((max(snaps.size, 1), n)),
                "snap_y": np.zeros((max(snaps.size, 1), m))}
        tr = _Trace(cap, 0, _ptr(logs["attempts"], ctypes.c_int32),
                    _ptr(logs["eta_used"], ctypes.c_double), _ptr(logs["beta"], ctypes.c_double),
                    _ptr(logs["omega"], ctypes.c_double),
                    _ptr(logs["check_code"], ctypes.c_int32),
                    _ptr(logs["check_kkt"], ctypes.c_double), int(snaps.size),
                    _ptr(snaps, ctypes.c_int64), _ptr(logs["snap_x"], ctypes.c_double),
                    _ptr(logs["snap_y"], ctypes.c_double))
        tr.margin = _ptr(logs["margin"], ctypes.c_double)
    if replay is not None:
        if tr is None:
            raise ValueError("a replay needs log_cap or snap_iters")
        ra = keep.arr(replay["attempts"], np.int32)
        rb = keep.arr(replay["beta"], np.float64)
        rcc = keep.arr(replay["check_code"], np.int32)
        tr.replay_count = int(min(ra.size, rb.size, rcc.size))
        tr.replay_attempts = _ptr(ra, ctypes.c_int32)
        tr.replay_beta = _ptr(rb, ctypes.c_double)
        tr.replay_check_code = _ptr(rcc, ctypes.c_int32)
    rc = (lib or _lib()).orc_solve(ctypes.byref(P), ctypes.byref(s), _ptr(x0a, ctypes.c_double),
                          _ptr(y0a, ctypes.c_double), float(omega0), _ptr(x, ctypes.c_double),
                          _ptr(y, ctypes.c_double), ctypes.byref(info),
                          ctypes.byref(tr) if tr is not None else None)
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    res = {k: getattr(info, k) for k, _ in _Info._fields_}
    res["x"], res["y"] = x, y
    if logs is not None:
        cnt = tr.count
        for k in ("attempts", "eta_used", "beta", "omega", "check_code", "check_kkt", "margin"):
            logs[k] = logs[k][:cnt]
        res["log"] = logs
    return res
