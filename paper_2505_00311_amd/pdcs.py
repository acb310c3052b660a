"""Python binding of libpdcs (include/pdcs.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
and torch device tensors into the pointers and sizes of the C ABI.  Loading
fails loudly when libpdcs.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdcs.so")

OK = 0
SOLVE_STATUS = {0: "optimal", 1: "iteration_limit", 2: "time_limit", 3: "numerical"}

_i64, _i32, _dbl, _vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
_pd = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n", _i64), ("m", _i64), ("nnz", _i64), ("n_box", _i64),
                ("row_ptr", _vp), ("col", _vp), ("val", _vp), ("c", _vp), ("h", _vp),
                ("l", _vp), ("u", _vp),
                ("n_xcones", _i64), ("xcone_type", _pi32), ("xcone_dim", _pi64),
                ("n_rcones", _i64), ("rcone_type", _pi32), ("rcone_dim", _pi64)]


class Settings(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i64), ("time_limit", _dbl),
                ("check_every", _i32), ("ruiz_iters", _i32), ("pock_chambolle", _i32),
                ("beta_mode", _i32), ("beta_const", _dbl), ("beta_grow", _dbl),
                ("beta_shrink", _dbl), ("step_reduce_exp", _dbl), ("step_grow_exp", _dbl),
                ("restart_sufficient", _dbl), ("restart_necessary", _dbl),
                ("restart_artificial", _dbl), ("max_attempts", _i32), ("out_on_device", _i32),
                ("step_mode", _i32), ("step_fixed", _dbl), ("power_iters", _i32),
                ("use_graph", _i32), ("time_kernels", _i32), ("precision", _i32),
                ("polish_tol", _dbl), ("polish_stall", _i32), ("autotune", _i32),
                ("batch_dropout", _i32), ("plain_pdhg", _i32), ("log_every", _dbl)]

KERNELS = ("primal", "spmv_g", "dual", "decide", "spmv_gt", "halpern")


class Info(ctypes.Structure):
    _fields_ = [("status", _i32), ("iterations", _i64), ("attempts", _i64), ("restarts", _i64),
                ("spmv", _i64), ("pobj", _dbl), ("dobj", _dbl), ("err_p", _dbl), ("err_d", _dbl),
                ("err_gap", _dbl), ("omega", _dbl), ("eta", _dbl), ("setup_s", _dbl),
                ("solve_s", _dbl), ("kernel_ms", _dbl * 6), ("kernel_launches", _i64 * 6),
                ("polish_iter", _i64), ("done_s", _dbl)]


class Trace(ctypes.Structure):
    _fields_ = [("cap", _i64), ("count", _i64), ("attempts", _pi32), ("eta_used", _pd),
                ("beta", _pd), ("omega", _pd), ("check_code", _pi32), ("check_kkt", _pd),
                ("n_snap", _i64), ("snap_iter", _pi64), ("snap_x", _pd), ("snap_y", _pd),
                ("replay_count", _i64), ("replay_attempts", _pi32), ("replay_beta", _pd),
                ("replay_check_code", _pi32)]


class PdcsError(RuntimeError):
    pass


_lib = None

SYMBOLS = ["pdcs_settings_default", "pdcs_problem_create", "pdcs_problem_create_device",
           "pdcs_problem_destroy", "pdcs_solve", "pdcs_scaling", "pdcs_spmv", "pdcs_spmv32",
           "pdcs_set_layout", "pdcs_get_layout", "pdcs_kkt", "pdcs_cones_create", "pdcs_cones_project",
           "pdcs_cones_destroy", "pdcs_project", "pdcs_project_fp32", "pdcs_project_noalloc", "pdcs_batch_create", "pdcs_batch_solve", "pdcs_batch_size",
           "pdcs_batch_destroy", "pdcs_mlp_create", "pdcs_mlp_num_params", "pdcs_mlp_forward",
           "pdcs_mlp_gradient", "pdcs_mlp_train_step", "pdcs_mlp_get_params", "pdcs_mlp_destroy",
           "pdcs_gemm_bf16", "pdcs_status_string", "pdcs_last_error"]


def load():
    """Loads libpdcs.so; raises if it is missing (build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PdcsError(f"{LIB_PATH} is not built; run `python -m paper_2505_00311_amd.build`")
    # torch's HIP runtime must be the process's one: torch asks for
    # libamdhip64.so, which would not match an already loaded libamdhip64.so.7,
    # and two runtimes cannot share the device
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    L.pdcs_settings_default.argtypes = [ctypes.POINTER(Settings)]
    L.pdcs_problem_create.argtypes = [ctypes.POINTER(ProblemDesc), _vp, ctypes.POINTER(_vp)]
    L.pdcs_problem_create_device.argtypes = [ctypes.POINTER(ProblemDesc), _vp, ctypes.POINTER(_vp)]
    L.pdcs_problem_destroy.argtypes = [_vp]
    L.pdcs_problem_destroy.restype = None
    L.pdcs_solve.argtypes = [_vp, ctypes.POINTER(Settings), _vp, _vp, _dbl, _vp, _vp,
                             ctypes.POINTER(Info), ctypes.POINTER(Trace)]
    L.pdcs_scaling.argtypes = [_vp, ctypes.POINTER(Settings), _vp, _vp]
    L.pdcs_spmv.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
    L.pdcs_spmv32.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
    L.pdcs_set_layout.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
    L.pdcs_get_layout.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.pdcs_kkt.argtypes = [_vp, _vp, _vp, _vp]
    L.pdcs_cones_create.argtypes = [_i64, _pi32, _pi64, _vp, ctypes.POINTER(_vp)]
    L.pdcs_cones_project.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
    L.pdcs_cones_destroy.argtypes = [_vp]
    L.pdcs_cones_destroy.restype = None
    L.pdcs_project.argtypes = [_i64, _pi32, _pi64, ctypes.c_int, _vp, _vp, _vp]
    L.pdcs_project_fp32.argtypes = [_i64, _pi32, _pi64, ctypes.c_int, _vp, _vp, _vp]
    L.pdcs_project_noalloc.argtypes = [_i64, _pi32, _pi64, ctypes.c_int, _vp, _vp, _vp]
    L.pdcs_batch_create.argtypes = [ctypes.POINTER(ProblemDesc), _i64, _vp, ctypes.POINTER(_vp)]
    L.pdcs_batch_solve.argtypes = [_vp, ctypes.POINTER(Settings), _vp, _vp, _vp,
                                   ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(Info)]
    L.pdcs_batch_size.argtypes = [_vp]
    L.pdcs_batch_size.restype = _i64
    L.pdcs_batch_destroy.argtypes = [_vp]
    L.pdcs_batch_destroy.restype = None
    L.pdcs_mlp_create.argtypes = [_i64, _i64, _i64, _i64, _vp, _vp, ctypes.POINTER(_vp)]
    L.pdcs_mlp_num_params.argtypes = [_vp]
    L.pdcs_mlp_num_params.restype = _i64
    L.pdcs_mlp_forward.argtypes = [_vp, _vp, _i64, _vp]
    L.pdcs_mlp_gradient.argtypes = [_vp, _vp, _vp, _i64, _vp, ctypes.POINTER(_dbl)]
    L.pdcs_mlp_train_step.argtypes = [_vp, _vp, _vp, _i64, ctypes.c_float, ctypes.POINTER(_dbl)]
    L.pdcs_mlp_get_params.argtypes = [_vp, _vp]
    L.pdcs_mlp_destroy.argtypes = [_vp]
    L.pdcs_mlp_destroy.restype = None
    L.pdcs_gemm_bf16.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _vp, _i64, _vp, _i64,
                                 _vp, ctypes.c_int, _vp, _vp, _i64, _vp]
    L.pdcs_status_string.argtypes = [ctypes.c_int]
    L.pdcs_status_string.restype = ctypes.c_char_p
    L.pdcs_last_error.argtypes = []
    L.pdcs_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        L = load()
        raise PdcsError(f"{L.pdcs_status_string(rc).decode()}: {L.pdcs_last_error().decode()}")


def settings_default(**overrides) -> Settings:
    s = Settings()
    _check(load().pdcs_settings_default(ctypes.byref(s)))
    for k, v in overrides.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _desc(inst, host, keep, from_device=False):
    """pdcs_problem_desc of an Instance; `host` pins the arrays it makes."""
    n_box = int(inst.n_box)
    rp, col, val = host(inst.row_ptr, np.int64), host(inst.col, np.int32), host(inst.val, np.float64)
    c, h = host(inst.c, np.float64), host(inst.h, np.float64)
    l = host(inst.l if n_box else np.zeros(1), np.float64)
    u = host(inst.u if n_box else np.zeros(1), np.float64)
    if from_device:
        import torch
        dev = [torch.from_numpy(a).cuda() for a in (rp, col, val, c, h, l, u)]
        torch.cuda.synchronize()
        keep += dev
        ptrs = [_dptr(t) for t in dev]
    else:
        ptrs = [ctypes.c_void_p(a.ctypes.data) for a in (rp, col, val, c, h, l, u)]
    xt, xd = host(inst.xcone_type, np.int32), host(inst.xcone_dim, np.int64)
    rt, rd = host(inst.rcone_type, np.int32), host(inst.rcone_dim, np.int64)
    return ProblemDesc(int(inst.n), int(inst.m), int(val.size), n_box, *ptrs,
                       int(xt.size), xt.ctypes.data_as(_pi32), xd.ctypes.data_as(_pi64),
                       int(rt.size), rt.ctypes.data_as(_pi32), rd.ctypes.data_as(_pi64))


class Batch:
    """A batch handle (pdcs_batch_create): independent instances solved together."""

    def __init__(self, insts, stream=None):
        L = load()
        keep = []

        def host(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a

        self.sizes = [(int(i.n), int(i.m)) for i in insts]
        self.stream = _stream(stream)
        descs = (ProblemDesc * len(insts))(*[_desc(i, host, keep) for i in insts])
        handle = ctypes.c_void_p()
        _check(L.pdcs_batch_create(descs, len(insts), self.stream, ctypes.byref(handle)))
        self.handle = handle

    def solve(self, settings: Settings | None = None, x0=None, y0=None, omega0=None):
        """pdcs_batch_solve -> list of dicts (info fields plus x, y).  x0, y0:
        lists of per-instance starting points (entries may be None); omega0:
        per-instance primal weights (<= 0: default)."""
        L = load()
        s = settings or settings_default()
        s.out_on_device = 0
        B = len(self.sizes)
        xs = [np.empty(n) for n, _ in self.sizes]
        ys = [np.empty(m) for _, m in self.sizes]
        px = (_vp * B)(*[ctypes.c_void_p(a.ctypes.data) for a in xs])
        py = (_vp * B)(*[ctypes.c_void_p(a.ctypes.data) for a in ys])
        keep = []

        def ptrs(vs):
            if vs is None:
                return None
            arr = (_vp * B)()
            for b, v in enumerate(vs):
                if v is not None:
                    a = np.ascontiguousarray(v, dtype=np.float64)
                    keep.append(a)
                    arr[b] = a.ctypes.data
            keep.append(arr)
            return ctypes.cast(arr, _vp)

        om = None
        if omega0 is not None:
            om = np.ascontiguousarray(omega0, dtype=np.float64)
        infos = (Info * B)()
        _check(L.pdcs_batch_solve(self.handle, ctypes.byref(s), ptrs(x0), ptrs(y0),
                                  None if om is None else ctypes.c_void_p(om.ctypes.data), px, py, infos))
        out = []
        for b in range(B):
            d = {k: getattr(infos[b], k) for k, _ in Info._fields_}
            d["x"], d["y"] = xs[b], ys[b]
            out.append(d)
        return out

    def close(self):
        if getattr(self, "handle", None):
            load().pdcs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


LAYOUT_DEFAULT = 0
LAYOUT_STREAM = -1


def slabs(S):
    """Layout code of the column-slab product with S slabs (PDCS_LAYOUT_SLABS)."""
    return -10 - int(S)


class Problem:
    """A problem handle (pdcs_problem_create / pdcs_problem_create_device)."""

    def __init__(self, inst, stream=None, from_device=False):
        L = load()
        self._keep = []
        self.n, self.m, self.n_box = int(inst.n), int(inst.m), int(inst.n_box)
        self.stream = _stream(stream)

        def host(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        desc = _desc(inst, host, self._keep, from_device)
        handle = ctypes.c_void_p()
        fn = L.pdcs_problem_create_device if from_device else L.pdcs_problem_create
        _check(fn(ctypes.byref(desc), self.stream, ctypes.byref(handle)))
        self.handle = handle
        self._keep = []

    def close(self):
        if getattr(self, "handle", None):
            load().pdcs_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ solve
    def solve(self, settings: Settings | None = None, x0=None, y0=None, omega0: float = 0.0,
              log_cap: int = 0, snap_iters=None, x_out=None, y_out=None, replay=None):
        """pdcs_solve.  Returns a dict of the info fields plus x, y (numpy, or the
        given device tensors x_out/y_out) and, if requested, the decision log.
        `replay`: another run's decision log (a dict with "attempts", "beta" and
        "check_code" arrays) whose decisions this solve takes."""
        L = load()
        s = settings or settings_default()
        on_dev = x_out is not None
        s.out_on_device = 1 if on_dev else 0
        if on_dev:
            xo, yo = x_out, y_out
            px, py = _dptr(xo), _dptr(yo)
        else:
            xo, yo = np.empty(self.n), np.empty(self.m)
            px, py = ctypes.c_void_p(xo.ctypes.data), ctypes.c_void_p(yo.ctypes.data)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        y0a = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
        info = Info()
        tr, logs = None, None
        if log_cap or snap_iters is not None:
            cap = max(int(log_cap), 1)
            snaps = np.ascontiguousarray(snap_iters if snap_iters is not None else [], np.int64)
            logs = {"attempts": np.zeros(cap, np.int32), "eta_used": np.zeros(cap),
                    "beta": np.zeros(cap), "omega": np.zeros(cap),
                    "check_code": np.zeros(cap, np.int32), "check_kkt": np.zeros(cap),
                    "snap_iter": snaps, "snap_x": np.zeros((max(snaps.size, 1), self.n)),
                    "snap_y": np.zeros((max(snaps.size, 1), self.m))}
            tr = Trace(cap, 0, logs["attempts"].ctypes.data_as(_pi32),
                       logs["eta_used"].ctypes.data_as(_pd), logs["beta"].ctypes.data_as(_pd),
                       logs["omega"].ctypes.data_as(_pd), logs["check_code"].ctypes.data_as(_pi32),
                       logs["check_kkt"].ctypes.data_as(_pd), int(snaps.size),
                       snaps.ctypes.data_as(_pi64), logs["snap_x"].ctypes.data_as(_pd),
                       logs["snap_y"].ctypes.data_as(_pd))
        if replay is not None:
            if tr is None:
                raise ValueError("a replay needs log_cap or snap_iters")
            ra = np.ascontiguousarray(replay["attempts"], np.int32)
            rb = np.ascontiguousarray(replay["beta"], np.float64)
            rc = np.ascontiguousarray(replay["check_code"], np.int32)
            logs["_replay"] = (ra, rb, rc)   # alive until the call returns
            tr.replay_count = int(min(ra.size, rb.size, rc.size))
            tr.replay_attempts = ra.ctypes.data_as(_pi32)
            tr.replay_beta = rb.ctypes.data_as(_pd)
            tr.replay_check_code = rc.ctypes.data_as(_pi32)
        _check(L.pdcs_solve(self.handle, ctypes.byref(s),
                            None if x0a is None else ctypes.c_void_p(x0a.ctypes.data),
                            None if y0a is None else ctypes.c_void_p(y0a.ctypes.data),
                            float(omega0), px, py, ctypes.byref(info),
                            ctypes.byref(tr) if tr is not None else None))
        out = {k: getattr(info, k) for k, _ in Info._fields_}
        out["kernel_ms"] = dict(zip(KERNELS, info.kernel_ms))
        out["kernel_launches"] = dict(zip(KERNELS, info.kernel_launches))
        out["x"], out["y"] = xo, yo
        if logs is not None:
            cnt = tr.count
            for k in ("attempts", "eta_used", "beta", "omega", "check_code", "check_kkt"):
                logs[k] = logs[k][:cnt]
            logs.pop("_replay", None)
            out["log"] = logs
        return out

    def scaling(self, settings: Settings | None = None):
        """pdcs_scaling -> (e [m], f [n])."""
        e, f = np.empty(self.m), np.empty(self.n)
        _check(load().pdcs_scaling(self.handle, ctypes.byref(settings or settings_default()),
                                   ctypes.c_void_p(e.ctypes.data), ctypes.c_void_p(f.ctypes.data)))
        return e, f

    def spmv(self, x_dev, y_dev, transpose=False, stream=None, fp32=False):
        """pdcs_spmv (pdcs_spmv32 with fp32) on device tensors: y = G x (or G^T x)."""
        fn = load().pdcs_spmv32 if fp32 else load().pdcs_spmv
        _check(fn(self.handle, 1 if transpose else 0, _dptr(x_dev), _dptr(y_dev),
                  _stream(stream) if stream is not None else self.stream))

    def set_layout(self, layout_g, layout_gt):
        """pdcs_set_layout: product layouts by code (LAYOUT_* / slabs(S) / lanes)."""
        _check(load().pdcs_set_layout(self.handle, int(layout_g), int(layout_gt)))

    def layout(self):
        """pdcs_get_layout -> (layout of G x, layout of G^T y)."""
        g, gt = ctypes.c_int(0), ctypes.c_int(0)
        _check(load().pdcs_get_layout(self.handle, ctypes.byref(g), ctypes.byref(gt)))
        return g.value, gt.value

    def kkt(self, x_dev, y_dev):
        """pdcs_kkt at unscaled device tensors -> dict."""
        out = np.empty(5)
        _check(load().pdcs_kkt(self.handle, _dptr(x_dev), _dptr(y_dev),
                               ctypes.c_void_p(out.ctypes.data)))
        return dict(zip(("err_p", "err_d", "err_gap", "pobj", "dobj"), out.tolist()))


def project(types, dims, v_dev, d_dev=None, dual=False, stream=None):
    """pdcs_project: in-place projection of the device tensor v_dev."""
    t = np.ascontiguousarray(types, np.int32)
    k = np.ascontiguousarray(dims, np.int64)
    _check(load().pdcs_project(int(t.size), t.ctypes.data_as(_pi32), k.ctypes.data_as(_pi64),
                               1 if dual else 0, None if d_dev is None else _dptr(d_dev),
                               _dptr(v_dev), _stream(stream)))


def project_fp32(types, dims, v_dev, d_dev=None, dual=False, stream=None):
    """pdcs_project_fp32: the mixed form's FP32 projections, in place."""
    t = np.ascontiguousarray(types, np.int32)
    k = np.ascontiguousarray(dims, np.int64)
    _check(load().pdcs_project_fp32(int(t.size), t.ctypes.data_as(_pi32), k.ctypes.data_as(_pi64),
                                    1 if dual else 0, None if d_dev is None else _dptr(d_dev),
                                    _dptr(v_dev), _stream(stream)))


def project_noalloc(types, dims, v_dev, d_dev=None, dual=False, stream=None):
    """pdcs_project_noalloc: pdcs_project with its scratch in a fixed device
    array (no device allocation), in place."""
    t = np.ascontiguousarray(types, np.int32)
    k = np.ascontiguousarray(dims, np.int64)
    _check(load().pdcs_project_noalloc(int(t.size), t.ctypes.data_as(_pi32), k.ctypes.data_as(_pi64),
                                       1 if dual else 0, None if d_dev is None else _dptr(d_dev),
                                       _dptr(v_dev), _stream(stream)))


class Cones:
    """A reusable projection plan (pdcs_cones_*): project() enqueues the
    projection of a device tensor in place on the stream without waiting."""

    def __init__(self, types, dims, stream=None):
        L = load()
        t = np.ascontiguousarray(types, np.int32)
        k = np.ascontiguousarray(dims, np.int64)
        self.size = int(k.sum())
        h = _vp()
        _check(L.pdcs_cones_create(int(t.size), t.ctypes.data_as(_pi32), k.ctypes.data_as(_pi64),
                                   _stream(stream), ctypes.byref(h)))
        self.handle = h

    def project(self, v_dev, d_dev=None, dual=False, stream=None):
        _check(load().pdcs_cones_project(self.handle, 1 if dual else 0,
                                         None if d_dev is None else _dptr(d_dev), _dptr(v_dev),
                                         _stream(stream)))

    def close(self):
        if self.handle:
            load().pdcs_cones_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The warm-start network (pdcs_mlp_*): device-resident parameters, BF16
    matrix-core GEMMs with FP32 accumulation, Adam training."""

    def __init__(self, n_in, hidden, n_out, params, max_batch, stream=None):
        L = load()
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.n_in, self.hidden, self.n_out, self.max_batch = n_in, hidden, n_out, max_batch
        handle = ctypes.c_void_p()
        _check(L.pdcs_mlp_create(n_in, hidden, n_out, max_batch, ctypes.c_void_p(p.ctypes.data),
                                 _stream(stream), ctypes.byref(handle)))
        self.handle = handle
        self.num_params = int(L.pdcs_mlp_num_params(handle))

    def forward(self, theta_dev, out_dev):
        _check(load().pdcs_mlp_forward(self.handle, _dptr(theta_dev), int(theta_dev.shape[0]), _dptr(out_dev)))

    def gradient(self, theta_dev, target_dev):
        g = np.empty(self.num_params, np.float32)
        loss = ctypes.c_double()
        _check(load().pdcs_mlp_gradient(self.handle, _dptr(theta_dev), _dptr(target_dev),
                                        int(theta_dev.shape[0]), ctypes.c_void_p(g.ctypes.data),
                                        ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, theta_dev, target_dev, lr):
        loss = ctypes.c_double()
        _check(load().pdcs_mlp_train_step(self.handle, _dptr(theta_dev), _dptr(target_dev),
                                          int(theta_dev.shape[0]), float(lr), ctypes.byref(loss)))
        return loss.value

    def params(self):
        p = np.empty(self.num_params, np.float32)
        _check(load().pdcs_mlp_get_params(self.handle, ctypes.c_void_p(p.ctypes.data)))
        return p

    def close(self):
        if getattr(self, "handle", None):
            load().pdcs_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_bf16(a_dev, b_dev, M, N, K, ta=0, tb=0, lda=None, ldb=None, bias_dev=None, relu=False,
              c32_dev=None, c16_dev=None, ldc=None, stream=None):
    """pdcs_gemm_bf16 on device tensors (a_dev, b_dev, c16_dev: int16/uint16 bit patterns)."""
    lda = lda if lda is not None else (M if ta else K)
    ldb = ldb if ldb is not None else (K if tb else N)
    ldc = ldc if ldc is not None else N
    nul = ctypes.c_void_p(None)
    _check(load().pdcs_gemm_bf16(ta, tb, M, N, K, _dptr(a_dev), lda, _dptr(b_dev), ldb,
                                 _dptr(bias_dev) if bias_dev is not None else nul, 1 if relu else 0,
                                 _dptr(c32_dev) if c32_dev is not None else nul,
                                 _dptr(c16_dev) if c16_dev is not None else nul, ldc, _stream(stream)))
