"""ctypes binding of ``libpovar.so`` (the C ABI in ``include/povar.h``).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the library.  The library must have been built (``python -m
paper_2405_05079_amd.build``); loading fails loudly otherwise.  PyTorch is
used only to hand over a HIP stream or device tensors when the caller asks.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpovar.so")

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ENUMERIC, ESTATE = range(7)
STATUS_NAMES = {0: "POVAR_OK", 1: "POVAR_EINVAL", 2: "POVAR_ENOMEM", 3: "POVAR_EDEVICE",
                4: "POVAR_EAGAIN", 5: "POVAR_ENUMERIC", 6: "POVAR_ESTATE"}
PRECISION = {"fp64": 0, "fp32_bulk": 1}
MANIFOLD = {"sphere": 0, "euclidean": 1}

# every symbol include/povar.h declares
EXPORTS = [
    "povar_options_default", "povar_ctx_create", "povar_ctx_destroy", "povar_last_error",
    "povar_problem_footprint", "povar_problem_create", "povar_problem_create_device",
    "povar_problem_destroy", "povar_solve", "povar_step", "povar_enqueue", "povar_get_report",
    "povar_get_cameras", "povar_get_points", "povar_get_trace", "povar_get_state", "povar_set_state",
    "povar_debug_linearize", "povar_debug_step", "povar_debug_camera_blocks", "povar_debug_layout_check",
    "povar_kernel_timing", "povar_kernel_times",
    "povar_problem_info", "povar_problem_layout", "povar_server_create", "povar_server_submit", "povar_server_poll",
    "povar_server_stats", "povar_server_destroy", "povar_refine_create", "povar_get_points_h",
    "povar_refine_debug_blocks", "povar_refine_debug_step", "povar_metric_upgrade", "povar_metric_debug_reduced",
    "povar_get_trace_diag", "povar_debug_series", "povar_server_profile", "povar_metric_upgrade_noalloc",
]


class PovarError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class MetricReport(C.Structure):
    _fields_ = [("cost_initial", C.c_double), ("cost_final", C.c_double), ("lambda_", C.c_double),
                ("iters", C.c_int32), ("stop", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("eta", C.c_double), ("series_order", C.c_int32),
                ("max_iters", C.c_int32), ("ftol", C.c_double), ("lambda0", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("precision", C.c_int32),
                ("manifold", C.c_int32), ("use_graph", C.c_int32), ("reserved", C.c_int32),
                ("series_rtol", C.c_double), ("init_seed", C.c_uint64)]


class Report(C.Structure):
    _fields_ = [("cost_initial", C.c_double), ("cost_final", C.c_double), ("lambda_final", C.c_double),
                ("grad_norm_final", C.c_double), ("seconds_total", C.c_double), ("seconds_series", C.c_double),
                ("iters", C.c_int32), ("accepted", C.c_int32), ("stop_reason", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib: Optional[C.CDLL] = None
_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)
_U64P = C.POINTER(C.c_uint64)


def lib() -> C.CDLL:
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_05079_amd.build` "
                           "(the PoVar path has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    sig = {
        "povar_options_default": (C.c_int, [C.POINTER(Options)]),
        "povar_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
        "povar_ctx_destroy": (C.c_int, [_P]),
        "povar_last_error": (C.c_char_p, [_P]),
        "povar_problem_footprint": (C.c_int, [C.c_int32, C.c_int32, C.c_int64, C.c_int32, _U64P]),
        "povar_problem_create": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P,
                                           C.POINTER(Options), C.POINTER(_P)]),
        "povar_problem_create_device": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P,
                                                  C.POINTER(Options), C.POINTER(_P)]),
        "povar_problem_destroy": (C.c_int, [_P]),
        "povar_solve": (C.c_int, [_P, C.POINTER(Report)]),
        "povar_step": (C.c_int, [_P, C.c_int32, C.POINTER(Report)]),
        "povar_enqueue": (C.c_int, [_P, C.c_int32]),
        "povar_get_report": (C.c_int, [_P, C.POINTER(Report)]),
        "povar_get_cameras": (C.c_int, [_P, _P]),
        "povar_get_points": (C.c_int, [_P, _P]),
        "povar_get_trace": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
        "povar_get_trace_diag": (C.c_int, [_P, C.c_int32, _P, _P]),
        "povar_debug_series": (C.c_int, [_P, _P, C.c_int32, _P]),
        "povar_get_state": (C.c_int, [_P, _P, _DP, _I32P, _DP]),
        "povar_set_state": (C.c_int, [_P, _P, C.c_double, C.c_int32]),
        "povar_debug_linearize": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _DP]),
        "povar_debug_step": (C.c_int, [_P, C.c_double, C.c_int32, _P, _P, _DP]),
        "povar_debug_camera_blocks": (C.c_int, [_P, C.c_double, _P]),
        "povar_debug_layout_check": (C.c_int, [C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, C.c_int32, _I64P]),
        "povar_kernel_timing": (C.c_int, [_P, C.c_int32]),
        "povar_kernel_times": (C.c_int, [_P, _DP, _I64P, _DP, _I64P]),
        "povar_problem_info": (C.c_int, [_P, _I64P, _I64P, _I32P, _U64P]),
        "povar_problem_layout": (C.c_int, [_P, _I32P, _I32P, _I64P, _I64P, _I32P]),
        "povar_server_create": (C.c_int, [_P, C.c_uint64, C.c_int32, C.POINTER(_P)]),
        "povar_server_submit": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P,
                                          C.POINTER(Options), _U64P]),
        "povar_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(Report), _P, _P, _P]),
        "povar_server_stats": (C.c_int, [_P, _I32P, _I32P, _I64P, _I64P]),
        "povar_server_destroy": (C.c_int, [_P]),
        "povar_server_profile": (C.c_int, [_P, _DP, _I64P]),
        "povar_refine_create": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P,
                                          C.POINTER(Options), C.POINTER(_P)]),
        "povar_get_points_h": (C.c_int, [_P, _P]),
        "povar_refine_debug_blocks": (C.c_int, [_P, C.c_double, _P, _P, _P, _P, _DP]),
        "povar_refine_debug_step": (C.c_int, [_P, C.c_double, C.c_int32, _P, _P, _P, _DP]),
        "povar_metric_upgrade": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int32, C.c_double, _P, _P, _P, _P, _P, _P, _P,
                                           C.POINTER(MetricReport)]),
        "povar_metric_debug_reduced": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _DP]),
        "povar_metric_upgrade_noalloc": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int32, C.c_double, _P, _P, _P, _P,
                                                   _P, _P, _P, C.POINTER(MetricReport)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


def make_options(eta=0.01, order=20, max_iters=50, ftol=1e-6, lambda0=1e-4, lambda_min=1e-12,
                 lambda_max=1e12, precision="fp64", manifold="sphere", use_graph=True,
                 series_rtol=0.0, init_seed=0) -> Options:
    o = Options()
    lib().povar_options_default(C.byref(o))
    o.eta, o.series_order, o.max_iters, o.ftol = eta, order, max_iters, ftol
    o.lambda0, o.lambda_min, o.lambda_max = lambda0, lambda_min, lambda_max
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.manifold = MANIFOLD[manifold] if isinstance(manifold, str) else int(manifold)
    o.use_graph = 1 if use_graph else 0
    o.series_rtol = series_rtol
    o.init_seed = int(init_seed)
    return o


def layout_check(cam_idx: np.ndarray, pt_idx: np.ndarray, meas: np.ndarray, n_cams: int, n_pts: int,
                 precision="fp32_bulk") -> dict:
    """Build a problem's device layout on the host and check its invariants
    (``povar_debug_layout_check``; no device needed).  Raises PovarError with
    the violated property."""
    cam = np.ascontiguousarray(cam_idx, dtype=np.int32)
    pt = np.ascontiguousarray(pt_idx, dtype=np.int32)
    m = np.ascontiguousarray(meas, dtype=np.float64).reshape(-1, 2)
    assert cam.shape[0] == pt.shape[0] == m.shape[0]
    out = (C.c_int64 * 8)()
    st = lib().povar_debug_layout_check(n_cams, n_pts, cam.shape[0], _ptr(cam), _ptr(pt), _ptr(m),
                                        PRECISION[precision], out)
    if st != OK:
        raise PovarError(st, lib().povar_last_error(None).decode())
    keys = ("blocked", "n_packets", "n_chunks", "n_slots", "n_runs", "lm_block", "device_bytes", "footprint")
    return dict(zip(keys, (int(v) for v in out)))


def footprint(n_cams: int, n_pts: int, n_obs: int, precision="fp32_bulk") -> int:
    out = C.c_uint64()
    st = lib().povar_problem_footprint(n_cams, n_pts, n_obs, PRECISION[precision], C.byref(out))
    if st != OK:
        raise PovarError(st, "invalid sizes")
    return int(out.value)


def _metric_inputs(cams, K):
    P = np.ascontiguousarray(cams, dtype=np.float64).reshape(-1, 12)
    Km = np.ascontiguousarray(K, dtype=np.float64).reshape(-1, 9)
    if P.shape[0] != Km.shape[0]:
        raise ValueError("cams and K must have one entry per camera")
    return P, Km


def metric_upgrade(ctx: "Context", cams: np.ndarray, K: np.ndarray, max_iters: int = 100,
                   ftol: float = 1e-14, noalloc: bool = False) -> dict:
    """Metric upgrade (``povar_metric_upgrade``, or with noalloc
    ``povar_metric_upgrade_noalloc``): cams (n, 12) or (n, 3, 4) projective
    cameras, K (n, 3, 3) intrinsics.  Returns H (4, 4), c, alpha, R (n, 3, 3),
    t (n, 3), the trace and the report."""
    P, Km = _metric_inputs(cams, K)
    n = P.shape[0]
    out = dict(H=np.empty(16), c=np.empty(3), alpha=np.empty(n), R=np.empty((n, 9)), t=np.empty((n, 3)))
    tc, ta = np.empty(max(max_iters, 1)), np.empty(max(max_iters, 1), dtype=np.int32)
    rep = MetricReport()
    fn = lib().povar_metric_upgrade_noalloc if noalloc else lib().povar_metric_upgrade
    ctx.check(fn(ctx.handle, n, _ptr(P), _ptr(Km), int(max_iters), float(ftol),
                 _ptr(out["H"]), _ptr(out["c"]), _ptr(out["alpha"]), _ptr(out["R"]),
                 _ptr(out["t"]), _ptr(tc), _ptr(ta), C.byref(rep)),
              "povar_metric_upgrade_noalloc" if noalloc else "povar_metric_upgrade")
    out["H"] = out["H"].reshape(4, 4)
    out["R"] = out["R"].reshape(n, 3, 3)
    out.update(trace_cost=tc[:rep.iters].copy(), trace_accept=ta[:rep.iters].astype(bool), iters=rep.iters,
               cost_initial=rep.cost_initial, cost_final=rep.cost_final, lambda_=rep.lambda_, stop=rep.stop)
    return out


def metric_debug_reduced(ctx: "Context", cams: np.ndarray, K: np.ndarray, c) -> dict:
    """The reduced metric-upgrade problem at c: alpha, J^T J, J^T r, cost."""
    P, Km = _metric_inputs(cams, K)
    n = P.shape[0]
    cv = np.ascontiguousarray(c, dtype=np.float64).reshape(3)
    alpha, JtJ, Jtr, cost = np.empty(n), np.empty(9), np.empty(3), C.c_double()
    ctx.check(lib().povar_metric_debug_reduced(ctx.handle, n, _ptr(P), _ptr(Km), _ptr(cv), _ptr(alpha),
                                               _ptr(JtJ), _ptr(Jtr), C.byref(cost)), "povar_metric_debug_reduced")
    return dict(alpha=alpha, JtJ=JtJ.reshape(3, 3), Jtr=Jtr, cost=cost.value)


class Context:
    """A HIP device and the stream all work of its problems runs on.
    stream: None (library-owned stream), an integer hipStream_t, or "torch"
    (torch.cuda.current_stream())."""

    def __init__(self, device: int = 0, stream=None):
        if stream == "torch":
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self.handle = C.c_void_p()
        st = lib().povar_ctx_create(device, C.c_void_p(stream) if stream else None, C.byref(self.handle))
        if st != OK:
            raise PovarError(st, lib().povar_last_error(None).decode())
        self.device = device
        self._problems = weakref.WeakSet()

    def check(self, st: int, what: str = ""):
        if st != OK:
            raise PovarError(st, (what + ": " if what else "") + lib().povar_last_error(self.handle).decode())

    def close(self):
        """Destroys every problem still open on this context, then the context."""
        if self.handle:
            for p in list(self._problems):
                p.close()
            self.check(lib().povar_ctx_destroy(self.handle), "povar_ctx_destroy")
            self.handle = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Problem:
    """One bundle-adjustment problem resident on the GPU."""

    def __init__(self, ctx: Context, n_cams: int, n_pts: int, cam_idx, pt_idx, meas, cams0, **opts):
        self.ctx = ctx
        self.n_cams, self.n_pts = int(n_cams), int(n_pts)
        self.options = make_options(**opts)
        self.handle = C.c_void_p()
        if _is_torch_cuda(cam_idx):
            st = lib().povar_problem_create_device(
                ctx.handle, self.n_cams, self.n_pts, int(cam_idx.shape[0]),
                C.c_void_p(cam_idx.data_ptr()), C.c_void_p(pt_idx.data_ptr()), C.c_void_p(meas.data_ptr()),
                C.c_void_p(cams0.data_ptr()) if cams0 is not None else None, C.byref(self.options),
                C.byref(self.handle))
        else:
            self._cam = np.ascontiguousarray(cam_idx, dtype=np.int32)
            self._pt = np.ascontiguousarray(pt_idx, dtype=np.int32)
            self._meas = np.ascontiguousarray(meas, dtype=np.float64).reshape(-1, 2)
            # cams0 None: the library draws seeded cameras (options init_seed)
            c0 = None if cams0 is None else np.ascontiguousarray(cams0, dtype=np.float64).reshape(self.n_cams, 12)
            st = lib().povar_problem_create(ctx.handle, self.n_cams, self.n_pts, int(self._cam.shape[0]),
                                            _ptr(self._cam), _ptr(self._pt), _ptr(self._meas),
                                            _ptr(c0) if c0 is not None else None,
                                            C.byref(self.options), C.byref(self.handle))
            del self._cam, self._pt, self._meas
        ctx.check(st, "povar_problem_create")
        ctx._problems.add(self)

    @classmethod
    def from_synth(cls, ctx: Context, prob, **opts) -> "Problem":
        opts.setdefault("eta", prob.eta)
        opts.setdefault("order", prob.order)
        return cls(ctx, prob.n_cams, prob.n_pts, prob.cam_idx, prob.pt_idx, prob.meas, prob.cams0, **opts)

    def _chk(self, st, what):
        self.ctx.check(st, what)

    def solve(self) -> dict:
        r = Report()
        self._chk(lib().povar_solve(self.handle, C.byref(r)), "povar_solve")
        return r.as_dict()

    def step(self, n: int) -> dict:
        r = Report()
        self._chk(lib().povar_step(self.handle, int(n), C.byref(r)), "povar_step")
        return r.as_dict()

    def enqueue(self, n: int):
        self._chk(lib().povar_enqueue(self.handle, int(n)), "povar_enqueue")

    def report(self) -> dict:
        r = Report()
        self._chk(lib().povar_get_report(self.handle, C.byref(r)), "povar_get_report")
        return r.as_dict()

    @classmethod
    def refine(cls, ctx: Context, n_cams: int, n_pts: int, cam_idx, pt_idx, meas, cams0, pts0,
               **opts) -> "Problem":
        """A second-stage problem (projective refinement, RiPoBA): cameras and
        homogeneous landmarks (n_pts x 4) refined jointly (povar_refine_create)."""
        self = cls.__new__(cls)
        self.ctx = ctx
        self.n_cams, self.n_pts = int(n_cams), int(n_pts)
        self.options = make_options(**opts)
        self.handle = C.c_void_p()
        cam = np.ascontiguousarray(cam_idx, dtype=np.int32)
        pt = np.ascontiguousarray(pt_idx, dtype=np.int32)
        m = np.ascontiguousarray(meas, dtype=np.float64).reshape(-1, 2)
        c0 = np.ascontiguousarray(cams0, dtype=np.float64).reshape(self.n_cams, 12)
        x0 = np.ascontiguousarray(pts0, dtype=np.float64).reshape(self.n_pts, 4)
        st = lib().povar_refine_create(ctx.handle, self.n_cams, self.n_pts, int(cam.shape[0]), _ptr(cam), _ptr(pt),
                                       _ptr(m), _ptr(c0), _ptr(x0), C.byref(self.options), C.byref(self.handle))
        ctx.check(st, "povar_refine_create")
        ctx._problems.add(self)
        return self

    def points_h(self) -> np.ndarray:
        out = np.empty((self.n_pts, 4))
        self._chk(lib().povar_get_points_h(self.handle, _ptr(out)), "povar_get_points_h")
        return out

    def refine_blocks(self, lam: float) -> dict:
        nc, npt = self.n_cams, self.n_pts
        out = dict(U=np.empty((nc, 12, 12)), bp=np.empty((nc, 12)), G=np.empty((npt, 4, 4)), bl=np.empty((npt, 4)))
        cost = C.c_double()
        self._chk(lib().povar_refine_debug_blocks(self.handle, float(lam), _ptr(out["U"]), _ptr(out["bp"]),
                                                  _ptr(out["G"]), _ptr(out["bl"]), C.byref(cost)),
                  "povar_refine_debug_blocks")
        out["cost"] = cost.value
        return out

    def refine_step(self, lam: float, order: int):
        dp, pt = np.empty((self.n_cams, 12)), np.empty((self.n_cams, 12))
        xt = np.empty((self.n_pts, 4))
        ct = C.c_double()
        self._chk(lib().povar_refine_debug_step(self.handle, float(lam), int(order), _ptr(dp), _ptr(pt), _ptr(xt),
                                                C.byref(ct)), "povar_refine_debug_step")
        return dp, pt, xt, ct.value

    def cameras(self) -> np.ndarray:
        out = np.empty((self.n_cams, 12))
        self._chk(lib().povar_get_cameras(self.handle, _ptr(out)), "povar_get_cameras")
        return out

    def points(self) -> np.ndarray:
        out = np.empty((self.n_pts, 3))
        self._chk(lib().povar_get_points(self.handle, _ptr(out)), "povar_get_points")
        return out

    def trace(self, n: int = 4096):
        it = self.report()["iters"]
        n = min(n, it)
        cost, lam, acc = np.empty(n), np.empty(n), np.empty(n, np.int32)
        if n:
            self._chk(lib().povar_get_trace(self.handle, n, _ptr(cost), _ptr(lam), _ptr(acc)), "povar_get_trace")
        return cost, lam, acc.astype(bool)

    def trace_diag(self, n: int = 4096):
        """Per-iteration |b_l| at the trial point and series seconds."""
        n = min(n, self.report()["iters"])
        bl, ss = np.empty(n), np.empty(n)
        if n:
            self._chk(lib().povar_get_trace_diag(self.handle, n, _ptr(bl), _ptr(ss)), "povar_get_trace_diag")
        return bl, ss

    def debug_series(self, x0, order: int) -> np.ndarray:
        """sum_{t=0..order} M^t x0 at the current linearisation and damping."""
        x = np.ascontiguousarray(x0, dtype=np.float64).reshape(self.n_cams, 12)
        out = np.empty((self.n_cams, 12))
        self._chk(lib().povar_debug_series(self.handle, _ptr(x), int(order), _ptr(out)), "povar_debug_series")
        return out

    def state(self):
        cams = np.empty((self.n_cams, 12))
        lam, it, cost = C.c_double(), C.c_int32(), C.c_double()
        self._chk(lib().povar_get_state(self.handle, _ptr(cams), C.byref(lam), C.byref(it), C.byref(cost)),
                  "povar_get_state")
        return cams, lam.value, it.value, cost.value

    def set_state(self, cams, lam: float, it: int):
        c = np.ascontiguousarray(cams, dtype=np.float64).reshape(self.n_cams, 12)
        self._chk(lib().povar_set_state(self.handle, _ptr(c), float(lam), int(it)), "povar_set_state")

    def debug_linearize(self) -> dict:
        nc, npt = self.n_cams, self.n_pts
        out = dict(U=np.empty((nc, 12, 12)), bp=np.empty((nc, 12)), g=np.empty((nc, 12)),
                   Vp=np.empty((npt, 3, 3)), X=np.empty((npt, 3)), z0=np.empty((npt, 3)))
        cost = C.c_double()
        self._chk(lib().povar_debug_linearize(self.handle, _ptr(out["U"]), _ptr(out["bp"]), _ptr(out["g"]),
                                              _ptr(out["Vp"]), _ptr(out["X"]), _ptr(out["z0"]),
                                              C.byref(cost)), "povar_debug_linearize")
        out["cost"] = cost.value
        return out

    def debug_step(self, lam: float, order: int):
        dp, pt = np.empty((self.n_cams, 12)), np.empty((self.n_cams, 12))
        ct = C.c_double()
        self._chk(lib().povar_debug_step(self.handle, float(lam), int(order), _ptr(dp), _ptr(pt), C.byref(ct)),
                  "povar_debug_step")
        return dp, pt, ct.value

    def debug_camera_blocks(self, lam: float) -> np.ndarray:
        """The damped camera block inverses K_i (n_cams, 12, 12) at damping `lam`."""
        K = np.empty((self.n_cams, 12, 12))
        self._chk(lib().povar_debug_camera_blocks(self.handle, float(lam), _ptr(K)), "povar_debug_camera_blocks")
        return K

    def kernel_timing(self, enable: bool):
        self._chk(lib().povar_kernel_timing(self.handle, 1 if enable else 0), "povar_kernel_timing")

    def kernel_times(self) -> dict:
        ml, mc = C.c_double(), C.c_double()
        nl, nc = C.c_int64(), C.c_int64()
        self._chk(lib().povar_kernel_times(self.handle, C.byref(ml), C.byref(nl), C.byref(mc), C.byref(nc)),
                  "povar_kernel_times")
        return dict(ms_landmark_pass=ml.value, n_landmark_pass=nl.value,
                    ms_camera_pass=mc.value, n_camera_pass=nc.value)

    def info(self) -> dict:
        a, b, d = C.c_int64(), C.c_int64(), C.c_uint64()
        c = C.c_int32()
        self._chk(lib().povar_problem_info(self.handle, C.byref(a), C.byref(b), C.byref(c), C.byref(d)),
                  "povar_problem_info")
        return dict(n_obs=a.value, n_packets=b.value, n_chunks=c.value, device_bytes=d.value)

    def layout(self) -> dict:
        b, lb, nh = C.c_int32(), C.c_int32(), C.c_int32()
        ns, nr = C.c_int64(), C.c_int64()
        self._chk(lib().povar_problem_layout(self.handle, C.byref(b), C.byref(lb), C.byref(ns), C.byref(nr),
                                             C.byref(nh)), "povar_problem_layout")
        return dict(blocked=bool(b.value), lm_block=lb.value, n_slots=ns.value, n_runs=nr.value,
                    coop_gather=bool(nh.value))

    def close(self):
        if self.handle:
            lib().povar_problem_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (povar_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int):
        self.ctx = ctx
        self.handle = C.c_void_p()
        ctx.check(lib().povar_server_create(ctx.handle, int(hbm_budget_bytes), int(max_slots),
                                            C.byref(self.handle)), "povar_server_create")
        self._sizes = {}

    def submit(self, prob, **opts) -> int:
        opts.setdefault("eta", prob.eta)
        opts.setdefault("order", prob.order)
        opts.setdefault("max_iters", prob.iters)
        o = make_options(**opts)
        cam = np.ascontiguousarray(prob.cam_idx, np.int32)
        pt = np.ascontiguousarray(prob.pt_idx, np.int32)
        meas = np.ascontiguousarray(prob.meas, np.float64)
        c0 = np.ascontiguousarray(prob.cams0, np.float64)
        t = C.c_uint64()
        st = lib().povar_server_submit(self.handle, prob.n_cams, prob.n_pts, cam.shape[0], _ptr(cam), _ptr(pt),
                                       _ptr(meas), _ptr(c0), C.byref(o), C.byref(t))
        self.ctx.check(st, "povar_server_submit")
        self._sizes[t.value] = (prob.n_cams, prob.n_pts)
        return t.value

    def poll(self, ticket: int):
        """None while running; else (report, cameras, points, times)."""
        nc, npt = self._sizes[ticket]
        cams, pts, times = np.empty((nc, 12)), np.empty((npt, 3)), np.empty(3)
        r = Report()
        st = lib().povar_server_poll(self.handle, ticket, C.byref(r), _ptr(cams), _ptr(pts), _ptr(times))
        if st == EAGAIN:
            return None
        self.ctx.check(st, "povar_server_poll")
        del self._sizes[ticket]
        return r.as_dict(), cams, pts, times

    def stats(self) -> dict:
        q, a = C.c_int32(), C.c_int32()
        f, b = C.c_int64(), C.c_int64()
        self.ctx.check(lib().povar_server_stats(self.handle, C.byref(q), C.byref(a), C.byref(f), C.byref(b)),
                       "povar_server_stats")
        return dict(queued=q.value, active=a.value, finished=f.value, batch_iters=b.value)

    def profile(self) -> dict:
        sec, cnt = (C.c_double * 4)(), (C.c_int64 * 3)()
        self.ctx.check(lib().povar_server_profile(self.handle, sec, cnt), "povar_server_profile")
        return dict(admit_s=sec[0], launch_s=sec[1], wait_s=sec[2], retire_s=sec[3], batch_iters=cnt[0],
                    readbacks=cnt[1], budget_waits=cnt[2])

    def close(self):
        if self.handle:
            lib().povar_server_destroy(self.handle)
            self.handle = C.c_void_p()


def _is_torch_cuda(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)
