"""Python binding of libksdf (argument marshalling only).

Every step of the fit, the query and the backward runs in the library's HIP
kernels; PyTorch provides device memory and the stream.  There is no fallback:
if ``libksdf.so`` is missing or no GPU is present, the calls raise.

    cells = build_cells(points_np, origin, h, margin, m_max, m_min)
    model = Model(cells, n_points, origin, h, ell=0.2, noise_var=1e-4)
    model.fit(points_cuda)
    out = model.query(queries_cuda, sign_cuda)      # mean, grad, var, var_f, argmin, status
    mean, grad, var, var_f = sdf(model, queries_cuda, sign=sign_cuda, theta=theta)  # autograd
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libksdf.so")

FP64, FP32 = 0, 1
DTYPE_F32, DTYPE_F64 = 0, 1
Q_NO_VALID_CELL, Q_CLAMPED, Q_GRAD_ZERO, Q_OUTSIDE_INDEX, Q_FIT_TIMEOUT = 1, 2, 4, 8, 16
C_FP64, C_FAILED = 1, 2
FIT_ADJOINT, FIT_ADJOINT_VARF, FIT_DENSE_INV = 1, 2, 4

EXPORTS = ["ksdf_build_cells", "ksdf_cellset_info", "ksdf_cellset_copy", "ksdf_cellset_destroy",
           "ksdf_model_bytes", "ksdf_model_create", "ksdf_model_index_bytes",
           "ksdf_model_attach_index", "ksdf_model_destroy", "ksdf_model_info", "ksdf_fit_cells",
           "ksdf_query_workspace_bytes", "ksdf_query", "ksdf_query_noalloc",
           "ksdf_backward_workspace_bytes",
           "ksdf_query_bucket", "ksdf_query_bucketed", "ksdf_query_backward", "ksdf_cost_backward", "ksdf_fit_query_workspace_bytes",
           "ksdf_fit_query",
           "ksdf_model_set_tuning", "ksdf_model_get_tuning", "ksdf_model_set_timing",
           "ksdf_model_timer_read", "ksdf_refit_workspace_bytes", "ksdf_refit_cells",
           "ksdf_count_queries_workspace_bytes", "ksdf_count_queries", "ksdf_model_check",
           "ksdf_model_set_wait_limit", "ksdf_bhm_sign", "ksdf_bhm_tau_workspace_bytes",
           "ksdf_bhm_update_tau", "ksdf_status_string",
           "ksdf_last_error"]


class KsdfError(RuntimeError):
    pass


TIMERS = {"fit": 0, "query": 1, "backward": 2, "fused": 3}
TIMER_SLOTS = 8


class Tuning(ctypes.Structure):
    _fields_ = [("query_sub", ctypes.c_int), ("query_block", ctypes.c_int),
                ("fused", ctypes.c_int), ("fit_min_bucket", ctypes.c_int),
                ("query_split", ctypes.c_int), ("query_lanes", ctypes.c_int),
                ("backward_lanes", ctypes.c_int),
                ("query_pairs", ctypes.c_int), ("query_mfma", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


KERNELS = {"rbf": 0, "matern32": 1}   # KSDF_KERNEL_* (Table I)


class BhmLayout(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("box", ctypes.c_double),
                ("dims", ctypes.c_int * 3), ("hinges", ctypes.c_int), ("gamma", ctypes.c_double)]


def _bhm_layout(origin, box, dims, hinges, gamma):
    return BhmLayout((ctypes.c_double * 3)(*map(float, origin)), float(box),
                     (ctypes.c_int * 3)(*map(int, dims)), int(hinges), float(gamma))


def bhm_sign(points: torch.Tensor, origin, box, dims, hinges, gamma, box_bhm: torch.Tensor,
             weights: torch.Tensor, tau: float = 0.0, logodds=False, stream=None):
    """Sign of the SDF from local BHM weights (eq. sign_prediction): int8 [Q] (+1 free),
    and with logodds=True also the log-odds l [Q] (float64)."""
    if box_bhm.dtype != torch.int32 or weights.dtype != torch.float64:
        raise ValueError("box_bhm must be int32 and weights float64")
    Q = len(points)
    sign = torch.empty(Q, dtype=torch.int8, device=points.device)
    lo = torch.empty(Q, dtype=torch.float64, device=points.device) if logodds else None
    dt = DTYPE_F64 if points.dtype == torch.float64 else DTYPE_F32
    lay = _bhm_layout(origin, box, dims, hinges, gamma)
    _check(lib().ksdf_bhm_sign(ctypes.byref(lay), _ptr(box_bhm), _ptr(weights), _ptr(points), dt, Q,
                               float(tau), _ptr(sign), _ptr(lo), _stream(stream)), "ksdf_bhm_sign")
    return (sign, lo) if logodds else sign


def bhm_update_tau(hits: torch.Tensor, origin, box, dims, hinges, gamma, box_bhm: torch.Tensor,
                   weights: torch.Tensor, alpha: float, tau: torch.Tensor, stream=None):
    """tau <- (1 - alpha) tau + alpha * mean l(hits), in place (device float64 [1])."""
    K = len(hits)
    nb = lib().ksdf_bhm_tau_workspace_bytes(K)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=hits.device)
    dt = DTYPE_F64 if hits.dtype == torch.float64 else DTYPE_F32
    lay = _bhm_layout(origin, box, dims, hinges, gamma)
    _check(lib().ksdf_bhm_update_tau(ctypes.byref(lay), _ptr(box_bhm), _ptr(weights), _ptr(hits), dt,
                                     K, float(alpha), _ptr(tau), _ptr(ws), nb, _stream(stream)),
           "ksdf_bhm_update_tau")


class Hyper(ctypes.Structure):
    _fields_ = [("ell", ctypes.c_double), ("noise_var", ctypes.c_double),
                ("alpha", ctypes.c_double), ("k_fuse", ctypes.c_int),
                ("precision", ctypes.c_int), ("cond_fp64_threshold", ctypes.c_double),
                ("flags", ctypes.c_int), ("kernel", ctypes.c_int)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load libksdf.so; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise KsdfError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        i, l, d, sz = ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_size_t
        pi = ctypes.POINTER(ctypes.c_int)
        pl = ctypes.POINTER(ctypes.c_long)
        pd = ctypes.POINTER(ctypes.c_double)
        psz = ctypes.POINTER(ctypes.c_size_t)
        H = ctypes.POINTER(Hyper)
        L.ksdf_build_cells.argtypes = [_vp, i, l, pd, d, d, i, i, _vp, pi, pi, ctypes.POINTER(_vp)]
        L.ksdf_cellset_info.argtypes = [_vp, pi, pl]
        L.ksdf_cellset_copy.argtypes = [_vp, _vp, _vp, _vp]
        L.ksdf_cellset_destroy.argtypes = [_vp]
        L.ksdf_cellset_destroy.restype = None
        L.ksdf_model_bytes.argtypes = [i, _vp, _vp, _vp, pd, d, l, H, pd, pd]
        L.ksdf_model_bytes.restype = sz
        L.ksdf_model_create.argtypes = [i, _vp, _vp, _vp, pd, d, l, H, pd, pd, _vp, sz, _vp,
                                        ctypes.POINTER(_vp)]
        L.ksdf_model_index_bytes.argtypes = [_vp]
        L.ksdf_model_index_bytes.restype = sz
        L.ksdf_model_attach_index.argtypes = [_vp, _vp, sz, _vp]
        L.ksdf_model_destroy.argtypes = [_vp]
        L.ksdf_model_destroy.restype = None
        L.ksdf_model_info.argtypes = [_vp, pi, pl, pi, pl, psz]
        L.ksdf_fit_cells.argtypes = [_vp, _vp, i, l, _vp, H, _vp, _vp]
        L.ksdf_query_workspace_bytes.argtypes = [_vp, l]
        L.ksdf_query_workspace_bytes.restype = sz
        L.ksdf_query.argtypes = [_vp, _vp, l, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, sz,
                                 _vp]
        L.ksdf_query_noalloc.argtypes = [_vp, _vp, l, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.ksdf_query_bucket.argtypes = [_vp, _vp, l, _vp, sz, _vp]
        L.ksdf_query_bucketed.argtypes = [_vp, _vp, l, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                          sz, _vp]
        L.ksdf_backward_workspace_bytes.argtypes = [_vp, l]
        L.ksdf_backward_workspace_bytes.restype = sz
        L.ksdf_query_backward.argtypes = [_vp, _vp, l, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                          _vp, sz, _vp]
        L.ksdf_cost_backward.argtypes = [_vp, _vp, l, _vp, _vp, _vp, _vp, ctypes.c_double,
                                         ctypes.c_double, _vp, _vp, _vp, _vp, sz, _vp]
        L.ksdf_fit_query_workspace_bytes.argtypes = [_vp, l]
        L.ksdf_fit_query_workspace_bytes.restype = sz
        L.ksdf_fit_query.argtypes = [_vp, _vp, i, l, _vp, H, _vp, _vp, l, _vp, _vp, _vp, _vp, _vp,
                                     _vp, _vp, _vp, _vp, sz, _vp]
        L.ksdf_refit_workspace_bytes.argtypes = [_vp, i]
        L.ksdf_refit_workspace_bytes.restype = sz
        L.ksdf_refit_cells.argtypes = [_vp, _vp, i, l, _vp, _vp, _vp, ctypes.c_double, i, _vp, _vp,
                                       _vp, _vp, sz, _vp]
        L.ksdf_count_queries_workspace_bytes.argtypes = [_vp]
        L.ksdf_count_queries_workspace_bytes.restype = sz
        L.ksdf_count_queries.argtypes = [_vp, _vp, l, _vp, ctypes.c_float, _vp, sz, _vp]
        L.ksdf_model_check.argtypes = [_vp, _vp]
        L.ksdf_model_set_wait_limit.argtypes = [_vp, l]
        L.ksdf_bhm_sign.argtypes = [ctypes.POINTER(BhmLayout), _vp, _vp, _vp, i, l, d, _vp, _vp, _vp]
        L.ksdf_bhm_tau_workspace_bytes.argtypes = [l]
        L.ksdf_bhm_tau_workspace_bytes.restype = sz
        L.ksdf_bhm_update_tau.argtypes = [ctypes.POINTER(BhmLayout), _vp, _vp, _vp, i, l, d, _vp,
                                          _vp, sz, _vp]
        L.ksdf_model_set_tuning.argtypes = [_vp, ctypes.POINTER(Tuning)]
        L.ksdf_model_get_tuning.argtypes = [_vp, ctypes.POINTER(Tuning)]
        L.ksdf_model_set_timing.argtypes = [_vp, i]
        L.ksdf_model_timer_read.argtypes = [_vp, i, ctypes.POINTER(ctypes.c_float), i,
                                            ctypes.POINTER(ctypes.c_int)]
        L.ksdf_status_string.argtypes = [i]
        L.ksdf_status_string.restype = ctypes.c_char_p
        L.ksdf_last_error.argtypes = []
        L.ksdf_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        L = lib()
        raise KsdfError(f"{what}: {L.ksdf_status_string(rc).decode()} ({rc}): "
                        f"{L.ksdf_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _d3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


@dataclasses.dataclass
class CellSet:
    offsets: np.ndarray   # int32 [n+1]
    samples: np.ndarray   # int32 [nnz]
    keys: np.ndarray      # int32 [n,3]

    @property
    def n(self):
        return len(self.offsets) - 1

    @property
    def m(self):
        return np.diff(self.offsets)


def build_cells(points, origin, h, margin, m_max, m_min, cap_grid=None, key_lo=(0, 0, 0)) -> CellSet:
    """Host cell builder (the per-octant training buffers with overlapping boxes)."""
    L = lib()
    pts = np.ascontiguousarray(points)
    if pts.dtype not in (np.float32, np.float64) or pts.ndim != 2 or pts.shape[1] != 3:
        raise ValueError("points must be [N,3] float32 or float64")
    dt = DTYPE_F64 if pts.dtype == np.float64 else DTYPE_F32
    cg = None if cap_grid is None else np.ascontiguousarray(cap_grid, dtype=np.uint8)
    klo = (ctypes.c_int * 3)(*[int(v) for v in key_lo])
    kd = (ctypes.c_int * 3)(*(cg.shape if cg is not None else (0, 0, 0)))
    hdl = ctypes.c_void_p()
    _check(L.ksdf_build_cells(pts.ctypes.data, dt, len(pts), _d3(origin), float(h), float(margin),
                              int(m_max), int(m_min), None if cg is None else cg.ctypes.data,
                              klo, kd, ctypes.byref(hdl)), "ksdf_build_cells")
    try:
        n, nnz = ctypes.c_int(), ctypes.c_long()
        _check(L.ksdf_cellset_info(hdl, ctypes.byref(n), ctypes.byref(nnz)), "ksdf_cellset_info")
        off = np.zeros(n.value + 1, np.int32)
        smp = np.zeros(max(nnz.value, 1), np.int32)
        keys = np.zeros((max(n.value, 1), 3), np.int32)
        _check(L.ksdf_cellset_copy(hdl, off.ctypes.data, smp.ctypes.data, keys.ctypes.data),
               "ksdf_cellset_copy")
    finally:
        L.ksdf_cellset_destroy(hdl)
    return CellSet(off, smp[:nnz.value], keys[:n.value])


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Model:
    """A fitted set of local GPs.  Its device memory (the per-cell store and the
    candidate lists) is two torch tensors this object owns; the library only holds
    views into them."""

    def __init__(self, cells: CellSet, n_points: int, origin, h: float, ell: float = 0.2,
                 noise_var: float = 1e-4, k_fuse: int = 8, precision: str = "fp32",
                 alpha: Optional[float] = None, cond_threshold: float = 1e6, query_box=None,
                 adjoint: bool = False, adjoint_var_f: bool = False, kernel: str = "rbf",
                 dense_inverse: bool = False, stream=None):
        if not torch.cuda.is_available():
            raise KsdfError("no GPU: libksdf needs a gfx950 device")
        self._lib = lib()
        self._h = ctypes.c_void_p()
        self.cells = cells
        self.n_points = int(n_points)
        self.origin = tuple(float(v) for v in origin)
        self.h = float(h)
        self.precision = FP64 if precision == "fp64" else FP32
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        flags = ((FIT_ADJOINT if adjoint or adjoint_var_f else 0) |
                 (FIT_ADJOINT_VARF if adjoint_var_f else 0) | (FIT_DENSE_INV if dense_inverse else 0))
        if kernel not in KERNELS:
            raise ValueError(f"kernel must be one of {sorted(KERNELS)}")
        self.kernel = kernel
        self.dense_inverse = bool(dense_inverse)
        self.hyper = Hyper(float(ell), float(noise_var), -1.0 if alpha is None else float(alpha),
                           int(k_fuse), self.precision, float(cond_threshold), flags,
                           KERNELS[kernel])
        self.device = torch.device("cuda", torch.cuda.current_device())
        qlo = qhi = None
        if query_box is not None:
            qlo, qhi = _d3(query_box[0]), _d3(query_box[1])
        off = np.ascontiguousarray(cells.offsets, np.int32)
        smp = np.ascontiguousarray(cells.samples, np.int32)
        keys = np.ascontiguousarray(cells.keys, np.int32)
        args = (cells.n, off.ctypes.data, smp.ctypes.data, keys.ctypes.data, _d3(origin), self.h,
                self.n_points, ctypes.byref(self.hyper), qlo, qhi)
        nb = self._lib.ksdf_model_bytes(*args)
        # the store and the candidate lists are caller-owned device memory
        self._store = torch.empty(max(nb, 1), dtype=torch.uint8, device=self.device)
        _check(self._lib.ksdf_model_create(*args, _ptr(self._store), nb, _stream(stream),
                                           ctypes.byref(self._h)), "ksdf_model_create")
        ib = self._lib.ksdf_model_index_bytes(self._h)
        self._index = torch.empty(ib, dtype=torch.uint8, device=self.device)
        _check(self._lib.ksdf_model_attach_index(self._h, _ptr(self._index), ib, _stream(stream)),
               "ksdf_model_attach_index")
        self._ws = None
        self.points = None
        self.sample_var = None

    @property
    def n_cells(self):
        return self.cells.n

    def info(self) -> dict:
        n, nnz, mm, ie, db = (ctypes.c_int(), ctypes.c_long(), ctypes.c_int(), ctypes.c_long(),
                              ctypes.c_size_t())
        _check(self._lib.ksdf_model_info(self._h, ctypes.byref(n), ctypes.byref(nnz),
                                         ctypes.byref(mm), ctypes.byref(ie), ctypes.byref(db)),
               "ksdf_model_info")
        return dict(n_cells=n.value, nnz=nnz.value, max_m=mm.value, index_entries=ie.value,
                    device_bytes=db.value)

    def tuning(self) -> dict:
        t = Tuning()
        _check(self._lib.ksdf_model_get_tuning(self._h, ctypes.byref(t)), "ksdf_model_get_tuning")
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning(**{**self.tuning(), **kw})
        _check(self._lib.ksdf_model_set_tuning(self._h, ctypes.byref(t)), "ksdf_model_set_tuning")

    def set_timing(self, on: bool = True):
        """Record HIP events around each phase's main kernel (off under graph capture)."""
        _check(self._lib.ksdf_model_set_timing(self._h, int(bool(on))), "ksdf_model_set_timing")

    def timer_read(self, phase: str) -> list:
        """Durations (ms, in launch order) of the launches of 'fit', 'query', 'backward'
        or 'fused' since the previous read."""
        buf = (ctypes.c_float * TIMER_SLOTS)()
        n = ctypes.c_int()
        _check(self._lib.ksdf_model_timer_read(self._h, TIMERS[phase], buf, TIMER_SLOTS,
                                               ctypes.byref(n)), "ksdf_model_timer_read")
        return [buf[i] for i in range(n.value)]

    def set_hyper(self, ell=None, noise_var=None, alpha=None):
        if ell is not None:
            self.hyper.ell = float(ell)
        if noise_var is not None:
            self.hyper.noise_var = float(noise_var)
        if alpha is not None:
            self.hyper.alpha = float(alpha)

    def fit(self, points: torch.Tensor, sample_var: Optional[torch.Tensor] = None,
            cell_status: Optional[torch.Tensor] = None, stream=None) -> None:
        if not points.is_cuda or points.dim() != 2 or points.shape[1] != 3 or not points.is_contiguous():
            raise ValueError("points must be a contiguous [N,3] CUDA tensor")
        if points.dtype not in (torch.float32, torch.float64):
            raise ValueError("points must be float32 or float64")
        dt = DTYPE_F64 if points.dtype == torch.float64 else DTYPE_F32
        if sample_var is not None and (sample_var.dtype != points.dtype or sample_var.numel() != len(points)):
            raise ValueError("sample_var must match the points' dtype and count")
        if cell_status is not None and (cell_status.dtype != torch.uint8 or cell_status.numel() < self.n_cells):
            raise ValueError("cell_status must be uint8 [n_cells]")
        _check(self._lib.ksdf_fit_cells(self._h, _ptr(points), dt, len(points), _ptr(sample_var),
                                        ctypes.byref(self.hyper), _ptr(cell_status),
                                        _stream(stream)), "ksdf_fit_cells")
        self.points = points
        self.sample_var = sample_var

    def _workspace(self, nbytes: int, given: Optional[torch.Tensor] = None):
        if given is not None:
            # caller-owned scratch, e.g. one per stream for calls that run concurrently
            if given.dtype != torch.uint8 or not given.is_cuda or given.numel() < nbytes:
                raise ValueError(f"workspace must be a uint8 CUDA tensor of at least {nbytes} bytes")
            return given
        if nbytes == 0:
            return None
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def new_workspace(self, Q: int) -> torch.Tensor:
        """Scratch for query() and backward() of up to Q points.  Calls on several
        streams at once each need their own (by default every call shares one)."""
        nb = max(self._lib.ksdf_query_workspace_bytes(self._h, Q),
                 self._lib.ksdf_backward_workspace_bytes(self._h, Q), 1)
        return torch.empty(nb, dtype=torch.uint8, device=self.device)

    def bucket(self, points: torch.Tensor, stream=None,
               workspace: Optional[torch.Tensor] = None):
        """The first step of query() alone (ksdf_query_bucket): sorts the points into the
        workspace; it does not read the fit, so it may run beside fit() on another
        stream.  query(..., bucketed=True) with the same points and workspace finishes."""
        if points.dtype != self.dtype or not points.is_cuda or not points.is_contiguous() \
                or points.dim() != 2 or points.shape[1] != 3:
            raise ValueError(f"points must be a contiguous [Q,3] CUDA {self.dtype} tensor")
        Q = len(points)
        nb = self._lib.ksdf_query_workspace_bytes(self._h, Q)
        ws = self._workspace(nb, workspace)
        _check(self._lib.ksdf_query_bucket(self._h, _ptr(points), Q, _ptr(ws), nb, _stream(stream)),
               "ksdf_query_bucket")

    def query(self, points: torch.Tensor, sign: Optional[torch.Tensor] = None, var_f=True,
              argmin=True, status=True, grad_var=False, out: Optional[dict] = None,
              stream=None, workspace: Optional[torch.Tensor] = None, bucketed=False) -> dict:
        """Per-query outputs: mean, grad [Q,3], var, and optionally var_f, argmin, status
        and grad_var [Q,3] (the variance of each gradient component, App. C).  bucketed:
        the workspace already holds bucket()'s sort of these points."""
        if points.dtype != self.dtype or not points.is_cuda or not points.is_contiguous() \
                or points.dim() != 2 or points.shape[1] != 3:
            raise ValueError(f"points must be a contiguous [Q,3] CUDA {self.dtype} tensor")
        if sign is not None and (sign.dtype != torch.int8 or sign.numel() != len(points)):
            raise ValueError("sign must be int8 [Q]")
        Q = len(points)
        if out is None:
            out = self._out(Q, points.device, var_f, argmin, status, grad_var)
        nb = self._lib.ksdf_query_workspace_bytes(self._h, Q)
        ws = self._workspace(nb, workspace)
        fn = self._lib.ksdf_query_bucketed if bucketed else self._lib.ksdf_query
        _check(fn(self._h, _ptr(points), Q, _ptr(sign), _ptr(out["mean"]),
                  _ptr(out["grad"]), _ptr(out["var"]), _ptr(out.get("var_f")),
                  _ptr(out.get("grad_var")), _ptr(out.get("argmin")), _ptr(out.get("status")), _ptr(ws), nb,
                  _stream(stream)), "ksdf_query_bucketed" if bucketed else "ksdf_query")
        return out

    def _out(self, Q, device, var_f=True, argmin=True, status=True, grad_var=False):
        dt = self.dtype
        out = dict(mean=torch.empty(Q, dtype=dt, device=device),
                   grad=torch.empty(Q, 3, dtype=dt, device=device),
                   var=torch.empty(Q, dtype=dt, device=device))
        if var_f:
            out["var_f"] = torch.empty(Q, dtype=dt, device=device)
        if argmin:
            out["argmin"] = torch.empty(Q, dtype=torch.int32, device=device)
        if status:
            out["status"] = torch.empty(Q, dtype=torch.uint8, device=device)
        if grad_var:
            out["grad_var"] = torch.empty(Q, 3, dtype=dt, device=device)
        return out

    def fit_query(self, points: torch.Tensor, queries: torch.Tensor, sign=None, sample_var=None,
                  cell_status=None, grad_var=False, out: Optional[dict] = None,
                  stream=None) -> dict:
        """Fit and query in one persistent fused launch (FP32 models)."""
        if not points.is_cuda or points.dim() != 2 or points.shape[1] != 3 or not points.is_contiguous():
            raise ValueError("points must be a contiguous [N,3] CUDA tensor")
        if queries.dtype != self.dtype or not queries.is_contiguous() or queries.shape[-1] != 3:
            raise ValueError(f"queries must be a contiguous [Q,3] CUDA {self.dtype} tensor")
        dt = DTYPE_F64 if points.dtype == torch.float64 else DTYPE_F32
        Q = len(queries)
        out = out if out is not None else self._out(Q, queries.device, grad_var=grad_var)
        nb = self._lib.ksdf_fit_query_workspace_bytes(self._h, Q)
        ws = self._workspace(nb)
        _check(self._lib.ksdf_fit_query(self._h, _ptr(points), dt, len(points), _ptr(sample_var),
                                        ctypes.byref(self.hyper), _ptr(cell_status), _ptr(queries), Q,
                                        _ptr(sign), _ptr(out["mean"]), _ptr(out["grad"]),
                                        _ptr(out["var"]), _ptr(out.get("var_f")),
                                        _ptr(out.get("grad_var")), _ptr(out.get("argmin")), _ptr(out.get("status")), _ptr(ws), nb,
                                        _stream(stream)), "ksdf_fit_query")
        self.points = points
        self.sample_var = sample_var
        return out

    def backward(self, points, sign, d_mean, d_grad=None, d_var=None, d_var_f=None, argmin=None,
                 stream=None, workspace: Optional[torch.Tensor] = None):
        """VJP: (d_points [Q,3], d_hyper [2] float64 = dL/d(ell, noise_var))."""
        Q = len(points)
        d_points = torch.empty(Q, 3, dtype=self.dtype, device=points.device)
        d_hyper = torch.empty(2, dtype=torch.float64, device=points.device)
        nb = self._lib.ksdf_backward_workspace_bytes(self._h, Q)
        ws = self._workspace(nb, workspace)
        c = [None if t is None else t.contiguous() for t in (d_mean, d_grad, d_var, d_var_f)]
        for t in c:
            if t is not None and t.dtype != self.dtype:
                raise ValueError("cotangents must match the model dtype")
        if argmin is not None and (argmin.dtype != torch.int32 or argmin.numel() != Q):
            raise ValueError("argmin must be int32 [Q]")
        _check(self._lib.ksdf_query_backward(self._h, _ptr(points), Q, _ptr(sign), _ptr(argmin),
                                             *[_ptr(t) for t in c], _ptr(d_points), _ptr(d_hyper),
                                             _ptr(ws), nb, _stream(stream)), "ksdf_query_backward")
        return d_points, d_hyper

    def cost_backward(self, points, sign, mean, var, argmin=None, margin: float = 0.3,
                      kvar: float = 1.0, cost: Optional[torch.Tensor] = None, stream=None,
                      workspace: Optional[torch.Tensor] = None):
        """Gradient of the softplus margin cost sum softplus(margin - mean + kvar sqrt(var))
        of a query's outputs: (d_points [Q,3], d_hyper [2] float64); the per-point cost
        goes to `cost` ([Q], model dtype) when given."""
        Q = len(points)
        d_points = torch.empty(Q, 3, dtype=self.dtype, device=points.device)
        d_hyper = torch.empty(2, dtype=torch.float64, device=points.device)
        nb = self._lib.ksdf_backward_workspace_bytes(self._h, Q)
        ws = self._workspace(nb, workspace)
        for t in (mean, var, cost):
            if t is not None and (t.dtype != self.dtype or t.numel() != Q or not t.is_contiguous()):
                raise ValueError("mean, var and cost must be contiguous [Q] tensors of the model dtype")
        if argmin is not None and (argmin.dtype != torch.int32 or argmin.numel() != Q):
            raise ValueError("argmin must be int32 [Q]")
        _check(self._lib.ksdf_cost_backward(self._h, _ptr(points), Q, _ptr(sign), _ptr(argmin),
                                            _ptr(mean), _ptr(var), float(margin), float(kvar),
                                            _ptr(cost), _ptr(d_points), _ptr(d_hyper), _ptr(ws), nb,
                                            _stream(stream)), "ksdf_cost_backward")
        return d_points, d_hyper

    def refit(self, points: torch.Tensor, dirty: torch.Tensor, qcount: torch.Tensor, eta: float,
              budget: int, sample_var=None, cell_status=None, stream=None):
        """Streaming refit (App. G): refit the min(budget, #dirty) cells of highest
        priority dirty * (1 + eta * qcount); resets their dirty counts and halves their
        query counts in place.  Returns (refit_cells int32 [min(budget, n_cells)],
        n_refit int32 [1]) on the device."""
        for t in (dirty, qcount):
            if t.dtype != torch.float32 or not t.is_cuda or t.numel() != self.n_cells:
                raise ValueError("dirty and qcount must be float32 CUDA tensors of n_cells")
        dt = DTYPE_F64 if points.dtype == torch.float64 else DTYPE_F32
        cells = torch.empty(max(min(int(budget), self.n_cells), 1), dtype=torch.int32,
                            device=points.device)
        n = torch.empty(1, dtype=torch.int32, device=points.device)
        nb = self._lib.ksdf_refit_workspace_bytes(self._h, int(budget))
        ws = self._workspace(nb)
        _check(self._lib.ksdf_refit_cells(self._h, _ptr(points), dt, len(points), _ptr(sample_var),
                                          _ptr(dirty), _ptr(qcount), float(eta), int(budget),
                                          _ptr(cells), _ptr(n), _ptr(cell_status), _ptr(ws), nb,
                                          _stream(stream)), "ksdf_refit_cells")
        return cells, n

    def count_queries(self, argmin: torch.Tensor, qcount: torch.Tensor, cap: float = 10000.0,
                      stream=None, workspace: Optional[torch.Tensor] = None):
        """App. G query counters: qcount[c] = min(qcount[c] + #(argmin == c), cap) for
        the valid argmin cells, one rounding per cell."""
        if argmin.dtype != torch.int32 or qcount.dtype != torch.float32:
            raise ValueError("argmin must be int32 and qcount float32")
        if not qcount.is_cuda or qcount.numel() != self.n_cells:
            raise ValueError("qcount must be a float32 CUDA tensor of n_cells")
        nb = self._lib.ksdf_count_queries_workspace_bytes(self._h)
        ws = self._workspace(nb, workspace)
        _check(self._lib.ksdf_count_queries(self._h, _ptr(argmin), argmin.numel(), _ptr(qcount),
                                            float(cap), _ptr(ws), nb, _stream(stream)),
               "ksdf_count_queries")

    def check(self, stream=None):
        """Raise if a fused fit+query launch stopped waiting for the fits since the last
        check (its queries carry Q_FIT_TIMEOUT); synchronises the stream."""
        _check(self._lib.ksdf_model_check(self._h, _stream(stream)), "ksdf_model_check")

    def set_wait_limit(self, sleeps: int):
        """Bound of the fused launch's wait for the fits, in sleeps (0: the default)."""
        _check(self._lib.ksdf_model_set_wait_limit(self._h, int(sleeps)), "ksdf_model_set_wait_limit")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            # launches may still read the store: let them finish before it is released
            torch.cuda.synchronize(self.device)
            self._lib.ksdf_model_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._store = self._index = self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _SDF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, points, theta, model: Model, sign):
        ctx.set_materialize_grads(False)
        if theta is not None:
            model.set_hyper(ell=float(theta[0]), noise_var=float(theta[1]))
            model.fit(model.points, model.sample_var)
        out = model.query(points.detach().contiguous(), sign, argmin=True, status=False)
        ctx.model = model
        ctx.sign = sign
        ctx.has_theta = theta is not None
        ctx.save_for_backward(points, out["argmin"])
        return out["mean"], out["grad"], out["var"], out["var_f"]

    @staticmethod
    def backward(ctx, g_mean, g_grad, g_var, g_var_f):
        points, argmin = ctx.saved_tensors
        m = ctx.model
        z = lambda g: None if g is None else g.contiguous()  # noqa: E731
        gm = g_mean if g_mean is not None else torch.zeros(len(points), dtype=m.dtype, device=points.device)
        d_points, d_hyper = m.backward(points.detach().contiguous(), ctx.sign, z(gm), z(g_grad),
                                       z(g_var), z(g_var_f), argmin=argmin)
        return d_points, (d_hyper if ctx.has_theta else None), None, None


def sdf(model: Model, points: torch.Tensor, sign: Optional[torch.Tensor] = None,
        theta: Optional[torch.Tensor] = None):
    """Differentiable (mean, grad, var, var_f).  With theta = tensor([ell, noise_var])
    (float64, requires_grad), the model is refitted at theta and dL/dtheta flows back."""
    return _SDF.apply(points, theta, model, sign)
