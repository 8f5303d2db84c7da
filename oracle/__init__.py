"""FP64 CPU oracle for the local-GP SDF back-end (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP path.  The arithmetic lives
in ``ksdf_oracle.cpp`` (plain C++17, double precision, OpenMP over independent
cells and queries); this module compiles it with g++ and marshals arrays.
``tiny_dense`` holds an independent NumPy/SciPy dense-GP check for tiny inputs.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ksdf_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

KERNELS = {"rbf": 0, "matern32": 1}   # Table I

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i8p = ctypes.POINTER(ctypes.c_int8)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_cells_build.restype = ctypes.c_void_p
        L.oracle_cells_build.argtypes = [_dp, ctypes.c_long, _dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, _u8p, _ip, _ip]
        L.oracle_cells_count.restype = ctypes.c_int
        L.oracle_cells_count.argtypes = [ctypes.c_void_p, _lp]
        L.oracle_cells_copy.argtypes = [ctypes.c_void_p, _ip, _ip, _ip, _dp]
        L.oracle_cells_free.argtypes = [ctypes.c_void_p]
        L.oracle_fit.restype = ctypes.c_int
        L.oracle_fit.argtypes = [_dp, _dp, ctypes.c_int, _ip, _ip, ctypes.c_double, ctypes.c_double,
                                 _dp, _dp, _ip, ctypes.c_int]
        L.oracle_query.restype = ctypes.c_long
        L.oracle_query.argtypes = ([_dp, _dp, ctypes.c_int, _ip, _ip, _dp, _dp, _dp] +
                                   [ctypes.c_double] * 3 + [ctypes.c_int, ctypes.c_double, ctypes.c_int] +
                                   [_dp, ctypes.c_long, _i8p, _dp, _dp, _dp, _dp, _ip, _ip, _dp, _dp,
                                    _dp, _dp, ctypes.c_int, _ip, _dp, _ip, _dp, _dp, _dp, _dp, _dp, _dp,
                                    ctypes.c_int])
        L.oracle_cond2.argtypes = [_dp, _dp, ctypes.c_int, _ip, _ip, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, _ip, ctypes.c_long, _dp, _dp, _dp]
        L.oracle_softmin.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.oracle_bhm.argtypes = [_dp, ctypes.c_double, _ip, ctypes.c_int, ctypes.c_double, _ip, _dp,
                                 _dp, ctypes.c_long, ctypes.c_double, _dp, _ip, _ip]
        L.oracle_vjp.restype = ctypes.c_double
        L.oracle_vjp.argtypes = ([_dp, ctypes.c_int, _ip, _ip, _dp, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp, ctypes.c_long, _i8p,
                                  ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp,
                                  _dp, _dp, _dp, _ip, _ip, ctypes.c_int])
        _lib = L
    return _lib


def softmin(q, x, alpha):
    """Softmin distance h and its gradient g with respect to the query (App. C)."""
    q = _f64(q).reshape(3)
    x = _f64(x).reshape(-1, 3)
    h = np.zeros(1)
    g = np.zeros(3)
    lib().oracle_softmin(_p(q, _dp), _p(x, _dp), len(x), float(alpha), _p(h, _dp), _p(g, _dp))
    return float(h[0]), g


def bhm(queries, origin, box, dims, hinges, gamma, box_bhm, weights, tau=0.0):
    """Log-odds l, has-map flag and SDF sign (+1 free) of local BHMs (eq.
    sign_prediction, App. B features); see ``oracle_bhm``."""
    q = _f64(queries).reshape(-1, 3)
    org = _f64(origin)
    dm = np.ascontiguousarray(dims, np.int32)
    bb = np.ascontiguousarray(box_bhm, np.int32)
    w = _f64(weights)
    lo = np.zeros(len(q))
    have = np.zeros(len(q), np.int32)
    sign = np.zeros(len(q), np.int32)
    lib().oracle_bhm(_p(org, _dp), float(box), _p(dm, _ip), int(hinges), float(gamma), _p(bb, _ip),
                     _p(w, _dp), _p(q, _dp), len(q), float(tau), _p(lo, _dp), _p(have, _ip),
                     _p(sign, _ip))
    return lo, have, sign


def bhm_update_tau(tau, hit_logodds, alpha):
    """eq. online_surf_logodds: tau <- (1 - alpha) tau + (alpha / K) sum_k l(x_k)."""
    h = np.asarray(hit_logodds, np.float64)
    return (1.0 - alpha) * tau + alpha / len(h) * h.sum()


def refit_priority(dirty, qcount, eta, budget):
    """The GP training queue of App. G: the cells with c2 > 0 ordered by decreasing
    s = c2 (1 + eta c0), ties to the lower id, the first `budget` of them.  The order is
    a decision taken in the precision of the counters (float32): the score is formed
    in float32 as c2 * (1 + (eta * c0)), one rounding per operation, eta rounded to
    float32 first."""
    c2 = np.asarray(dirty, np.float32)
    c0 = np.asarray(qcount, np.float32)
    e = np.float32(eta)
    ids = [i for i in range(len(c2)) if c2[i] > 0]
    score = {i: np.float32(c2[i] * np.float32(np.float32(1.0) + np.float32(e * c0[i])))
             for i in ids}
    ids.sort(key=lambda i: (-score[i], i))
    return np.asarray(ids[:budget], np.int32)


def threads() -> int:
    """Worker threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclasses.dataclass
class Cells:
    offsets: np.ndarray    # int32 [n+1]
    samples: np.ndarray    # int32 [nnz]
    keys: np.ndarray       # int32 [n,3]
    centres: np.ndarray    # float64 [n,3]

    @property
    def n(self):
        return len(self.offsets) - 1

    @property
    def m(self):
        return np.diff(self.offsets)


def build_cells(points, origin, h, margin, m_max, m_min, cap_grid=None, key_lo=(0, 0, 0)) -> Cells:
    L = lib()
    pts = _f64(points)
    org = _f64(origin)
    cg = None if cap_grid is None else np.ascontiguousarray(cap_grid, dtype=np.uint8)
    klo = np.ascontiguousarray(key_lo, dtype=np.int32)
    kd = np.ascontiguousarray(cg.shape if cg is not None else (0, 0, 0), dtype=np.int32)
    hdl = L.oracle_cells_build(_p(pts, _dp), len(pts), _p(org, _dp), h, margin, m_max, m_min,
                               _p(cg, _u8p), _p(klo, _ip), _p(kd, _ip))
    nnz = ctypes.c_long()
    n = L.oracle_cells_count(hdl, ctypes.byref(nnz))
    off = np.zeros(n + 1, np.int32)
    smp = np.zeros(nnz.value, np.int32)
    keys = np.zeros((n, 3), np.int32)
    ctr = np.zeros((n, 3), np.float64)
    L.oracle_cells_copy(hdl, _p(off, _ip), _p(smp, _ip), _p(keys, _ip), _p(ctr, _dp))
    L.oracle_cells_free(hdl)
    return Cells(off, smp, keys, ctr)


def cells_for(wl) -> Cells:
    return build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                       wl.m_cap_grid, wl.key_lo)


@dataclasses.dataclass
class Fit:
    a: np.ndarray        # [nnz]
    L: np.ndarray        # concatenated row-major m x m factors
    lofs: np.ndarray     # [n+1] offsets into L
    ok: np.ndarray       # [n] 1 if the cell factored
    n_failed: int

    def factor(self, c, cells: Cells):
        m = cells.offsets[c + 1] - cells.offsets[c]
        return self.L[self.lofs[c]:self.lofs[c + 1]].reshape(m, m)


def fit(points, cells: Cells, ell, noise, svar=None, kernel="rbf") -> Fit:
    L = lib()
    pts = _f64(points)
    sv = None if svar is None else _f64(svar)
    m = cells.m.astype(np.int64)
    lofs = np.concatenate([[0], np.cumsum(m * m)])
    a = np.zeros(cells.offsets[-1], np.float64)
    Lf = np.zeros(int(lofs[-1]), np.float64)
    ok = np.zeros(cells.n, np.int32)
    nf = L.oracle_fit(_p(pts, _dp), _p(sv, _dp), cells.n, _p(cells.offsets, _ip),
                      _p(cells.samples, _ip), ell, noise, _p(a, _dp), _p(Lf, _dp), _p(ok, _ip),
                      KERNELS[kernel])
    return Fit(a, Lf, lofs, ok, nf)


TIE_REL = 1e-6    # reading R6: relative width of the tie band at the K-th distance
TIE_EXTRA = 8     # list width beyond K for the tie group


def query(points, cells: Cells, f: Fit, queries, ell, noise, alpha=None, k_fuse=8,
          tie_rel=TIE_REL, d_mode=0, sign=None, svar=None, all_candidates=False,
          kernel="rbf") -> dict:
    """All outputs of the back-end at each query (see ``oracle_query``).

    The primary outputs use the K nearest cells by exact distance (ties by id).  The
    candidate list ``cand`` [Q, K + TIE_EXTRA] (-1 padded) holds those K cells, or,
    where the K-th place is tied within ``tie_rel`` (reading R6), the strictly nearer
    cells followed by the whole tie group; ``tie`` [Q,3] = (n_def, n_tie, n_pick)
    (n_tie = 0 without a tie: any n_pick of the n_tie tied cells complete the set).
    ``ucand`` holds each listed cell's u.  With all_candidates, also every listed
    cell's gradient, variances and ratio (keys cgrad [Q,W,3], cgrad_var [Q,W,3], cvar,
    cvar_f, cratio [Q,W]).  grad_var [Q,3] is the SDF gradient variance V[grad_k u] of
    App. C; ratio and fratio are the argmin cell's cancellation ratios of the direction
    w and of the scaled mean f'."""
    L = lib()
    pts = _f64(points)
    q = _f64(queries).reshape(-1, 3)
    nq = len(q)
    cw = k_fuse + TIE_EXTRA
    alpha = 1.0 / (2 * ell * ell) if alpha is None else alpha
    sv = None if svar is None else _f64(svar)
    sg = None if sign is None else np.ascontiguousarray(sign, dtype=np.int8)
    out = {k: np.zeros(nq) for k in ("mean", "var", "var_f", "u_best", "u_second", "ratio", "fratio")}
    out["grad"] = np.zeros((nq, 3))
    out["grad_var"] = np.zeros((nq, 3))
    out["argmin"] = np.zeros(nq, np.int32)
    out["status"] = np.zeros(nq, np.int32)
    out["cand"] = np.zeros((nq, cw), np.int32)
    out["ucand"] = np.zeros((nq, cw))
    out["tie"] = np.zeros((nq, 3), np.int32)
    if all_candidates:
        out["cgrad"] = np.zeros((nq, cw, 3))
        out["cgrad_var"] = np.zeros((nq, cw, 3))
        for k in ("cvar", "cvar_f", "cratio"):
            out[k] = np.zeros((nq, cw))
    g = out.get
    ctr = _f64(cells.centres)
    over = L.oracle_query(_p(pts, _dp), _p(sv, _dp), cells.n, _p(cells.offsets, _ip),
                          _p(cells.samples, _ip), _p(ctr, _dp), _p(f.a, _dp), _p(f.L, _dp), ell,
                          noise, alpha, k_fuse, float(tie_rel), d_mode, _p(q, _dp), nq, _p(sg, _i8p),
                          _p(out["mean"], _dp), _p(out["grad"], _dp), _p(out["var"], _dp),
                          _p(out["var_f"], _dp), _p(out["argmin"], _ip), _p(out["status"], _ip),
                          _p(out["u_best"], _dp), _p(out["u_second"], _dp), _p(out["ratio"], _dp),
                          _p(out["fratio"], _dp), cw, _p(out["cand"], _ip), _p(out["ucand"], _dp),
                          _p(out["tie"], _ip), _p(g("cgrad"), _dp), _p(g("cvar"), _dp),
                          _p(g("cvar_f"), _dp), _p(g("cratio"), _dp), _p(out["grad_var"], _dp),
                          _p(g("cgrad_var"), _dp), KERNELS[kernel])
    out["list_overflow"] = int(over)
    out["sign"] = np.ones(nq, np.int8) if sg is None else sg.copy()
    return out


def cond2(points, cells: Cells, ell, noise, svar=None, kernel="rbf", ids=None):
    """Exact cond_2 of the cells' A = K + Sigma (eigenvalues by cyclic Jacobi), for
    every cell or for the cell ids given; returns (cond, smallest eigenvalue,
    largest eigenvalue), one entry per cell (or per id)."""
    pts = _f64(points)
    sv = None if svar is None else _f64(svar)
    sel = None if ids is None else np.ascontiguousarray(ids, np.int32)
    n = cells.n if sel is None else len(sel)
    cond = np.zeros(n)
    lo = np.zeros(n)
    hi = np.zeros(n)
    lib().oracle_cond2(_p(pts, _dp), _p(sv, _dp), cells.n, _p(cells.offsets, _ip),
                       _p(cells.samples, _ip), float(ell), float(noise), KERNELS[kernel],
                       _p(sel, _ip), n, _p(cond, _dp), _p(lo, _dp), _p(hi, _dp))
    return cond, lo, hi


def vjp(points, cells: Cells, queries, ell, noise, alpha=None, k_fuse=8, tie_rel=TIE_REL, sign=None,
        mode=0, margin=0.3, weight=1.0, d_mean=None, d_grad=None, d_var=None, d_var_f=None,
        per_point=False, force_argmin=None, kernel="rbf", forced_used=False):
    """Dual-number VJP.  mode 0: given cotangents; mode 1: softplus collision cost.
    Returns (loss, d_points [Q,3], d_hyper [2] = d/d(l, sigma^2)), and with per_point
    also each query's own contribution to d_hyper [Q,2].  force_argmin [Q] (optional,
    -1 = none): differentiate at that cell where it is one of the query's listed
    candidates (a near-tie resolved the other way, which the caller has checked against
    the tolerance); with forced_used, also return where it was used (1), refused (0)
    or not given (-1)."""
    L = lib()
    pts = _f64(points)
    q = _f64(queries).reshape(-1, 3)
    sg = None if sign is None else np.ascontiguousarray(sign, dtype=np.int8)
    dp = np.zeros((len(q), 3))
    dh = np.zeros(2)
    pp = np.zeros((len(q), 2)) if per_point else None
    fa = None if force_argmin is None else np.ascontiguousarray(force_argmin, dtype=np.int32)
    fu = np.full(len(q), -1, np.int32)
    cot = [None if c is None else _f64(c) for c in (d_mean, d_grad, d_var, d_var_f)]
    ctr = _f64(cells.centres)
    loss = L.oracle_vjp(_p(pts, _dp), cells.n, _p(cells.offsets, _ip), _p(cells.samples, _ip),
                        _p(ctr, _dp), ell, noise, -1.0 if alpha is None else alpha, k_fuse,
                        float(tie_rel), _p(q, _dp), len(q), _p(sg, _i8p), mode, margin, weight,
                        *[_p(c, _dp) for c in cot], _p(dp, _dp), _p(dh, _dp), _p(pp, _dp),
                        _p(fa, _ip), _p(fu, _ip), KERNELS[kernel])
    res = (loss, dp, dh, pp) if per_point else (loss, dp, dh)
    return res + (fu,) if forced_used else res


def run(points, cells: Cells, queries, ell, noise, **kw):
    """Fit then query, returning (fit, outputs)."""
    f = fit(points, cells, ell, noise, svar=kw.get("svar"), kernel=kw.get("kernel", "rbf"))
    return f, query(points, cells, f, queries, ell, noise, **kw)
