"""Element-wise comparison of GPU outputs with the FP64 oracle.

Tolerances (the parity contract):
  mean   |d| <= tau * max(|ref|, 1 m), tau = 1e-4 (FP32) / 1e-10 (FP64); where
         |ref| < 1 cm the square-root zone also passes with |d(u^2)| <= 2 l^2 tau'
         (tau' = 1e-5 / 1e-11), because sqrt amplifies the error of u^2 near 0.
  grad   |d| <= max(tau, G(ratio, u)) for every point, with the direction's error
         model G = ratio * (g0 + g1 * |u| / 1 m): the direction w/|w| is a sum whose
         terms cancel, so a relative error e of the terms moves it by about
         e * ratio, ratio = sum|a_i| e_i |x*-x_i| / |w| being the oracle's
         cancellation ratio of the argmin cell.  FP32: g0 = 3e-7 (weights and
         kernel values to a few float ulps), g1 = 3e-7 (the kernel exponent's
         rounding grows with the distance to the cell); FP64: g0 = 1e-14, g1 = 0.
         Unit vectors differ by at most 2, so for very large ratios the bound no
         longer constrains: those points are counted in the report.
  var    |d| <= 1e-3 |ref| (FP32) / 1e-10 |ref| (FP64).
  var_f  |d| <= 1e-3 (FP32) / 1e-10 (FP64), relative to the prior variance k(x,x) = 1.
  grad_var (when the GPU output holds it) |d_k| <= 1e-3 (FP32) / 1e-10 (FP64) x max_k
         |ref_k|: the three components share one scale, and a component can be near 0
         (the (1 - v_k^2) factor of the dominant direction) while the others are not.

Which cell answers a query.  The oracle's candidates are the K nearest cells by
exact FP64 distance (ties by id).  Reading R6: where the K-th place is tied (cells
within 1e-6 relative of the K-th distance outnumber the free places), any choice of
the tied cells is an acceptable candidate set, and the oracle lists the strictly
nearer cells and the whole tie group with every listed cell's outputs.  Reading
R7: within a set, a cell whose u is within the mean tolerance of the minimum is an
acceptable argmin.  The GPU's argmin cell c is accepted when it is listed, no
strictly nearer cell has a u meaningfully below u_c, and enough tied cells have no
u meaningfully below u_c to complete a set of K; every output is then compared
with the oracle's values for that cell.
"""
from __future__ import annotations

import numpy as np

TOL = {
    "fp32": dict(tau=1e-4, tau_sq=1e-5, var=1e-3, var_f=1e-3, g0=3e-7, g1=3e-7),
    "fp64": dict(tau=1e-10, tau_sq=1e-11, var=1e-10, var_f=1e-10, g0=1e-14, g1=0.0),
}


def _mean_ok(d, ref, ell, t):
    ok = np.abs(d - ref) <= t["tau"] * np.maximum(np.abs(ref), 1.0)
    sq = (np.abs(ref) < 0.01) & (np.abs(d * d - ref * ref) <= 2 * ell * ell * t["tau_sq"])
    return ok | sq


def _not_above(x, y, ell, t):
    """x is not meaningfully larger than y (x <= y, or equal within the mean
    tolerance); +inf is not above +inf."""
    with np.errstate(invalid="ignore"):
        return (x <= y) | _mean_ok(x, y, ell, t)


def grad_bound(ratio, u, precision):
    """Allowed |d grad| for the oracle's cancellation ratio and distance u (m)."""
    t = TOL[precision]
    return np.maximum(t["tau"], np.asarray(ratio) * (t["g0"] + t["g1"] * np.abs(u)))


def accepted_cells(am, ora, ell, precision):
    """For each query: the column of the GPU's argmin cell in the oracle's candidate
    list (-1 if not listed) and whether that cell is an acceptable answer (R6, R7)."""
    t = TOL[precision]
    am = np.asarray(am)
    Q = len(am)
    cand, uc, tie = ora["cand"], ora["ucand"], ora["tie"]
    W = cand.shape[1]
    col = np.full(Q, -1)
    hit = (cand == am[:, None]) & (am[:, None] >= 0)
    has = hit.any(1)
    col[has] = np.argmax(hit[has], 1)
    ug = np.where(has, uc[np.arange(Q), np.maximum(col, 0)], np.inf)
    pos = np.arange(W)[None, :]
    n_def, n_tie, n_pick = tie[:, 0:1], tie[:, 1:2], tie[:, 2:3]
    listed = cand >= 0
    definite = listed & (pos < n_def)
    tied = listed & (pos >= n_def) & (n_tie > 0)
    below = ~_not_above(ug[:, None], uc, ell, t)          # u_c meaningfully below u_g
    below &= pos != col[:, None]
    ok_def = ~(definite & below).any(1)
    bad_tied = (tied & below).sum(1)
    ok_tie = (n_tie[:, 0] == 0) | (n_tie[:, 0] - bad_tied >= n_pick[:, 0])
    return col, has & np.isfinite(ug) & ok_def & ok_tie


def compare(gpu: dict, ora: dict, ell: float, precision: str, sign=None) -> dict:
    """Return a report; report['failures'] lists (name, count, first index)."""
    t = TOL[precision]
    Q = len(ora["mean"])
    s = np.asarray(ora["sign"] if sign is None else sign, np.float64)
    rep = dict(n=Q, failures=[], near_tie=0, cand_tie=int((ora["tie"][:, 1] > 0).sum()),
               list_overflow=int(ora.get("list_overflow", 0)))

    def fail(name, mask):
        bad = np.where(~mask)[0]
        if len(bad):
            rep["failures"].append((name, len(bad), int(bad[0])))

    if rep["list_overflow"]:
        rep["failures"].append(("candidate_list_overflow", rep["list_overflow"], -1))
    gmean = np.asarray(gpu["mean"], np.float64)
    gnv = (np.asarray(gpu["status"]) & 1) != 0
    onv = (ora["status"] & 1) != 0
    am = np.asarray(gpu["argmin"])
    col, acc = accepted_cells(am, ora, ell, precision)
    ambiguous = ora["tie"][:, 1] > 0
    # no valid cell: only where the oracle agrees (or a tied set could have none)
    fail("no_valid_flag", (gnv == onv) | (ambiguous & gnv))
    fail("no_valid_mean", ~gnv | np.isinf(gmean))
    v = ~gnv
    fail("argmin_accepted", ~v | acc)
    rep["near_tie"] = int(np.sum(v & acc & (am != ora["argmin"])))
    idx = np.where(v & acc)[0]
    c = col[idx]
    ug = ora["ucand"][idx, c]
    m_mean = np.ones(Q, bool)
    m_mean[idx] = _mean_ok(gmean[idx], s[idx] * ug, ell, t)
    fail("mean", m_mean)
    cg = ora["cgrad"][idx, c]
    cvar = ora["cvar"][idx, c]
    cvf = ora["cvar_f"][idx, c]
    crat = ora["cratio"][idx, c]
    gg = np.asarray(gpu["grad"], np.float64)[idx]
    gerr = np.linalg.norm(gg - cg, axis=1)
    gb = grad_bound(crat, ug, precision)
    m_grad = np.ones(Q, bool)
    m_grad[idx] = gerr <= gb
    fail("grad", m_grad)
    rep["grad_unconstrained"] = int(np.sum(gb >= 2.0))
    rep["grad_err_over_bound_max"] = float((gerr / gb).max()) if idx.size else 0.0
    gv = np.asarray(gpu["var"], np.float64)[idx]
    m_var = np.ones(Q, bool)
    m_var[idx] = np.abs(gv - cvar) <= t["var"] * np.abs(cvar)
    fail("var", m_var)
    if gpu.get("var_f") is not None:
        gf = np.asarray(gpu["var_f"], np.float64)[idx]
        m_vf = np.ones(Q, bool)
        m_vf[idx] = np.abs(gf - cvf) <= t["var_f"]
        fail("var_f", m_vf)
    if gpu.get("grad_var") is not None:
        ggv = np.asarray(gpu["grad_var"], np.float64)[idx]
        cgv = ora["cgrad_var"][idx, c]
        scale = np.abs(cgv).max(1)
        gverr = np.abs(ggv - cgv).max(1)
        m_gv = np.ones(Q, bool)
        m_gv[idx] = gverr <= t["var"] * scale
        fail("grad_var", m_gv)
        rep["grad_var_relerr_max"] = float((gverr / np.maximum(scale, 1e-300)).max()) if idx.size else 0.0
        # no-valid queries report +inf
        fail("grad_var_no_valid", ~gnv | np.isinf(np.asarray(gpu["grad_var"])).all(1))
    # error statistics (for reports)
    fin = np.isfinite(gmean[idx])
    rel = np.abs(gmean[idx][fin] - s[idx][fin] * ug[fin]) / np.maximum(np.abs(ug[fin]), 1.0)
    rep["mean_err_max"] = float(rel.max()) if rel.size else 0.0
    rep["mean_err_p9999"] = float(np.quantile(rel, 0.9999)) if rel.size else 0.0
    rep["grad_err_max"] = float(gerr.max()) if idx.size else 0.0
    rep["grad_err_p9999"] = float(np.quantile(gerr, 0.9999)) if idx.size else 0.0
    vr = np.abs(gv - cvar) / np.maximum(np.abs(cvar), 1e-300)
    rep["var_relerr_max"] = float(vr.max()) if idx.size else 0.0
    rep["var_relerr_p9999"] = float(np.quantile(vr, 0.9999)) if idx.size else 0.0
    if gpu.get("var_f") is not None and idx.size:
        rep["var_f_err_max"] = float(np.abs(gf - cvf).max())
        rep["var_f_err_p9999"] = float(np.quantile(np.abs(gf - cvf), 0.9999))
    return rep


def assert_parity(gpu, ora, ell, precision, sign=None, label=""):
    rep = compare(gpu, ora, ell, precision, sign)
    assert not rep["failures"], f"{label} parity failures {rep['failures']} report {rep}"
    return rep


def hyper_within(dh, odh, pp_abs, rel=1e-3, per_term=1e-4):
    """d_hyper against the oracle.  d_hyper is a sum over queries of terms that can
    cancel; each term carries the FP32 error of its own query, so the sum is held to
    rel x |sum| or, where the terms cancel, per_term x sum_q |term_q| (per_term = the
    forward tolerance).  Returns (ok per component, |error|, allowed)."""
    err = np.abs(np.asarray(dh) - np.asarray(odh))
    allowed = np.maximum(rel * np.abs(odh), per_term * np.asarray(pp_abs))
    return err <= allowed, err, allowed


EPS32 = 2.0 ** -24
VJP_COND = 2.0   # FP32 per-point VJP bound: max(1e-3, VJP_COND * cond_2(A_c) * 2^-24)


def vjp_bounds(cond, precision, tol):
    """Per-point relative bound on d_points.  FP32 models take the weights and the
    fit's adjoint vectors from solves with an FP32 factor of A_c (refined against a
    float-float A); their relative error grows with cond_2(A_c), and near the surface
    the VJP (du/dx = w/(f' u)) amplifies it.  Measured on the test workloads: at most
    0.82 cond_2 2^-24; the bound takes twice cond_2 2^-24, and never less than tol
    (1e-3).  FP64 models: tol (1e-8) throughout."""
    if precision == "fp64":
        return np.full(len(cond), tol)
    return np.maximum(tol, VJP_COND * np.asarray(cond) * EPS32)


def vjp_report(dp, dh, am, wl, cells, q, sign, precision, mode=0, cot=None, kernel="rbf",
               tol_p=None, tol_h=None):
    """Compare a GPU VJP (d_points [Q,3], d_hyper [2] or None, the forward's argmin [Q])
    with the oracle's dual-number VJP at every point; returns a report (see check_vjp)."""
    import oracle   # test infrastructure only
    tol_p = tol_p if tol_p is not None else (1e-8 if precision == "fp64" else 1e-3)
    tol_h = tol_h if tol_h is not None else tol_p
    f = oracle.fit(wl.points, cells, wl.ell, wl.noise_var, kernel=kernel)
    o = oracle.query(wl.points, cells, f, q, wl.ell, wl.noise_var, sign=sign, kernel=kernel)
    valid = (o["status"] & 1) == 0
    col, acc = accepted_cells(am, o, wl.ell, precision)
    force = np.where(valid & acc & (np.asarray(am) != o["argmin"]), am, -1).astype(np.int32)
    kw = {} if mode == 1 else (cot or {})
    _, odp, odh, opp, used = oracle.vjp(wl.points, cells, q, wl.ell, wl.noise_var, sign=sign,
                                        mode=mode, per_point=True, force_argmin=force,
                                        forced_used=True, kernel=kernel, **kw)
    cell = np.where(force >= 0, force, o["argmin"])
    ids, inv = np.unique(np.maximum(cell, 0), return_inverse=True)
    cond_c, _, _ = oracle.cond2(wl.points, cells, wl.ell, wl.noise_var, kernel=kernel, ids=ids)
    cond = cond_c[inv]
    nr = np.linalg.norm(odp, axis=1)
    scale = np.maximum(nr, 1e-3 * np.median(nr[valid]) if valid.any() else 1.0)
    err = np.linalg.norm(np.asarray(dp, np.float64) - odp, axis=1) / scale
    bound = vjp_bounds(cond, precision, tol_p)
    rep = dict(n=len(q), argmin_not_accepted=int(np.sum(valid & ~acc)),
               forced=int((force >= 0).sum()), forced_refused=int(np.sum(used[force >= 0] != 1)),
               err_max=float(err.max()) if len(err) else 0.0,
               err_p9999=float(np.quantile(err, 0.9999)) if len(err) else 0.0,
               err_over_bound_max=float((err / bound).max()) if len(err) else 0.0,
               over_tol=int((err > tol_p).sum()), over_bound=int((err > bound).sum()),
               cond_max=float(cond.max()) if len(cond) else 0.0)
    if dh is not None:
        hok, herr, hallow = hyper_within(dh, odh, np.abs(opp).sum(0), rel=tol_h, per_term=tol_h / 10)
        rep.update(d_hyper=np.asarray(dh).tolist(), d_hyper_oracle=np.asarray(odh).tolist(),
                   d_hyper_err=herr.tolist(), d_hyper_allowed=hallow.tolist(),
                   d_hyper_ok=bool(np.all(hok)))
    rep["_worst"] = np.argsort(-(err / bound))[:5].tolist()
    return rep


def check_vjp(dp, dh, am, wl, cells, q, sign, precision, mode=0, cot=None, kernel="rbf",
              tol_p=None, tol_h=None, label=""):
    """Compare a GPU VJP (d_points [Q,3], d_hyper [2], the forward's argmin [Q]) with
    the oracle's dual-number VJP at every point.  The GPU's argmin must be an
    acceptable cell (R6, R7); where it differs from the oracle's own choice the oracle
    differentiates at the GPU's cell (and must accept it).  d_points: norm-wise
    relative error (floor 1e-3 x the median norm) within vjp_bounds; d_hyper: within
    tol_h relative or, where the per-query terms cancel, tol_h / 10 of sum |term|."""
    rep = vjp_report(dp, dh, am, wl, cells, q, sign, precision, mode, cot, kernel, tol_p, tol_h)
    print(f"{label}: {rep}", flush=True)
    assert rep["argmin_not_accepted"] == 0, f"{label}: GPU argmin cells not acceptable"
    assert rep["forced_refused"] == 0, f"{label}: the oracle refused a forced cell"
    assert rep["over_bound"] == 0, (f"{label}: {rep['over_bound']} points over the bound, "
                                    f"worst {rep['err_max']:.3g} at {rep['_worst']}")
    assert rep["d_hyper_ok"], (f"{label}: d_hyper {rep['d_hyper']} vs oracle {rep['d_hyper_oracle']}: "
                               f"error {rep['d_hyper_err']} over {rep['d_hyper_allowed']}")
    return rep
