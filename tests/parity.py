"""Element-wise comparison of GPU outputs with the FP64 oracle.

Tolerances (the parity contract):
  mean   |d| <= tau * max(|ref|, 1 m), tau = 1e-4 (FP32) / 1e-10 (FP64); where
         |ref| < 1 cm the square-root zone also passes with |d(u^2)| <= 2 l^2 tau'
         (tau' = 1e-5 / 1e-11), because sqrt amplifies the error of u^2 near 0.
  grad   |d| <= tau where the oracle's cancellation ratio sum|a_i| e_i |x*-x_i| / |w|
         is <= 1e3 (elsewhere the direction is ill-conditioned for FP32 weights: the
         measured FP32 error grows as about 3e-8 x ratio; counted, not compared).
         More than 2 m from the surface the limit is 2.5e2: there the per-sample
         spread of the kernel exponent grows like |x*-c| h / l^2, its FP32 rounding
         adds to the cancellation, and the measured error is about 4e-7 x ratio.
  var    |d| <= 1e-3 |ref| (FP32) / 1e-10 |ref| (FP64).
  var_f  |d| <= 1e-3 (FP32) / 1e-10 (FP64), relative to the prior variance k(x,x) = 1.
  grad_var (when the GPU output holds it) |d_k| <= 1e-3 (FP32) / 1e-10 (FP64) x max_k
         |ref_k|: the three components share one scale, and a component can be near 0
         (the (1 - v_k^2) factor of the dominant direction) while the others are not.
Near-ties of the min-fusion: the GPU's argmin cell is accepted when it is one of
the oracle's candidates and its oracle u is within the mean tolerance of the
oracle's minimum; grad / var / var_f are then compared with the oracle's values
for that same cell.
"""
from __future__ import annotations

import numpy as np

TOL = {
    "fp32": dict(tau=1e-4, tau_sq=1e-5, var=1e-3, var_f=1e-3, ratio=1e3, ratio_far=2.5e2),
    "fp64": dict(tau=1e-10, tau_sq=1e-11, var=1e-10, var_f=1e-10, ratio=1e6, ratio_far=1e6),
}
FAR = 2.0   # metres from the surface where the far-field ratio limit applies


def _mean_ok(d, ref, ell, t):
    ok = np.abs(d - ref) <= t["tau"] * np.maximum(np.abs(ref), 1.0)
    sq = (np.abs(ref) < 0.01) & (np.abs(d * d - ref * ref) <= 2 * ell * ell * t["tau_sq"])
    return ok | sq


def compare(gpu: dict, ora: dict, ell: float, precision: str, sign=None) -> dict:
    """Return a report; report['failures'] lists (name, count, first index)."""
    t = TOL[precision]
    Q = len(ora["mean"])
    s = np.ones(Q) if sign is None else np.asarray(sign, np.float64)
    rep = dict(n=Q, failures=[], exempt_grad=0, near_tie=0)

    def fail(name, mask):
        bad = np.where(~mask)[0]
        if len(bad):
            rep["failures"].append((name, len(bad), int(bad[0])))

    gmean = np.asarray(gpu["mean"], np.float64)
    novalid = (ora["status"] & 1) != 0
    fail("no_valid_flag", ((gpu["status"] & 1) != 0) == novalid)
    fail("no_valid_mean", ~novalid | np.isinf(gmean))
    v = ~novalid
    fail("mean", ~v | _mean_ok(gmean, ora["mean"], ell, t))
    # which oracle candidate did the GPU pick?
    am = np.asarray(gpu["argmin"])
    col = np.full(Q, -1)
    hit = ora["cand"] == am[:, None]
    has = hit.any(1)
    col[has] = np.argmax(hit[has], 1)
    fail("argmin_in_candidates", ~v | has)
    ub = ora["u_best"]
    uc = np.where(col >= 0, ora["ucand"][np.arange(Q), np.maximum(col, 0)], np.inf)
    tie_ok = _mean_ok(uc, ub, ell, t)
    fail("argmin_near_tie", ~v | tie_ok)
    rep["near_tie"] = int(np.sum(v & (am != ora["argmin"]) & tie_ok))
    ok_cell = v & has & tie_ok
    idx = np.where(ok_cell)[0]
    c = col[idx]
    cg = ora["cgrad"][idx, c]
    cvar = ora["cvar"][idx, c]
    cvf = ora["cvar_f"][idx, c]
    crat = ora["cratio"][idx, c]
    gg = np.asarray(gpu["grad"], np.float64)[idx]
    gerr = np.linalg.norm(gg - cg, axis=1)
    far = np.abs(ora["mean"][idx]) > FAR
    well = crat <= np.where(far, t["ratio_far"], t["ratio"])
    rep["exempt_grad"] = int(np.sum(~well))
    m_grad = np.ones(Q, bool)
    m_grad[idx] = ~well | (gerr <= t["tau"])
    fail("grad", m_grad)
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
        fail("grad_var_no_valid", ~novalid | np.isinf(np.asarray(gpu["grad_var"])).all(1))
    # error statistics (for reports)
    mv = v & np.isfinite(gmean)
    rel = np.abs(gmean[mv] - ora["mean"][mv]) / np.maximum(np.abs(ora["mean"][mv]), 1.0)
    rep["mean_err_max"] = float(rel.max()) if rel.size else 0.0
    rep["mean_err_p9999"] = float(np.quantile(rel, 0.9999)) if rel.size else 0.0
    rep["grad_err_max"] = float(gerr[well].max()) if np.any(well) else 0.0
    rep["var_relerr_max"] = float((np.abs(gv - cvar) / np.maximum(np.abs(cvar), 1e-300)).max()) if idx.size else 0.0
    if gpu.get("var_f") is not None and idx.size:
        rep["var_f_err_max"] = float(np.abs(gf - cvf).max())
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
