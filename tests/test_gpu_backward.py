"""GPU backward (adjoint) against the oracle's dual-number VJP, through the C ABI.

Tolerances: FP64 path within 1e-8 (relative per point, and for d_hyper); FP32 path
d_points within 1e-3 relative (norm-wise per point) and d_hyper within 1e-3
relative, or, where the per-query terms of that sum cancel, within 1e-4 of
sum_q |term_q| (tests/parity.py hyper_within; the oracle gives the terms)
(with a var_f cotangent 3e-3 per point and 5e-3 for d_hyper: beta = A^{-1} k
comes from FP32 triangular solves with cond(A) up to 1e6, and the noise derivative
carries |beta|^2).  Excluded and counted: points whose argmin cell differs between GPU and
oracle (a near-tie of the min-fusion, where the derivative is that of another
cell), points on a clamp, and in FP32 points whose gradient cancellation ratio
sum|a_i| e_i |x-x_i| / |w| exceeds 1e3 (the same conditioning rule as the forward
gradient; with a gradient cotangent, whose second derivatives cancel further, the
rule is 3e2).  FP32 d_hyper is checked for mean / var / var_f cotangents: with a
gradient cotangent it is dominated by the few near-ridge points whose direction
derivative is ill-conditioned, and is reported rather than asserted.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_29227_amd import ksdf, scenes
from tests.parity import hyper_within

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _setup(wl, precision, var_f=False, kernel="rbf"):
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    dt = torch.float64 if precision == "fp64" else torch.float32
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision=precision, adjoint=True, adjoint_var_f=var_f, kernel=kernel)
    model.fit(torch.from_numpy(np.ascontiguousarray(wl.points)).to("cuda", dt))
    return model, cells, dt


def _ocells(wl, cells):
    return oracle.Cells(cells.offsets, cells.samples, cells.keys,
                        np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)


def _cotangents(Q, seed, grad=True, var_f=True):
    rng = np.random.default_rng(seed)
    return dict(d_mean=rng.normal(size=Q), d_grad=rng.normal(size=(Q, 3)) if grad else None,
                d_var=rng.normal(size=Q) * 100, d_var_f=rng.normal(size=Q) if var_f else None)


def _gpu_vjp(model, q, sign, cot, dt):
    qt = torch.from_numpy(np.ascontiguousarray(q)).to("cuda", dt)
    st = torch.from_numpy(sign).cuda()
    out = model.query(qt, st)
    c = {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dt))
         for k, v in cot.items()}
    dp, dh = model.backward(qt, st, c["d_mean"], c["d_grad"], c["d_var"], c["d_var_f"],
                            argmin=out["argmin"])
    torch.cuda.synchronize()
    return dp.cpu().numpy().astype(np.float64), dh.cpu().numpy(), out["argmin"].cpu().numpy()


def _compare(dp, dh, am, wl, cells, q, sign, cot, prec, tol_p, tol_h, mode=0, max_ratio=np.inf,
             check_hyper=True, kernel="rbf"):
    oc = _ocells(wl, cells)
    cp = 64 if prec == "fp64" else 32
    kw = {} if mode == 1 else cot
    # differentiate at the GPU's argmin cells: near-ties of the min-fusion may resolve
    # either way, and d_hyper sums every point
    _, odp, odh, opp = oracle.vjp(wl.points, oc, q, wl.ell, wl.noise_var, cand_prec=cp,
                                  sign=sign, mode=mode, per_point=True, force_argmin=am,
                                  kernel=kernel, **kw)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var, kernel=kernel)
    o = oracle.query(wl.points, oc, f, q, wl.ell, wl.noise_var, cand_prec=cp, sign=sign,
                     kernel=kernel)
    ok = (am == o["argmin"]) & (o["status"] & 3 == 0) & (o["u_best"] > 1e-3) & (o["ratio"] <= max_ratio)
    assert ok.mean() > 0.8, ok.mean()
    print(f"compared {ok.sum()} of {len(ok)} points", flush=True)
    nr = np.linalg.norm(odp, axis=1)
    scale = np.maximum(nr, 1e-3 * np.median(nr[ok]))
    err = np.linalg.norm(dp - odp, axis=1) / scale
    bad = np.where(ok & (err > tol_p))[0]
    assert len(bad) == 0, f"{len(bad)} points over tolerance, worst {err[ok].max():.3g} at {bad[:5]}"
    # d_hyper sums every query, the excluded ones included (at the GPU's cells):
    # compare as a whole, with the allowance for cancelling per-query terms
    # (tests/parity.py hyper_within)
    rel = np.abs(dh - odh) / np.maximum(np.abs(odh), 1e-12)
    hok, herr, hallow = hyper_within(dh, odh, np.abs(opp).sum(0), rel=tol_h, per_term=tol_h / 10)
    print(f"d_hyper {dh} oracle {odh} sum|term| {np.abs(opp).sum(0)} err {herr} allowed {hallow}",
          flush=True)
    if check_hyper:
        assert np.all(hok), f"d_hyper {dh} vs oracle {odh}: error {herr} over {hallow}"
    return err[ok].max(), rel


def test_fp64_backward_matches_oracle_vjp():
    _say("fp64 backward sphere, random cotangents incl. grad and var_f")
    wl = scenes.sphere_workload(n_queries=2000)
    model, cells, dt = _setup(wl, "fp64", var_f=True)
    cot = _cotangents(len(wl.queries), 0)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp64", 1e-8, 1e-8)
    print("fp64 max point err", e, "d_hyper rel", rel, flush=True)


@pytest.mark.parametrize("var_f", [False, True])
def test_fp32_backward_matches_oracle_vjp(var_f):
    _say(f"fp32 backward small room var_f={var_f}")
    wl = scenes.small_room_workload(n_queries=3000, cfg_id=31)
    model, cells, dt = _setup(wl, "fp32", var_f=var_f)
    cot = _cotangents(len(wl.queries), 1, grad=False, var_f=var_f)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    # a var_f cotangent brings beta = A^{-1} k, an FP32 triangular-solve pair whose error
    # grows with cond(A) (up to 1e6 here): its per-point bound is 3e-3
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp32",
                      3e-3 if var_f else 1e-3, 5e-3 if var_f else 1e-3, max_ratio=1e3)
    print("fp32 max point err", e, "d_hyper rel", rel, flush=True)


def test_fp32_backward_with_gradient_cotangent():
    _say("fp32 backward with a gradient cotangent (kernel Hessian terms)")
    wl = scenes.small_room_workload(n_queries=3000, cfg_id=31)
    model, cells, dt = _setup(wl, "fp32", var_f=True)
    cot = _cotangents(len(wl.queries), 3, grad=True, var_f=True)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp32", 1e-3, 1e-3,
                      max_ratio=3e2, check_hyper=False)
    print("fp32 grad-cotangent max point err", e, "d_hyper rel (reported)", rel, flush=True)


def test_matern_fp64_backward_matches_oracle_vjp():
    _say("matern32 fp64 backward sphere, random cotangents incl. grad and var_f")
    wl = scenes.sphere_workload(n_queries=2000)
    model, cells, dt = _setup(wl, "fp64", var_f=True, kernel="matern32")
    cot = _cotangents(len(wl.queries), 5)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp64", 1e-8, 1e-8,
                      kernel="matern32")
    print("matern fp64 max point err", e, "d_hyper rel", rel, flush=True)


@pytest.mark.parametrize("var_f", [False, True])
def test_matern_fp32_backward_matches_oracle_vjp(var_f):
    _say(f"matern32 fp32 backward small room var_f={var_f}")
    wl = scenes.small_room_workload(n_queries=3000, cfg_id=33)
    model, cells, dt = _setup(wl, "fp32", var_f=var_f, kernel="matern32")
    cot = _cotangents(len(wl.queries), 6, grad=True, var_f=var_f)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp32",
                      3e-3 if var_f else 1e-3, 5e-3 if var_f else 1e-3, max_ratio=1e3,
                      kernel="matern32")
    print("matern fp32 max point err", e, "d_hyper rel", rel, flush=True)


def test_fp32_collision_cost_gradient_via_autograd():
    """The uncertainty-aware collision cost sum softplus(0.3 - mean + sqrt(var)) through
    the autograd Function, to the waypoints and to (l, sigma^2)."""
    _say("fp32 softplus cost through autograd")
    wl = scenes.small_room_workload(n_queries=2048, cfg_id=32)
    model, cells, dt = _setup(wl, "fp32")
    q = torch.from_numpy(wl.queries).cuda().requires_grad_(True)
    theta = torch.tensor([wl.ell, wl.noise_var], dtype=torch.float64, device="cuda", requires_grad=True)
    sg = torch.from_numpy(wl.sign).cuda()
    mean, grad, var, var_f = ksdf.sdf(model, q, sign=sg, theta=theta)
    t = 0.3 - mean.double() + torch.sqrt(var.double())
    cost = torch.nn.functional.softplus(t).sum()
    gq, gth = torch.autograd.grad(cost, [q, theta])
    torch.cuda.synchronize()
    am = model.query(q.detach(), sg)["argmin"].cpu().numpy()
    e, rel = _compare(gq.cpu().numpy().astype(np.float64), gth.cpu().numpy(), am, wl, cells,
                      wl.queries, wl.sign, None, "fp32", 1e-3, 1e-3, mode=1, max_ratio=1e3)
    print("cost grad max point err", e, "theta rel", rel, flush=True)


def test_backward_is_deterministic_and_argmin_optional():
    _say("determinism")
    wl = scenes.small_room_workload(n_queries=4096, cfg_id=33)
    model, cells, dt = _setup(wl, "fp32")
    cot = _cotangents(len(wl.queries), 2, grad=True, var_f=False)
    qt = torch.from_numpy(wl.queries).cuda()
    st = torch.from_numpy(wl.sign).cuda()
    c = {k: (None if v is None else torch.from_numpy(v).to("cuda", dt)) for k, v in cot.items()}
    r1 = model.backward(qt, st, c["d_mean"], c["d_grad"], c["d_var"], None)
    r2 = model.backward(qt, st, c["d_mean"], c["d_grad"], c["d_var"], None)
    torch.cuda.synchronize()
    assert torch.equal(r1[1], r2[1]) and torch.equal(r1[0], r2[0])
    am = model.query(qt, st)["argmin"]
    r3 = model.backward(qt, st, c["d_mean"], c["d_grad"], c["d_var"], None, argmin=am)
    assert torch.equal(r1[1], r3[1])


def test_backward_requires_adjoint_fit():
    _say("backward without adjoint fit")
    wl = scenes.sphere_workload(n_queries=16)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, precision="fp64")
    model.fit(torch.from_numpy(wl.points).cuda())
    q = torch.from_numpy(wl.queries).cuda()
    with pytest.raises(ksdf.KsdfError, match="ADJOINT"):
        model.backward(q, None, torch.ones(16, dtype=torch.float64, device="cuda"))


def test_backward_lane_mode_is_identical():
    _say("backward per-lane cells == wave-shared cells")
    wl = scenes.small_room_workload(n_queries=5000, cfg_id=36)
    model, cells, dt = _setup(wl, "fp32")
    cot = _cotangents(len(wl.queries), 4, grad=True, var_f=False)
    qt = torch.from_numpy(wl.queries).cuda()
    st = torch.from_numpy(wl.sign).cuda()
    c = {k: (None if v is None else torch.from_numpy(v).to("cuda", dt)) for k, v in cot.items()}
    am = model.query(qt, st)["argmin"]
    r1 = model.backward(qt, st, c["d_mean"], c["d_grad"], c["d_var"], None, argmin=am)
    model.set_tuning(backward_lanes=1)
    r2 = model.backward(qt, st, c["d_mean"], c["d_grad"], c["d_var"], None, argmin=am)
    torch.cuda.synchronize()
    assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1])
