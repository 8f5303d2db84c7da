"""GPU backward (adjoint) against the oracle's dual-number VJP, through the C ABI.

Every point is compared (tests/parity.py check_vjp): the GPU's argmin cell must be
acceptable under readings R6 and R7, and where it differs from the oracle's own
choice the oracle differentiates at the GPU's cell.  FP64 models: d_points within
1e-8 relative per point and d_hyper within 1e-8.  FP32 models: d_points within
max(1e-3, 2 cond_2(A_c) 2^-24) relative per point (norm-wise, floor 1e-3 of the
median norm), the bound growing with the exact condition number of the argmin cell
c because the weights and adjoint vectors come from solves with an FP32 factor;
d_hyper within 1e-3 relative, or, where the per-query terms of that sum cancel,
within 1e-4 of sum_q |term_q| (the oracle gives the terms), for every cotangent
kind (mean, var, var_f and the gradient's kernel-Hessian terms).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_29227_amd import ksdf, scenes
from tests.parity import check_vjp

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


def _compare(dp, dh, am, wl, cells, q, sign, cot, prec, mode=0, kernel="rbf"):
    rep = check_vjp(dp, dh, am, wl, _ocells(wl, cells), q, sign, prec, mode=mode, cot=cot,
                    kernel=kernel, label=f"{prec} {kernel} mode {mode}")
    return rep["err_max"], rep["d_hyper_err"]


def test_fp64_backward_matches_oracle_vjp():
    _say("fp64 backward sphere, random cotangents incl. grad and var_f")
    wl = scenes.sphere_workload(n_queries=2000)
    model, cells, dt = _setup(wl, "fp64", var_f=True)
    cot = _cotangents(len(wl.queries), 0)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp64")
    print("fp64 max point err", e, "d_hyper rel", rel, flush=True)


@pytest.mark.parametrize("var_f", [False, True])
def test_fp32_backward_matches_oracle_vjp(var_f):
    _say(f"fp32 backward small room var_f={var_f}")
    wl = scenes.small_room_workload(n_queries=3000, cfg_id=31)
    model, cells, dt = _setup(wl, "fp32", var_f=var_f)
    cot = _cotangents(len(wl.queries), 1, grad=False, var_f=var_f)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp32")
    print("fp32 max point err", e, "d_hyper rel", rel, flush=True)


def test_fp32_backward_with_gradient_cotangent():
    _say("fp32 backward with a gradient cotangent (kernel Hessian terms)")
    wl = scenes.small_room_workload(n_queries=3000, cfg_id=31)
    model, cells, dt = _setup(wl, "fp32", var_f=True)
    cot = _cotangents(len(wl.queries), 3, grad=True, var_f=True)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp32")
    print("fp32 grad-cotangent max point err", e, "d_hyper err", rel, flush=True)


def test_matern_fp64_backward_matches_oracle_vjp():
    _say("matern32 fp64 backward sphere, random cotangents incl. grad and var_f")
    wl = scenes.sphere_workload(n_queries=2000)
    model, cells, dt = _setup(wl, "fp64", var_f=True, kernel="matern32")
    cot = _cotangents(len(wl.queries), 5)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp64", kernel="matern32")
    print("matern fp64 max point err", e, "d_hyper rel", rel, flush=True)


@pytest.mark.parametrize("var_f", [False, True])
def test_matern_fp32_backward_matches_oracle_vjp(var_f):
    _say(f"matern32 fp32 backward small room var_f={var_f}")
    wl = scenes.small_room_workload(n_queries=3000, cfg_id=33)
    model, cells, dt = _setup(wl, "fp32", var_f=var_f, kernel="matern32")
    cot = _cotangents(len(wl.queries), 6, grad=True, var_f=var_f)
    dp, dh, am = _gpu_vjp(model, wl.queries, wl.sign, cot, dt)
    e, rel = _compare(dp, dh, am, wl, cells, wl.queries, wl.sign, cot, "fp32", kernel="matern32")
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
                      wl.queries, wl.sign, None, "fp32", mode=1)
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
