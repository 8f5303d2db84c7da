"""Parity at full workload sizes, in the launch configuration the benchmark uses.

The GPU answers every query of the workload; the oracle recomputes a seeded sample
of them one by one (the whole fit, then the sampled queries), and the sample is
compared element by element with tests/parity.py's tolerances.  Samples mix uniform
picks with queries near the surface, where the square root and cancellation make the
FP32 path hardest.  The backward is checked against the oracle's dual-number VJP on
every one of the first 1,024 trajectory points (tests/parity.py check_vjp).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_29227_amd import ksdf, scenes, tune
from tests.bhm_bound import abs_terms
from tests.parity import assert_parity, check_vjp

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _ocells(wl, cells):
    return oracle.Cells(cells.offsets, cells.samples, cells.keys,
                        np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)


def _model(wl, query_box=None, adjoint=False):
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision="fp32", query_box=query_box, adjoint=adjoint)
    return model, cells


def _sample(out, n_uniform, n_near, seed):
    rng = np.random.default_rng(seed)
    mean = out["mean"].cpu().numpy()
    Q = len(mean)
    uni = rng.choice(Q, size=min(n_uniform, Q), replace=False)
    near = np.where(np.abs(mean) < 0.05)[0]
    near = rng.choice(near, size=min(n_near, len(near)), replace=False) if len(near) else near
    return np.unique(np.concatenate([uni, near]))


def _check_sample(wl, cells, out, idx, label):
    oc = _ocells(wl, cells)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var)
    o = oracle.query(wl.points, oc, f, wl.queries[idx], wl.ell, wl.noise_var,
                     sign=wl.sign[idx], all_candidates=True)
    g = {k: v.cpu().numpy()[idx] for k, v in out.items()}
    rep = assert_parity(g, o, wl.ell, "fp32", wl.sign[idx], label=label)
    print(f"{label}: {len(idx)} sampled queries, mean err max {rep['mean_err_max']:.3g}, "
          f"grad err max {rep['grad_err_max']:.3g} ({rep['grad_err_over_bound_max']:.3g} of its "
          f"bound), near ties {rep['near_tie']}, candidate ties {rep['cand_tie']}", flush=True)
    return rep


def test_room_grid_full_size():
    _say("room 256^3 grid, 16,777,216 queries, sampled oracle check")
    wl = scenes.room_workload("grid")
    model, cells = _model(wl, query_box=(np.zeros(3), np.array([10.0, 8.0, 3.0])))
    tune.apply(model, len(wl.queries))
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    sg = torch.from_numpy(wl.sign).cuda()
    out = model.fit_query(pts, q, sg, grad_var=True)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert int(((st & 1) != 0).sum()) == 0
    idx = _sample(out, 12000, 4000, 20)
    _check_sample(wl, cells, out, idx, "room grid")
    model.close()


def test_room_batch_uneven_full_size():
    _say("room batch, uneven m on [8,128], 4,194,304 random queries")
    wl = scenes.room_workload("batch")
    model, cells = _model(wl, query_box=(np.zeros(3), np.array([10.0, 8.0, 3.0])))
    m = cells.m
    assert m.min() >= 8 and m.max() > 100, (m.min(), m.max())
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    sg = torch.from_numpy(wl.sign).cuda()
    model.set_tuning(fused=1)
    fused = model.fit_query(pts, q, sg)
    torch.cuda.synchronize()
    fused = {k: v.clone() for k, v in fused.items()}
    model.set_tuning(fused=0)
    sep = model.fit_query(pts, q, sg)
    torch.cuda.synchronize()
    # the fused launch fits with whole workgroups, the separate launches with one wave per
    # cell up to m = 64: both are held to the oracle on the same sample
    idx = _sample(sep, 12000, 4000, 21)
    _check_sample(wl, cells, sep, idx, "room batch")
    _check_sample(wl, cells, fused, idx, "room batch, fused")
    model.close()


def _softplus_cotangents(out):
    sd = torch.sqrt(torch.clamp_min(out["var"], 1e-30))
    s = torch.sigmoid(0.3 - out["mean"] + sd)
    return -s, s / (2 * sd)


def _backward_check(wl, cells, model, tq, tsg, label):
    q = torch.from_numpy(tq).cuda()
    sg = torch.from_numpy(tsg).cuda()
    out = model.query(q, sg)
    dm, dv = _softplus_cotangents(out)
    dp, _ = model.backward(q, sg, dm.contiguous(), None, dv.contiguous(), None, argmin=out["argmin"])
    torch.cuda.synchronize()
    assert torch.isfinite(dp).all()
    # FP64 check on the first 1,024 points: their own backward (d_hyper of that set)
    n = 1024
    q1, s1 = q[:n].contiguous(), sg[:n].contiguous()
    o1 = model.query(q1, s1)
    dm1, dv1 = _softplus_cotangents(o1)
    dp1, dh1 = model.backward(q1, s1, dm1.contiguous(), None, dv1.contiguous(), None,
                              argmin=o1["argmin"])
    torch.cuda.synchronize()
    assert torch.equal(dp1, dp[:n]), "a point's VJP depends on the batch it is in"
    check_vjp(dp1.cpu().numpy(), dh1.cpu().numpy(), o1["argmin"].cpu().numpy(), wl,
              _ocells(wl, cells), tq[:n], tsg[:n], "fp32", mode=1, label=label)


def test_room_trajectory_backward_full_size():
    _say("room trajectories 4,096 x 64, softplus cost backward, FP64 check on 1,024 points")
    wl = scenes.room_workload("grid", grid_n=4)
    model, cells = _model(wl, query_box=(np.zeros(3), np.array([10.0, 8.0, 3.0])), adjoint=True)
    model.fit(torch.from_numpy(wl.points).cuda())
    tq, tsg = scenes.room_trajectories(wl)
    _backward_check(wl, cells, model, tq, tsg, "room trajectories")
    model.close()


def test_terrain_full_size():
    _say("outdoor terrain, 256^3 grid + 16,384 x 64 trajectory backward, sampled oracle checks")
    wl = scenes.terrain_workload(grid_n=256)
    print(f"terrain: {len(wl.points)} samples", flush=True)
    model, cells = _model(wl, query_box=(np.zeros(3), np.array([100.0, 100.0, 25.0])), adjoint=True)
    m = cells.m
    print(f"cells {cells.n}, m {m.min()}..{m.max()}, mean {m.mean():.1f}", flush=True)
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    sg = torch.from_numpy(wl.sign).cuda()
    model.fit(pts)
    out = model.query(q, sg, grad_var=True)
    torch.cuda.synchronize()
    idx = _sample(out, 12000, 4000, 22)
    _check_sample(wl, cells, out, idx, "terrain grid")
    tq, tsg = scenes.terrain_trajectories(wl)
    _backward_check(wl, cells, model, tq, tsg, "terrain trajectories")
    model.close()


def test_matern_room_grid_full_size():
    _say("matern32 room 256^3 grid (the bench's Matern leg), sampled oracle check")
    wl = scenes.room_workload("grid")
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision="fp32", query_box=(np.zeros(3), np.array([10.0, 8.0, 3.0])),
                       kernel="matern32")
    model.fit(torch.from_numpy(wl.points).cuda())
    out = model.query(torch.from_numpy(wl.queries).cuda(), torch.from_numpy(wl.sign).cuda(),
                      grad_var=True)
    torch.cuda.synchronize()
    idx = _sample(out, 6000, 2000, 23)
    oc = _ocells(wl, cells)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var, kernel="matern32")
    o = oracle.query(wl.points, oc, f, wl.queries[idx], wl.ell, wl.noise_var,
                     sign=wl.sign[idx], all_candidates=True, kernel="matern32")
    g = {k: v.cpu().numpy()[idx] for k, v in out.items()}
    rep = assert_parity(g, o, wl.ell, "fp32", wl.sign[idx], label="matern room grid")
    print(f"matern room grid: {len(idx)} sampled, mean err max {rep['mean_err_max']:.3g}", flush=True)
    model.close()


def test_bhm_sign_room_grid_full_size():
    _say("bhm sign on the room 256^3 grid (the bench's sign leg), sampled oracle check")
    wl = scenes.room_workload("grid")
    b = scenes.bhm_weights(wl)
    q = torch.from_numpy(wl.queries).cuda()
    sign, lo = ksdf.bhm_sign(q, b["origin"], b["box"], b["dims"], b["hinges"], b["gamma"],
                             torch.from_numpy(b["box_bhm"]).cuda(),
                             torch.from_numpy(b["weights"]).cuda(), tau=0.0, logodds=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(24)
    g = lo.cpu().numpy()
    have = np.where(np.isfinite(g))[0]
    idx = np.unique(np.concatenate([rng.choice(len(g), 20000, replace=False),
                                    rng.choice(have, min(20000, len(have)), replace=False)]))
    olo, oh, osg = oracle.bhm(wl.queries[idx].astype(np.float64), b["origin"], b["box"], b["dims"],
                              b["hinges"], b["gamma"], b["box_bhm"], b["weights"], tau=0.0)
    h = oh == 1
    assert np.array_equal(np.isfinite(g[idx]), h)
    # float queries: FP32 log-odds within 100 roundings of sum |terms| (test_gpu_bhm)
    tol = 100 * 2.0 ** -24 * abs_terms(wl.queries[idx].astype(np.float64), b)
    assert np.all(np.abs(g[idx][h] - olo[h]) <= tol[h])
    s = sign.cpu().numpy()[idx].astype(np.int32)
    clear = ~h | (np.abs(olo) > tol)
    assert np.array_equal(s[clear], osg[clear])
    print(f"bhm grid: {len(idx)} sampled, {int(h.sum())} inside maps", flush=True)
