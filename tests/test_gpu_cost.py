"""ksdf_cost_backward: the softplus margin cost's gradient with the cotangents formed
inside the backward kernel, against ksdf_query_backward fed the same cotangents from
torch (FP64, rounded to the model's precision), and the per-point cost against an FP64
softplus of the forward outputs.  The VJP itself is held to the oracle by the
backward tests; here the two entry points must agree up to the cotangents' rounding."""
import numpy as np
import pytest
import torch

from paper_2603_29227_amd import ksdf, scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _cotangents(mean, var, margin, kvar, dtype):
    sd = torch.sqrt(torch.clamp_min(var.double(), 1e-30))
    t = margin - mean.double() + kvar * sd
    s = torch.sigmoid(t)
    return (-s).to(dtype).contiguous(), (kvar * s / (2 * sd)).to(dtype).contiguous(), t


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("margin,kvar", [(0.3, 1.0), (0.05, 2.5)])
def test_cost_backward_matches_backward_with_cotangents(precision, margin, kvar):
    _say(f"cost backward {precision} margin {margin} kvar {kvar}")
    wl = scenes.small_room_workload(n_queries=8, cfg_id=61)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision=precision, adjoint=True)
    dt = torch.float32 if precision == "fp32" else torch.float64
    model.fit(torch.from_numpy(wl.points).cuda().to(dt))
    tq, tsg = scenes.room_trajectories(wl, n_traj=96, n_way=64)
    q = torch.from_numpy(tq).cuda().to(dt).contiguous()
    sg = torch.from_numpy(tsg).cuda()
    Q = len(q)
    out = model.query(q, sg)
    dm, dv, t = _cotangents(out["mean"], out["var"], margin, kvar, dt)
    dp_ref, dh_ref = model.backward(q, sg, dm, None, dv, None, argmin=out["argmin"])
    cost = torch.full((Q,), -1.0, dtype=dt, device="cuda")
    dp, dh = model.cost_backward(q, sg, out["mean"], out["var"], argmin=out["argmin"],
                                 margin=margin, kvar=kvar, cost=cost)
    torch.cuda.synchronize()
    assert torch.isfinite(dp).all() and torch.isfinite(dh).all()
    # softplus in FP64 from the same forward outputs
    tt = t.cpu().numpy()
    want = np.maximum(tt, 0) + np.log1p(np.exp(-np.abs(tt)))
    got = cost.double().cpu().numpy()
    rel = 1e-5 if precision == "fp32" else 1e-12
    np.testing.assert_allclose(got, want, rtol=rel, atol=rel * 1e-2)
    # the VJP is linear in the cotangents, which agree to a few roundings
    e = (dp - dp_ref).abs().max().item()
    s = dp_ref.abs().max().item()
    print(f"d_points: max difference {e:.3g} over max {s:.3g}; d_hyper {dh.tolist()} vs "
          f"{dh_ref.tolist()}", flush=True)
    assert e <= (1e-5 if precision == "fp32" else 1e-12) * max(s, 1.0)
    np.testing.assert_allclose(dh.cpu().numpy(), dh_ref.cpu().numpy(),
                               rtol=1e-4 if precision == "fp32" else 1e-10, atol=1e-8)
    model.close()


def test_cost_backward_rejects_bad_arguments():
    _say("cost backward argument checks")
    wl = scenes.small_room_workload(n_queries=64, cfg_id=62)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       adjoint=True)
    model.fit(torch.from_numpy(wl.points).cuda())
    q = torch.from_numpy(wl.queries).cuda()
    out = model.query(q)
    with pytest.raises(ksdf.KsdfError):
        model.cost_backward(q, None, out["mean"], out["var"], margin=float("nan"))
    with pytest.raises(ValueError):
        model.cost_backward(q, None, out["mean"].double(), out["var"])
    model.close()
