"""GPU parity of the Matern 3/2 kernel variant (Table I, App. D) against the FP64
oracle, element by element (tests/parity.py's tolerances), for FP64 and FP32 models,
with every output including the gradient variance, and fused fit+query served by
separate launches (the backward is tested in test_gpu_backward.py)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_29227_amd import ksdf, scenes
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _cells(wl):
    return ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                            wl.m_cap_grid, wl.key_lo)


def _ocells(wl, cells):
    return oracle.Cells(cells.offsets, cells.samples, cells.keys,
                        np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)


def _run(wl, precision):
    cells = _cells(wl)
    dt = torch.float64 if precision == "fp64" else torch.float32
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision=precision, kernel="matern32")
    st = torch.zeros(max(cells.n, 1), dtype=torch.uint8, device="cuda")
    model.fit(torch.from_numpy(np.ascontiguousarray(wl.points)).to("cuda", dt), cell_status=st)
    out = model.query(torch.from_numpy(np.ascontiguousarray(wl.queries)).to("cuda", dt),
                      torch.from_numpy(wl.sign).cuda(), grad_var=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    oc = _ocells(wl, cells)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var, kernel="matern32")
    o = oracle.query(wl.points, oc, f, wl.queries, wl.ell, wl.noise_var, kernel="matern32",
                     sign=wl.sign, all_candidates=True)
    return model, cells, g, o, st.cpu().numpy()[:cells.n]


def test_matern_sphere_fp64():
    _say("matern32 sphere fp64, 10k queries")
    wl = scenes.sphere_workload()
    model, _, g, o, _ = _run(wl, "fp64")
    rep = assert_parity(g, o, wl.ell, "fp64", wl.sign, label="matern sphere fp64")
    assert rep["mean_err_max"] < 1e-10
    model.close()


@pytest.mark.parametrize("uneven", [False, True])
def test_matern_small_room_fp32(uneven):
    _say(f"matern32 small room fp32 uneven={uneven}")
    wl = scenes.small_room_workload(n_queries=4096, uneven=uneven)
    model, _, g, o, _ = _run(wl, "fp32")
    rep = assert_parity(g, o, wl.ell, "fp32", wl.sign, label=f"matern room uneven={uneven}")
    print(rep, flush=True)
    model.close()


def test_matern_fit_query_and_limits():
    _say("matern32 fit_query (fused tuning) vs fit + query; backward needs the adjoint flag")
    wl = scenes.small_room_workload(n_queries=2048)
    cells = _cells(wl)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       kernel="matern32")
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    sg = torch.from_numpy(wl.sign).cuda()
    model.set_tuning(fused=1)
    a = {k: v.clone() for k, v in model.fit_query(pts, q, sg).items()}
    model.fit(pts)
    b = model.query(q, sg)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), f"fit_query and fit + query differ in {k}"
    # the matrix-core option of the RBF two-kernel query leaves a Matern model alone
    model.set_tuning(fused=0, query_split=1, query_block=64, query_mfma=1)
    model.fit(pts)
    c = model.query(q, sg)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], c[k]), f"query_mfma changed the Matern {k}"
    # a model fitted without the adjoint flag has no backward
    with pytest.raises(ksdf.KsdfError):
        model.backward(q, sg, torch.ones_like(b["mean"]))
    model.close()


@pytest.mark.parametrize("tuning", [
    dict(query_split=0, query_block=64, query_sub=2),
    dict(query_split=1, query_block=64, query_sub=2, query_lanes=0),
    dict(query_split=1, query_block=256, query_sub=4, query_lanes=0),
    dict(query_split=1, query_block=256, query_sub=1, query_lanes=1),
])
def test_matern_fp32_launch_shapes_match_each_other_and_oracle(tuning):
    """The Matern cell value rides the RBF's wave-shared query (one kernel or two,
    wave-shared or per-lane cells): every launch shape gives the same outputs, bit for
    bit, and they pass parity with the oracle."""
    _say(f"matern32 fp32 launch shape {tuning}")
    wl = scenes.small_room_workload(n_queries=6000, cfg_id=47, uneven=True)
    cells = _cells(wl)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       kernel="matern32")
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    sg = torch.from_numpy(wl.sign).cuda()
    model.fit(pts)
    model.set_tuning(query_split=0, query_block=64, query_sub=2, query_lanes=0)
    base = {k: v.clone() for k, v in model.query(q, sg, grad_var=True).items()}
    model.set_tuning(**tuning)
    got = model.query(q, sg, grad_var=True)
    torch.cuda.synchronize()
    for k in base:
        assert torch.equal(base[k], got[k]), f"{k} differs under {tuning}"
    oc = _ocells(wl, cells)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var, kernel="matern32")
    o = oracle.query(wl.points, oc, f, wl.queries, wl.ell, wl.noise_var, kernel="matern32",
                     sign=wl.sign, all_candidates=True)
    rep = assert_parity({k: v.cpu().numpy() for k, v in got.items()}, o, wl.ell, "fp32", wl.sign,
                        label=f"matern {tuning}")
    print(rep, flush=True)
    model.close()
