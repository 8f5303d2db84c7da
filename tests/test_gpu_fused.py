"""The persistent fused fit+query launch against separate fit and query launches and
against the oracle, on cells with uneven m.  The fused launch fits every cell with a
whole workgroup while the separate launches fit cells of up to 64 samples with one
wave each (rows in registers), so the two agree within the parity tolerances, not
bit for bit: both are held to the oracle, with the same FP64-refit decisions and
argmin cells except at near ties."""
import numpy as np
import pytest
import torch

from paper_2603_29227_amd import ksdf, scenes
from tests.parity import assert_parity
from tests.test_gpu_parity import oracle_run

pytestmark = pytest.mark.gpu


def _run_both(wl, precision="fp32"):
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    dt = torch.float64 if precision == "fp64" else torch.float32
    pts = torch.from_numpy(np.ascontiguousarray(wl.points)).to("cuda", dt)
    q = torch.from_numpy(np.ascontiguousarray(wl.queries)).to("cuda", dt)
    sg = torch.from_numpy(wl.sign).cuda()
    a = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                   precision=precision)
    st_a = torch.zeros(cells.n, dtype=torch.uint8, device="cuda")
    a.fit(pts, cell_status=st_a)
    out_a = a.query(q, sg)
    b = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                   precision=precision)
    st_b = torch.zeros(cells.n, dtype=torch.uint8, device="cuda")
    out_b = b.fit_query(pts, q, sg, cell_status=st_b)
    # a second fused call on the same model reuses every buffer
    out_b = b.fit_query(pts, q, sg, cell_status=st_b, out=out_b)
    torch.cuda.synchronize()
    return cells, {k: v.cpu().numpy() for k, v in out_a.items()}, \
        {k: v.cpu().numpy() for k, v in out_b.items()}, st_a.cpu().numpy(), st_b.cpu().numpy()


@pytest.mark.parametrize("case", ["uneven_small_room", "sphere_fp32", "room_fp32"])
def test_fused_launch_matches_separate_launches_and_oracle(case):
    print(f"[gpu-case] fused {case}", flush=True)
    if case == "uneven_small_room":
        wl = scenes.small_room_workload(n_queries=6000, uneven=True, cfg_id=41)
    elif case == "sphere_fp32":
        wl = scenes.sphere_workload(n_queries=3000)
        wl = scenes.Workload(**{**wl.__dict__, "points": wl.points.astype(np.float32),
                                "queries": wl.queries.astype(np.float32)})
    else:
        wl = scenes.small_room_workload(n_queries=3000, cfg_id=42)
    cells, sep, fus, st_a, st_b = _run_both(wl)
    np.testing.assert_array_equal(st_a, st_b)
    o = oracle_run(wl, cells, wl.queries, wl.sign, "fp32")
    assert_parity(fus, o, wl.ell, "fp32", label=f"fused {case}")
    assert_parity(sep, o, wl.ell, "fp32", label=f"separate {case}")
    assert np.mean(sep["argmin"] == fus["argmin"]) > 0.99


def test_fused_with_no_queries_still_fits():
    print("[gpu-case] fused, zero queries", flush=True)
    wl = scenes.small_room_workload(n_queries=64, cfg_id=43)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    m = ksdf.Model(cells, len(wl.points), wl.origin, wl.h)
    m.set_tuning(fused=1)
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    m.fit_query(pts, torch.zeros(0, 3, dtype=torch.float32, device="cuda"))
    out = m.query(q)
    # the same fused fit, launched with queries: the cells' fits agree bit for bit
    ref = ksdf.Model(cells, len(wl.points), wl.origin, wl.h)
    ref.set_tuning(fused=1)
    want = {k: v.clone() for k, v in ref.fit_query(pts, q).items()}
    torch.cuda.synchronize()
    for k in ("mean", "grad", "var", "argmin", "status"):
        assert torch.equal(out[k], want[k]), k


def test_fused_wait_expiry_is_reported():
    """The fused launch's bounded wait for the fits, forced from the host with a limit
    of one sleep: every kernel still ends normally; queries answered by workgroups
    that stopped waiting carry Q_FIT_TIMEOUT, ksdf_model_check reports the expiry once
    (KSDF_ERR_TIMEOUT) and then clears it; the other queries equal a fused launch
    that waited, bit for bit.  With the default bound nothing is flagged."""
    print("[gpu-case] fused launch, forced wait expiry", flush=True)
    wl = scenes.small_room_workload(n_queries=200_000, uneven=True, cfg_id=44)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    sg = torch.from_numpy(wl.sign).cuda()
    ref = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var)
    ref.set_tuning(fused=1, query_split=0)
    want = {k: v.clone() for k, v in ref.fit_query(pts, q, sg).items()}
    ref.check()
    m = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var)
    m.set_tuning(fused=1, query_split=0)
    m.set_wait_limit(1)
    got = m.fit_query(pts, q, sg)
    torch.cuda.synchronize()
    flagged = (got["status"] & ksdf.Q_FIT_TIMEOUT) != 0
    n_flag = int(flagged.sum())
    print(f"forced expiry: {n_flag} of {len(q)} queries flagged", flush=True)
    assert n_flag > 0
    with pytest.raises(ksdf.KsdfError, match="timeout|wait"):
        m.check()
    m.check()   # reported once
    keep = ~flagged
    for k in ("mean", "grad", "var", "var_f", "argmin"):
        assert torch.equal(got[k][keep], want[k][keep]), k
    assert torch.equal(got["status"][keep], want["status"][keep])
    m.set_wait_limit(0)
    got = m.fit_query(pts, q, sg)
    torch.cuda.synchronize()
    m.check()
    for k in want:
        assert torch.equal(got[k], want[k]), k
    m.close()
    ref.close()
