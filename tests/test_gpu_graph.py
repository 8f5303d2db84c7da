"""HIP-graph capture of whole steps, and the launch-shape knobs.

A captured step (fit + query + backward, or the fused fit+query) is replayed several
times with new input values copied into its static inputs, with eager work of the
same model between the replays; every replay must equal, bit for bit, the eager call
made on the same inputs.  Every tuning of the launch shape must give the same outputs
as the default one, bit for bit, and pass parity against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_29227_amd import ksdf, scenes
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _model(wl, precision="fp32", adjoint=False):
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    return ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                      precision=precision, adjoint=adjoint, dense_inverse=True), cells


def _equal(a: dict, b: dict, keys=("mean", "grad", "var", "var_f", "argmin", "status")):
    for k in keys:
        assert torch.equal(a[k], b[k]), f"{k} differs"


def _clone(d):
    return {k: v.clone() for k, v in d.items()}


@pytest.mark.parametrize("mfma", [0, 1])
def test_graph_fit_query_backward_replays_match_eager(mfma):
    _say(f"graph: fit + query + backward, 3 replays with eager work between, query_mfma={mfma}")
    wl = scenes.small_room_workload(n_queries=20000, cfg_id=41, uneven=True)
    model, _ = _model(wl, adjoint=True)
    if mfma:   # the two-kernel query with the matrix-core pass 2 (its inverse formed by the fit)
        model.set_tuning(fused=0, query_split=1, query_block=64, query_mfma=1)
    dev = torch.device("cuda")
    P = torch.from_numpy(wl.points).to(dev, torch.float32)
    q = torch.from_numpy(wl.queries).to(dev, torch.float32)
    sg = torch.from_numpy(wl.sign).to(dev)
    rng = np.random.default_rng(5)
    dm = torch.from_numpy(rng.normal(size=len(q))).to(dev, torch.float32)
    dv = torch.from_numpy(rng.normal(size=len(q))).to(dev, torch.float32)
    out = model._out(len(q), dev)

    def step():
        model.fit(P)
        model.query(q, sg, out=out)
        return model.backward(q, sg, dm, None, dv, None, argmin=out["argmin"])

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()  # warm-up: sizes the workspace, takes the launch attributes
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dpg, dhg = step()
    shift = torch.tensor([0.0, 0.0, 0.0], device=dev)
    P0, q0 = P.clone(), q.clone()
    for rep in range(3):
        # new inputs in the static buffers: a small rigid shift of samples and queries
        shift.uniform_(-0.01, 0.01)
        P.copy_(P0 + shift)
        q.copy_(q0 + 0.5 * shift)
        g.replay()
        torch.cuda.synchronize()
        got = _clone(out)
        gdp, gdh = dpg.clone(), dhg.clone()
        # eager work of the same model between replays (refits, other queries)
        model.fit(P0)
        model.query(q0[:1000].contiguous(), sg[:1000].contiguous())
        ref_out = model._out(len(q), dev)
        model.fit(P)
        model.query(q, sg, out=ref_out)
        rdp, rdh = model.backward(q, sg, dm, None, dv, None, argmin=ref_out["argmin"])
        torch.cuda.synchronize()
        _equal(got, ref_out)
        assert torch.equal(gdp, rdp), f"replay {rep}: d_points differ"
        assert torch.equal(gdh, rdh), f"replay {rep}: d_hyper differ"
    model.close()


def test_concurrent_calls_on_two_streams_match_serial():
    _say("query + backward on a second stream beside a grid query, own workspaces, 3 rounds")
    wl = scenes.small_room_workload(n_queries=30000, cfg_id=43, uneven=True)
    model, _ = _model(wl, adjoint=True)
    dev = torch.device("cuda")
    P = torch.from_numpy(wl.points).to(dev, torch.float32)
    q = torch.from_numpy(wl.queries).to(dev, torch.float32)
    sg = torch.from_numpy(wl.sign).to(dev)
    q2 = (q[:6000] * 0.999).contiguous()
    sg2 = sg[:6000].contiguous()
    dm = torch.from_numpy(np.random.default_rng(9).normal(size=len(q2))).to(dev, torch.float32)
    model.set_tuning(fused=0, query_split=1, query_block=64, query_mfma=1)
    model.fit(P)
    ref = _clone(model.query(q, sg))
    ref2 = _clone(model.query(q2, sg2))
    rdp, rdh = model.backward(q2, sg2, dm, argmin=ref2["argmin"])
    torch.cuda.synchronize()
    rdp, rdh = rdp.clone(), rdh.clone()
    with pytest.raises(ValueError):
        model.query(q2, sg2, workspace=torch.empty(1, dtype=torch.uint8, device=dev))
    side = torch.cuda.Stream()
    ws2 = model.new_workspace(len(q2))
    out, out2 = model._out(len(q), dev), model._out(len(q2), dev)
    for rep in range(3):
        main = torch.cuda.current_stream()
        side.wait_stream(main)
        with torch.cuda.stream(side):
            model.query(q2, sg2, out=out2, workspace=ws2)
            dp, dh = model.backward(q2, sg2, dm, argmin=out2["argmin"], workspace=ws2)
        model.query(q, sg, out=out)
        main.wait_stream(side)
        torch.cuda.synchronize()
        _equal(out, ref)
        _equal(out2, ref2)
        assert torch.equal(dp, rdp) and torch.equal(dh, rdh), f"round {rep}: backward differs"
    model.close()


@pytest.mark.parametrize("fused", [1, 0])
def test_graph_fit_query_call_replays_match_eager(fused):
    """fused=1: the persistent launch; fused=0: the fit with the query's bucketing on the
    model's second stream beside it (forked and joined inside the captured call)."""
    _say(f"graph: fit_query (fused={fused}), 3 replays")
    wl = scenes.small_room_workload(n_queries=30000, cfg_id=42, uneven=True)
    model, _ = _model(wl)
    model.set_tuning(fused=fused, query_split=1 - fused)
    dev = torch.device("cuda")
    P = torch.from_numpy(wl.points).to(dev, torch.float32)
    q = torch.from_numpy(wl.queries).to(dev, torch.float32)
    sg = torch.from_numpy(wl.sign).to(dev)
    out = model._out(len(q), dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        model.fit_query(P, q, sg, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        model.fit_query(P, q, sg, out=out)
    gen = torch.Generator(device=dev).manual_seed(3)
    lo = torch.tensor(wl.queries.min(0), device=dev, dtype=torch.float32)
    hi = torch.tensor(wl.queries.max(0), device=dev, dtype=torch.float32)
    for rep in range(3):
        q.copy_(lo + (hi - lo) * torch.rand(q.shape, device=dev, generator=gen))
        g.replay()
        torch.cuda.synchronize()
        got = _clone(out)
        model.query(q[:500].contiguous(), None)
        ref = model.fit_query(P, q, sg)
        torch.cuda.synchronize()
        _equal(got, ref)
    model.close()


@pytest.mark.parametrize("tuning", [
    dict(query_sub=1, query_block=256, fused=1, fit_min_bucket=16, query_split=0),
    dict(query_sub=2, query_block=64, fused=0, fit_min_bucket=32, query_split=0),
    dict(query_sub=4, query_block=64, fused=1, fit_min_bucket=64, query_split=1),
    dict(query_sub=4, query_block=256, fused=0, fit_min_bucket=16, query_split=1),
    dict(query_sub=2, query_block=64, fused=0, fit_min_bucket=16, query_split=1, query_lanes=1,
         backward_lanes=1),
])
def test_tuning_preserves_outputs(tuning):
    _say(f"tuning {tuning}")
    wl = scenes.small_room_workload(n_queries=12000, cfg_id=43, uneven=True)
    model, cells = _model(wl)
    dev = torch.device("cuda")
    P = torch.from_numpy(wl.points).to(dev, torch.float32)
    q = torch.from_numpy(wl.queries).to(dev, torch.float32)
    sg = torch.from_numpy(wl.sign).to(dev)
    # the fused launch fits every cell with a workgroup, the separate fit with one wave
    # per cell up to m = 64: each tuning is compared with the default of its own fit
    model.set_tuning(fused=1)
    base_fused = _clone(model.fit_query(P, q, sg))
    model.set_tuning(fused=0)
    model.fit(P)
    base_sep = _clone(model.query(q, sg))
    torch.cuda.synchronize()
    model.set_tuning(**tuning)
    assert all(model.tuning()[k] == v for k, v in tuning.items())
    a = model.fit_query(P, q, sg)
    torch.cuda.synchronize()
    a = _clone(a)
    model.fit(P)
    b = model.query(q, sg)
    torch.cuda.synchronize()
    _equal(a, base_fused if tuning["fused"] else base_sep)
    _equal(b, base_sep)
    oc = oracle.Cells(cells.offsets, cells.samples, cells.keys,
                      np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var)
    o = oracle.query(wl.points, oc, f, wl.queries, wl.ell, wl.noise_var,
                     sign=wl.sign, all_candidates=True)
    assert_parity({k: v.cpu().numpy() for k, v in b.items()}, o, wl.ell, "fp32", wl.sign,
                  label=str(tuning))
    model.close()


@pytest.mark.parametrize("tuning", [
    dict(query_sub=4, query_block=64, fused=0, query_split=1, query_pairs=1),
    dict(query_sub=2, query_block=256, fused=0, query_split=1, query_pairs=1, query_lanes=1),
])
def test_query_pairs_matches_wave_walk_and_oracle(tuning):
    """The pair form of pass 1 evaluates every candidate (no pruning); it must pass
    parity and agree with the wave-shared walk except where a near-tied cell's
    float-float re-evaluation is triggered differently."""
    _say(f"query pairs {tuning}")
    wl = scenes.small_room_workload(n_queries=12000, cfg_id=44, uneven=True)
    model, cells = _model(wl)
    dev = torch.device("cuda")
    P = torch.from_numpy(wl.points).to(dev, torch.float32)
    q = torch.from_numpy(wl.queries).to(dev, torch.float32)
    sg = torch.from_numpy(wl.sign).to(dev)
    model.set_tuning(fused=0, query_split=1, query_pairs=0)
    model.fit(P)
    base = _clone(model.query(q, sg, grad_var=True))
    model.set_tuning(**tuning)
    b = model.query(q, sg, grad_var=True)
    again = model.query(q, sg, grad_var=True)
    torch.cuda.synchronize()
    _equal(b, again, keys=("mean", "grad", "var", "var_f", "grad_var", "argmin", "status"))
    diff = torch.zeros(len(q), dtype=torch.bool, device=dev)
    for k in ("mean", "var", "var_f", "argmin", "status"):
        diff |= base[k] != b[k]
    diff |= (base["grad"] != b["grad"]).any(1)
    print(f"pairs vs wave walk: {int(diff.sum())} of {len(q)} queries differ", flush=True)
    assert int(diff.sum()) <= len(q) // 100
    oc = oracle.Cells(cells.offsets, cells.samples, cells.keys,
                      np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var)
    o = oracle.query(wl.points, oc, f, wl.queries, wl.ell, wl.noise_var,
                     sign=wl.sign, all_candidates=True)
    assert_parity({k: v.cpu().numpy() for k, v in b.items()}, o, wl.ell, "fp32", wl.sign,
                  label=f"pairs {tuning}")
    model.close()


@pytest.mark.parametrize("block", [64, 256])
def test_query_mfma_gp_variance(block):
    """The matrix-core GP variance (query_mfma) changes only var_f, within the parity
    tolerance of the forward substitution it replaces."""
    _say(f"query_mfma block {block}")
    wl = scenes.small_room_workload(n_queries=12000, cfg_id=46)
    model, cells = _model(wl)
    dev = torch.device("cuda")
    P = torch.from_numpy(wl.points).to(dev, torch.float32)
    q = torch.from_numpy(wl.queries).to(dev, torch.float32)
    sg = torch.from_numpy(wl.sign).to(dev)
    model.set_tuning(fused=0, query_split=1, query_block=block, query_mfma=0)
    model.fit(P)
    base = _clone(model.query(q, sg, grad_var=True))
    model.set_tuning(query_mfma=1)
    b = model.query(q, sg, grad_var=True)
    again = model.query(q, sg, grad_var=True)
    torch.cuda.synchronize()
    _equal(b, again, keys=("mean", "grad", "var", "var_f", "grad_var", "argmin", "status"))
    _equal(b, base, keys=("mean", "grad", "var", "grad_var", "argmin", "status"))
    d = (b["var_f"] - base["var_f"]).abs().max().item()
    print(f"query_mfma: max |var_f difference| {d:.3g}", flush=True)
    assert d <= 1e-4
    oc = oracle.Cells(cells.offsets, cells.samples, cells.keys,
                      np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var)
    o = oracle.query(wl.points, oc, f, wl.queries, wl.ell, wl.noise_var,
                     sign=wl.sign, all_candidates=True)
    assert_parity({k: v.cpu().numpy() for k, v in b.items()}, o, wl.ell, "fp32", wl.sign,
                  label=f"query_mfma {block}")
    # a fit with the knob on, and the fused launch, keep the dense L^{-1} current
    for fused in (0, 1):
        model.set_tuning(fused=fused, query_split=1 - fused, query_mfma=0)
        model.fit(P * 1.001)               # a different factor, left stale
        model.set_tuning(query_mfma=1)
        if fused:
            model.fit_query(P, q, sg)
        else:
            model.fit(P)
        model.set_tuning(fused=0, query_split=1, query_mfma=1)
        c = _clone(model.query(q, sg, grad_var=True))
        if not fused:
            torch.cuda.synchronize()
            _equal(c, b, keys=("mean", "grad", "var", "var_f", "grad_var", "argmin", "status"))
            continue
        # the fused launch fits with its own workgroup kernel, so its factor differs
        # from the separate fit's by rounding: compare with the forward substitution
        # on the factor it left
        model.set_tuning(query_mfma=0)
        fs = model.query(q, sg, grad_var=True)
        torch.cuda.synchronize()
        _equal(c, fs, keys=("mean", "grad", "var", "grad_var", "argmin", "status"))
        d = (c["var_f"] - fs["var_f"]).abs().max().item()
        print(f"query_mfma after the fused fit: max |var_f difference| {d:.3g}", flush=True)
        assert d <= 1e-4
    model.close()


def test_tuning_rejects_invalid_values():
    _say("tuning validation")
    wl = scenes.sphere_workload(n_queries=16)
    model, _ = _model(wl, precision="fp64")
    for bad in (dict(query_sub=3), dict(query_block=128), dict(fused=2), dict(fit_min_bucket=8),
                dict(query_split=2), dict(query_lanes=2), dict(backward_lanes=-1),
                dict(query_pairs=3), dict(query_mfma=2)):
        with pytest.raises(ksdf.KsdfError):
            model.set_tuning(**bad)
    model.close()


def test_kernel_timers_report_each_launch():
    _say("kernel timers")
    wl = scenes.small_room_workload(n_queries=5000, cfg_id=44)
    model, _ = _model(wl, adjoint=True)
    dev = torch.device("cuda")
    P = torch.from_numpy(wl.points).to(dev, torch.float32)
    q = torch.from_numpy(wl.queries).to(dev, torch.float32)
    with pytest.raises(ksdf.KsdfError):
        model.timer_read("query")  # timing is off
    model.set_timing(True)
    model.fit(P)
    out = model.query(q)
    model.query(q[:100].contiguous())
    model.backward(q, None, torch.ones(len(q), device=dev), argmin=out["argmin"])
    fits, qs, bw = model.timer_read("fit"), model.timer_read("query"), model.timer_read("backward")
    assert len(fits) == 1 and len(qs) == 2 and len(bw) == 1
    assert all(t > 0 for t in fits + qs + bw)
    assert model.timer_read("query") == []
    for _ in range(ksdf.TIMER_SLOTS + 1):
        model.query(q[:64].contiguous())
    with pytest.raises(ksdf.KsdfError):
        model.timer_read("query")  # more launches than slots since the last read
    model.set_timing(False)
    model.close()
