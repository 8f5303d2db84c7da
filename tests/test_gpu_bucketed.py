"""A query in two calls: the bucketing of the points (which reads the candidate index,
not the fit) on a second stream beside a fit, then the rest of the query on the fitted
model.  The two calls must give the one-call query's outputs bit for bit, for every
launch shape of the query and for FP64 models (where the bucketing is a no-op)."""
import pytest
import torch

from paper_2603_29227_amd import ksdf, scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _setup(uneven, precision="fp32", n_queries=20000):
    wl = scenes.small_room_workload(n_queries=n_queries, cfg_id=44, uneven=uneven)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision=precision, dense_inverse=not uneven and precision == "fp32")
    dt = torch.float32 if precision == "fp32" else torch.float64
    P = torch.from_numpy(wl.points).to("cuda", dt)
    q = torch.from_numpy(wl.queries).to("cuda", dt)
    sg = torch.from_numpy(wl.sign).to("cuda")
    return model, P, q, sg


def _equal(a, b):
    for k in ("mean", "grad", "var", "var_f", "argmin", "status"):
        assert torch.equal(a[k], b[k]), f"{k} differs"


@pytest.mark.parametrize("uneven,tuning", [
    (False, dict(query_split=1, query_sub=2, query_block=64, query_mfma=1)),
    (True, dict(query_split=1, query_sub=4, query_block=64)),
    (True, dict(query_split=1, query_sub=1, query_block=256, query_lanes=1)),
    (True, dict(query_split=1, query_sub=2, query_block=256, query_pairs=1)),
    (True, dict(query_split=0, query_sub=2, query_block=64)),
])
def test_bucket_beside_fit_then_bucketed_query_equals_query(uneven, tuning):
    _say(f"bucket beside fit, then bucketed query: uneven={uneven} {tuning}")
    model, P, q, sg = _setup(uneven)
    model.set_tuning(fused=0, **tuning)
    main = torch.cuda.current_stream()
    model.fit(P)
    ref = {k: v.clone() for k, v in model.query(q, sg).items()}
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    ws = model.new_workspace(len(q))
    for n in (len(q), len(q) // 3 + 7):   # the second call reuses the workspace, fewer points
        qn = q[:n].contiguous()
        sn = sg[:n].contiguous()
        want = {k: v[:n] for k, v in ref.items()}
        side.wait_stream(main)
        with torch.cuda.stream(side):
            model.bucket(qn, workspace=ws)
        model.fit(P)                      # the same cells again, on the main stream
        main.wait_stream(side)
        got = model.query(qn, sn, workspace=ws, bucketed=True)
        torch.cuda.synchronize()
        _equal(got, want)
    model.close()


def test_bucketed_query_of_fp64_model_is_the_query():
    _say("bucket / bucketed query of an FP64 model")
    model, P, q, sg = _setup(True, precision="fp64", n_queries=3000)
    model.fit(P)
    ref = {k: v.clone() for k, v in model.query(q, sg).items()}
    model.bucket(q)
    got = model.query(q, sg, bucketed=True)
    torch.cuda.synchronize()
    _equal(got, ref)
    model.close()
