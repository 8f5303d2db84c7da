"""ksdf_query_noalloc (the query for callers that cannot allocate) against ksdf_query
through the C ABI: the same outputs, bit for bit, on two calls in a row (the second
with fewer queries, so it runs on what the first left in the fixed scratch), the
size limit refused on the host, and nothing allocated by torch during the calls."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2603_29227_amd import ksdf, scenes

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20   # KSDF_NOALLOC_SCRATCH_BYTES


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _outs(Q):
    f = dict(device="cuda")
    return dict(mean=torch.full((Q,), 7.0, dtype=torch.float32, **f),
                grad=torch.full((Q, 3), 7.0, dtype=torch.float32, **f),
                var=torch.full((Q,), 7.0, dtype=torch.float32, **f),
                var_f=torch.full((Q,), 7.0, dtype=torch.float32, **f),
                grad_var=torch.full((Q, 3), 7.0, dtype=torch.float32, **f),
                argmin=torch.full((Q,), -7, dtype=torch.int32, **f),
                status=torch.full((Q,), 255, dtype=torch.uint8, **f))


def _call(L, fn, h, q, sg, o, *ws):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return fn(h, _p(q), len(q), _p(sg), _p(o["mean"]), _p(o["grad"]), _p(o["var"]), _p(o["var_f"]),
              _p(o["grad_var"]), _p(o["argmin"]), _p(o["status"]), *ws, s)


@pytest.mark.parametrize("split", [1, 0])
def test_noalloc_query_matches_query_on_two_calls(split):
    print(f"[gpu-case] ksdf_query_noalloc vs ksdf_query, query_split={split}", flush=True)
    wl = scenes.small_room_workload(n_queries=60_000, uneven=True, cfg_id=61)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var)
    model.set_tuning(query_split=split)
    model.fit(torch.from_numpy(wl.points).cuda())
    L, h = model._lib, model._h
    q_all = torch.from_numpy(wl.queries).cuda()
    sg_all = torch.from_numpy(wl.sign).cuda()
    for Q in (60_000, 23_457):          # the second call is smaller
        q, sg = q_all[:Q].contiguous(), sg_all[:Q].contiguous()
        nb = L.ksdf_query_workspace_bytes(h, Q)
        assert 0 < nb <= SCRATCH
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        ref = _outs(Q)
        assert _call(L, L.ksdf_query, h, q, sg, ref, _p(ws), nb) == 0
        got = _outs(Q)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        assert _call(L, L.ksdf_query_noalloc, h, q, sg, got) == 0
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        for k in ref:
            assert torch.equal(ref[k], got[k]), (Q, k)
    model.close()


def test_noalloc_query_refuses_sizes_beyond_the_scratch():
    print("[gpu-case] ksdf_query_noalloc size limit", flush=True)
    wl = scenes.sphere_workload(n_queries=16)
    wl = scenes.Workload(**{**wl.__dict__, "points": wl.points.astype(np.float32),
                            "queries": wl.queries.astype(np.float32)})
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var)
    model.fit(torch.from_numpy(wl.points).cuda())
    L, h = model._lib, model._h
    big = 1
    while L.ksdf_query_workspace_bytes(h, big) <= SCRATCH:
        big *= 2
    # the host refuses before touching the (unallocated) point and output arrays
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dummy = torch.zeros(4, dtype=torch.float32, device="cuda")
    rc = L.ksdf_query_noalloc(h, _p(dummy), big, None, _p(dummy), _p(dummy), _p(dummy), None, None,
                              None, None, s)
    assert rc == -3, rc
    assert b"scratch" in L.ksdf_last_error()
    model.close()
