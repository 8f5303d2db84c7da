"""The C ABI's ownership contract on the GPU: a model created, fitted and queried
entirely in caller-owned (torch) buffers through the raw entry points, and the
host-detected errors of undersized or misplaced buffers (KSDF_ERR_WORKSPACE,
KSDF_ERR_INVALID_ARGUMENT) that leave every kernel unlaunched."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2603_29227_amd import ksdf, scenes

pytestmark = pytest.mark.gpu

ERR_ARG, ERR_WS, ERR_UNSUP = -1, -3, -6


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _raw_model(wl, cells, flags=0, precision=ksdf.FP32):
    L = ksdf.lib()
    hp = ksdf.Hyper(wl.ell, wl.noise_var, -1.0, 8, precision, 1e6, flags, 0)
    off = np.ascontiguousarray(cells.offsets, np.int32)
    smp = np.ascontiguousarray(cells.samples, np.int32)
    keys = np.ascontiguousarray(cells.keys, np.int32)
    args = (cells.n, off.ctypes.data, smp.ctypes.data, keys.ctypes.data, ksdf._d3(wl.origin), wl.h,
            len(wl.points), ctypes.byref(hp), None, None)
    return L, hp, args


def test_raw_abi_model_in_torch_buffers_matches_the_model_class():
    _say("raw C ABI: create, attach, fit, query in torch buffers")
    wl = scenes.small_room_workload(n_queries=2048, cfg_id=51)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    L, hp, args = _raw_model(wl, cells, flags=ksdf.FIT_ADJOINT)
    nb = L.ksdf_model_bytes(*args)
    assert nb > 0
    store = torch.empty(nb, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    # too small, then misaligned: refused before any work
    assert L.ksdf_model_create(*args, _p(store), nb - 1, _stream(), ctypes.byref(h)) == ERR_WS
    assert not h.value
    big = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    assert L.ksdf_model_create(*args, ctypes.c_void_p(big.data_ptr() + 4), nb, _stream(),
                               ctypes.byref(h)) == ERR_ARG
    assert L.ksdf_model_create(*args, _p(store), nb, _stream(), ctypes.byref(h)) == 0
    ib = L.ksdf_model_index_bytes(h)
    assert ib >= 4
    lst = torch.empty(ib, dtype=torch.uint8, device="cuda")
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    sg = torch.from_numpy(wl.sign).cuda()
    Q = len(q)
    out = {k: torch.empty(s_, dtype=torch.float32, device="cuda")
           for k, s_ in (("mean", Q), ("grad", (Q, 3)), ("var", Q), ("var_f", Q))}
    am = torch.empty(Q, dtype=torch.int32, device="cuda")
    st = torch.empty(Q, dtype=torch.uint8, device="cuda")
    assert L.ksdf_fit_cells(h, _p(pts), ksdf.DTYPE_F32, len(pts), None, ctypes.byref(hp), None,
                            _stream()) == 0
    qws = L.ksdf_query_workspace_bytes(h, Q)
    ws = torch.empty(max(qws, 1), dtype=torch.uint8, device="cuda")

    def query(ws_bytes):
        return L.ksdf_query(h, _p(q), Q, _p(sg), _p(out["mean"]), _p(out["grad"]), _p(out["var"]),
                            _p(out["var_f"]), None, _p(am), _p(st), _p(ws), ws_bytes, _stream())

    # queries need the candidate lists
    assert query(qws) == ERR_ARG
    assert L.ksdf_model_attach_index(h, _p(lst), ib - 1, _stream()) == ERR_WS
    assert L.ksdf_model_attach_index(h, _p(lst), ib, _stream()) == 0
    if qws > 0:
        assert query(qws - 1) == ERR_WS
    assert query(qws) == 0
    # the same through the Model class (its own torch store)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       adjoint=True)
    model.fit(pts)
    ref = model.query(q, sg)
    torch.cuda.synchronize()
    for k in ("mean", "grad", "var", "var_f"):
        assert torch.equal(out[k], ref[k]), k
    assert torch.equal(am, ref["argmin"]) and torch.equal(st, ref["status"])
    n_cells, nnz, max_m, entries, dev_bytes = (ctypes.c_int(), ctypes.c_long(), ctypes.c_int(),
                                               ctypes.c_long(), ctypes.c_size_t())
    L.ksdf_model_info(h, ctypes.byref(n_cells), ctypes.byref(nnz), ctypes.byref(max_m),
                      ctypes.byref(entries), ctypes.byref(dev_bytes))
    assert dev_bytes.value == nb + ib and entries.value * 4 == ib
    L.ksdf_model_destroy(h)
    model.close()


def test_undersized_workspaces_are_refused_on_the_host():
    """Every call that takes a workspace refuses one below its *_workspace_bytes query
    (or a null one) with KSDF_ERR_WORKSPACE, before any launch: the outputs stay as
    they were."""
    _say("undersized workspaces: query, fit_query, backward, refit, BHM tau")
    wl = scenes.small_room_workload(n_queries=512, cfg_id=52)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       adjoint=True)
    L, h = model._lib, model._h
    pts = torch.from_numpy(wl.points).cuda()
    q = torch.from_numpy(wl.queries).cuda()
    Q = len(q)
    model.fit(pts)
    out = model._out(Q, q.device)
    for t in out.values():
        t.fill_(7)
    s = _stream()

    def ws_for(n):
        return torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")

    need = L.ksdf_query_workspace_bytes(h, Q)
    assert need > 0
    ws = ws_for(need)
    assert L.ksdf_query(h, _p(q), Q, None, _p(out["mean"]), _p(out["grad"]), _p(out["var"]),
                        None, None, None, None, _p(ws), need - 1, s) == ERR_WS
    assert L.ksdf_query(h, _p(q), Q, None, _p(out["mean"]), _p(out["grad"]), _p(out["var"]),
                        None, None, None, None, None, need, s) == ERR_WS
    need = L.ksdf_fit_query_workspace_bytes(h, Q)
    ws = ws_for(need)
    assert L.ksdf_fit_query(h, _p(pts), ksdf.DTYPE_F32, len(pts), None, ctypes.byref(model.hyper),
                            None, _p(q), Q, None, _p(out["mean"]), _p(out["grad"]), _p(out["var"]),
                            None, None, None, None, _p(ws), need - 1, s) == ERR_WS
    need = L.ksdf_backward_workspace_bytes(h, Q)
    ws = ws_for(need)
    dm = torch.ones(Q, dtype=torch.float32, device="cuda")
    dp = torch.full((Q, 3), 7.0, dtype=torch.float32, device="cuda")
    dh = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    assert L.ksdf_query_backward(h, _p(q), Q, None, None, _p(dm), None, None, None, _p(dp), _p(dh),
                                 _p(ws), need - 1, s) == ERR_WS
    need = L.ksdf_refit_workspace_bytes(h, 16)
    ws = ws_for(need)
    dirty = torch.ones(cells.n, dtype=torch.float32, device="cuda")
    qc = torch.zeros(cells.n, dtype=torch.float32, device="cuda")
    sel = torch.empty(16, dtype=torch.int32, device="cuda")
    nsel = torch.empty(1, dtype=torch.int32, device="cuda")
    assert L.ksdf_refit_cells(h, _p(pts), ksdf.DTYPE_F32, len(pts), None, _p(dirty), _p(qc), 0.5, 16,
                              _p(sel), _p(nsel), None, _p(ws), need - 1, s) == ERR_WS
    K = 100
    need = L.ksdf_bhm_tau_workspace_bytes(K)
    ws = ws_for(need)
    lay = ksdf._bhm_layout((0, 0, 0), 0.16, (4, 4, 4), 7, 100.0)
    bb = torch.full((64,), -1, dtype=torch.int32, device="cuda")
    w = torch.zeros(344, dtype=torch.float64, device="cuda")
    tau = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert L.ksdf_bhm_update_tau(ctypes.byref(lay), _p(bb), _p(w), _p(q), ksdf.DTYPE_F32, K, 0.5,
                                 _p(tau), _p(ws), need - 1, s) == ERR_WS
    torch.cuda.synchronize()
    for t in out.values():
        assert torch.all(t == 7)
    assert torch.all(dp == 7) and torch.all(dh == 7) and torch.all(dirty == 1) and tau.item() == 0
    # a model without room for the dense inverses refuses the matrix-core tuning
    with pytest.raises(ksdf.KsdfError, match="DENSE_INV"):
        model.set_tuning(query_split=1, query_mfma=1)
    model.close()
