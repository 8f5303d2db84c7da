"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by
element, on seeded synthetic workloads (see tests/parity.py for the tolerances)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_29227_amd import ksdf, scenes
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def gpu_run(wl, queries=None, sign=None, precision="fp32", k_fuse=8, query_box=None, svar=None,
            cells=None):
    cells = cells or ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                                      wl.m_cap_grid, wl.key_lo)
    q = wl.queries if queries is None else queries
    s = wl.sign if (queries is None and sign is None) else sign
    dt = torch.float64 if precision == "fp64" else torch.float32
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       k_fuse=k_fuse, precision=precision, query_box=query_box)
    pts = torch.from_numpy(np.ascontiguousarray(wl.points)).to("cuda", dt)
    st = torch.zeros(max(cells.n, 1), dtype=torch.uint8, device="cuda")
    sv = None if svar is None else torch.from_numpy(svar).to("cuda", dt)
    model.fit(pts, sample_var=sv, cell_status=st)
    qt = torch.from_numpy(np.ascontiguousarray(q)).to("cuda", dt)
    sg = None if s is None else torch.from_numpy(np.ascontiguousarray(s)).to("cuda")
    out = model.query(qt, sg, grad_var=True)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["cell_status"] = st.cpu().numpy()[:cells.n]
    return model, cells, res


def oracle_run(wl, cells, queries, sign, precision, k_fuse=8, svar=None):
    oc = oracle.Cells(cells.offsets, cells.samples, cells.keys,
                      np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var, svar=svar)
    return oracle.query(wl.points, oc, f, queries, wl.ell, wl.noise_var, k_fuse=k_fuse,
                        sign=sign, svar=svar, all_candidates=True)


def test_sphere_fp64_plain_path_matches_oracle():
    _say("sphere fp64 full 10k queries")
    wl = scenes.sphere_workload()
    _, cells, g = gpu_run(wl, precision="fp64")
    o = oracle_run(wl, cells, wl.queries, wl.sign, "fp64")
    rep = assert_parity(g, o, wl.ell, "fp64", label="sphere fp64")
    assert rep["mean_err_max"] < 1e-10


def test_sphere_fp32_matches_oracle():
    _say("sphere fp32")
    wl = scenes.sphere_workload()
    wl32 = scenes.Workload(**{**wl.__dict__, "points": wl.points.astype(np.float32),
                              "queries": wl.queries.astype(np.float32)})
    _, cells, g = gpu_run(wl32, precision="fp32")
    o = oracle_run(wl32, cells, wl32.queries, wl32.sign, "fp32")
    assert_parity(g, o, wl.ell, "fp32", label="sphere fp32")


@pytest.mark.parametrize("uneven", [False, True])
def test_small_room_fp32_matches_oracle(uneven):
    _say(f"small room fp32 uneven={uneven}")
    wl = scenes.small_room_workload(n_queries=4096, uneven=uneven)
    _, cells, g = gpu_run(wl)
    o = oracle_run(wl, cells, wl.queries, wl.sign, "fp32")
    rep = assert_parity(g, o, wl.ell, "fp32", label=f"small room uneven={uneven}")
    print(rep, flush=True)


def test_per_sample_variance_fp32():
    _say("per-sample variance")
    wl = scenes.small_room_workload(n_queries=1024, cfg_id=21)
    rng = np.random.default_rng(0)
    sv = rng.uniform(2e-5, 3e-4, len(wl.points)).astype(np.float32)
    _, cells, g = gpu_run(wl, svar=sv)
    o = oracle_run(wl, cells, wl.queries, wl.sign, "fp32", svar=sv.astype(np.float64))
    assert_parity(g, o, wl.ell, "fp32", label="per-sample variance")


def test_queries_outside_index_use_exact_scan():
    _say("queries outside the index lattice")
    wl = scenes.sphere_workload(n_queries=64)
    q = np.array([[30.0, 0.0, 0.0], [-5.0, 7.0, 2.0], [0.0, 0.0, -12.0], [0.3, 0.2, 0.1]])
    _, cells, g = gpu_run(wl, queries=q, sign=np.ones(4, np.int8), precision="fp64")
    assert np.all((g["status"][:3] & ksdf.Q_OUTSIDE_INDEX) != 0)
    assert (g["status"][3] & ksdf.Q_OUTSIDE_INDEX) == 0
    o = oracle_run(wl, cells, q, np.ones(4, np.int8), "fp64")
    assert_parity(g, o, wl.ell, "fp64", label="outside index")


def test_k_fuse_larger_than_cell_count_and_single_cell():
    _say("single cell, k_fuse 8")
    rng = np.random.default_rng(3)
    pts = (rng.normal(size=(20, 3)) * 0.05).astype(np.float64)
    wl = scenes.Workload(99, "tiny", pts, (0.0, 0.0, 0.0), 1.0, 0.5, 32, 1,
                         rng.normal(size=(50, 3)) * 0.5, np.ones(50, np.int8))
    _, cells, g = gpu_run(wl, precision="fp64")
    assert cells.n >= 1
    o = oracle_run(wl, cells, wl.queries, wl.sign, "fp64")
    assert_parity(g, o, wl.ell, "fp64", label="tiny")


def test_failed_cells_are_excluded_and_reported():
    _say("non-SPD cells")
    # duplicated samples with zero noise cannot be factored in any precision
    base = np.array([[0.1, 0.1, 0.1], [2.1, 0.1, 0.1]])
    pts = np.repeat(base, 3, 0).astype(np.float32)
    wl = scenes.Workload(98, "dup", pts, (0.0, 0.0, 0.0), 1.0, 0.5, 8, 1,
                         np.array([[0.5, 0.5, 0.5], [1.9, 0.2, 0.2]], np.float32),
                         np.ones(2, np.int8), noise_var=0.0)
    _, cells, g = gpu_run(wl)
    assert np.all(g["cell_status"] & ksdf.C_FAILED)
    assert np.all(g["status"] & ksdf.Q_NO_VALID_CELL)
    assert np.all(np.isinf(g["mean"])) and np.all(g["var_f"] == 1.0) and np.all(g["grad"] == 0)
    assert np.all(np.isposinf(g["grad_var"]))


def test_ill_conditioned_cells_fall_back_to_fp64():
    _say("forced FP64 fallback")
    wl = scenes.small_room_workload(n_queries=512, cfg_id=22)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       cond_threshold=10.0)
    pts = torch.from_numpy(wl.points).cuda()
    st = torch.zeros(cells.n, dtype=torch.uint8, device="cuda")
    model.fit(pts, cell_status=st)
    out = model.query(torch.from_numpy(wl.queries).cuda(), torch.from_numpy(wl.sign).cuda())
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert np.all(st.cpu().numpy() & ksdf.C_FP64)
    o = oracle_run(wl, cells, wl.queries, wl.sign, "fp32")
    assert_parity(g, o, wl.ell, "fp32", label="all FP64 refit")


def test_empty_query_and_argument_errors():
    _say("empty query, argument errors")
    wl = scenes.sphere_workload(n_queries=8)
    model, cells, _ = gpu_run(wl, precision="fp64")
    out = model.query(torch.zeros(0, 3, dtype=torch.float64, device="cuda"))
    assert out["mean"].numel() == 0
    with pytest.raises(ksdf.KsdfError):
        ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=float("nan"), precision="fp64")
    with pytest.raises(ksdf.KsdfError):
        ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=0.2, k_fuse=40, precision="fp64")
    bad = ksdf.CellSet(cells.offsets.copy(), cells.samples.copy(), cells.keys.copy())
    bad.samples[0] = len(wl.points) + 5
    with pytest.raises(ksdf.KsdfError):
        ksdf.Model(bad, len(wl.points), wl.origin, wl.h, precision="fp64")


def test_far_queries_over_sloped_patches_fp32():
    """Far from a sloped patch, the corner of the samples' bounding box can be much
    nearer than any sample; against that reference every kernel term is tiny and the
    smaller ones underflow in FP32.  Regression for the nearest-sample fallback."""
    _say("far queries over sloped patches (FP32 underflow regression)")
    rng = np.random.default_rng(5)
    n1 = 100
    xy = (np.stack(np.meshgrid(np.arange(n1), np.arange(n1), indexing="ij"), -1).reshape(-1, 2)
          + rng.random((n1 * n1, 2))) * 0.03
    z = 0.6 * xy[:, 0] + 0.35 * xy[:, 1] + rng.normal(0, 0.005, len(xy))
    pts = np.column_stack([xy, z]).astype(np.float32)
    q = np.column_stack([rng.uniform(0, 3, 4000), rng.uniform(0, 3, 4000),
                         rng.uniform(6, 16, 4000)]).astype(np.float32)
    wl = scenes.Workload(90, "sloped_patch", pts, (0.0, 0.0, 0.0), 0.5, 0.25, 32, 1, q,
                         np.ones(len(q), np.int8))
    model, cells, res = gpu_run(wl)
    ora = oracle_run(wl, cells, q, wl.sign, "fp32")
    rep = assert_parity(res, ora, wl.ell, "fp32", wl.sign, label="sloped far")
    assert np.all(np.isfinite(res["mean"]))
    print("sloped far:", rep["mean_err_max"], flush=True)
    # the pair form of pass 1 takes the same nearest-sample fallback
    model.set_tuning(query_split=1, query_pairs=1)
    out = model.query(torch.from_numpy(q).cuda(), torch.from_numpy(wl.sign).cuda(), grad_var=True)
    torch.cuda.synchronize()
    res2 = {k: v.cpu().numpy() for k, v in out.items()}
    assert_parity(res2, ora, wl.ell, "fp32", wl.sign, label="sloped far, pairs")


def test_fp64_fallback_decision_matches_exact_condition_number():
    """The FP64 refit rule (Cholesky in FP64 only where cond_2(A) > 1e6) against the
    oracle's exact cond_2.  Cells in the strong-correlation limit of App. E (64 samples
    within 1e-5 m of one point) have cond_2 = (64 + s2) / s2, so per-sample variances
    place them on both sides of the threshold: s2 = 2e-4, 1e-4, 8e-5 (cond 3.2e5 to
    8e5) stay FP32, s2 = 5e-5, 4e-5, 2e-5 (1.28e6 to 3.2e6) go to FP64.  The natural
    cell of a noisy patch (cond about 3.6e5) stays FP32.  Queries around the clusters then
    match the oracle."""
    _say("FP64 fallback decision at cond 1e6 (strong-correlation cells)")
    rng = np.random.default_rng(11)
    s2s = [2e-4, 1e-4, 8e-5, 5e-5, 4e-5, 2e-5]
    pts, sv = [], []
    for i, s2 in enumerate(s2s):
        pts.append(np.array([0.5 + 2.0 * i, 0.5, 0.5]) + rng.uniform(-1e-5, 1e-5, (64, 3)))
        sv.append(np.full(64, s2))
    xy = rng.uniform(0, 1, (400, 2))
    pts.append(np.column_stack([xy[:, 0] + 0.0, xy[:, 1] + 3.0, 0.5 + rng.normal(0, 0.005, 400)]))
    sv.append(np.full(400, 1e-4))
    P = np.concatenate(pts).astype(np.float32)
    S = np.concatenate(sv).astype(np.float32)
    q = np.concatenate([c[:1] + rng.normal(0, 0.2, (64, 3)) for c in pts]).astype(np.float32)
    wl = scenes.Workload(97, "cond_cells", P, (0.0, 0.0, 0.0), 1.0, 0.5, 64, 1, q,
                         np.ones(len(q), np.int8))
    model, cells, g = gpu_run(wl, svar=S)
    oc = oracle.Cells(cells.offsets, cells.samples, cells.keys, (cells.keys + 0.5) * 1.0)
    cond, _, _ = oracle.cond2(P, oc, wl.ell, wl.noise_var, svar=S.astype(np.float64))
    fp64 = (g["cell_status"] & ksdf.C_FP64) != 0
    print("cells", cells.n, "m", cells.m.tolist(), "cond", np.round(cond).tolist(), "fp64", fp64.tolist(),
          flush=True)
    assert (cond > 1e6).sum() == 3 and (cond < 1e6).sum() == cells.n - 3
    np.testing.assert_array_equal(fp64, cond > 1e6)
    o = oracle_run(wl, cells, q, wl.sign, "fp32", svar=S.astype(np.float64))
    assert_parity(g, o, wl.ell, "fp32", label="strong-correlation cells")


@pytest.mark.parametrize("tuning", [
    dict(query_split=1, query_block=64, query_sub=2, query_lanes=0),
    dict(query_split=1, query_block=256, query_sub=1, query_lanes=1),
    dict(query_split=0, query_block=64, query_sub=4),
])
def test_tied_candidates_give_the_same_answer_in_any_query_order(tuning):
    """Queries on the lattice of cell faces and centres sit exactly midway between cell
    centres in x and y, so FP32 candidate distances tie.  The K nearest cells are kept in (distance,
    id) order whichever path a wave takes (the wave-shared scan of one index box, or each
    lane's own scan) and whatever the wave's other queries are: shuffling the queries,
    which regroups them into other waves, changes no output bit.  The outputs also pass
    parity with the oracle (ties at the K-th place accepted as R6 reads them)."""
    _say(f"tied candidate distances, shuffled query order, {tuning}")
    wl = scenes.small_room_workload(n_queries=16, cfg_id=48)
    # x and y on the half-lattice of cell faces and centres (tie groups of up to four
    # mirrored cells), z generic
    half = wl.h / 2
    rng = np.random.default_rng(48)
    pts = [np.array([wl.origin[0] + half * i, wl.origin[1] + half * j, rng.uniform(0.05, 2.95)])
           for i in range(1, 80) for j in range(1, 64) for _ in range(2)]
    q = np.asarray(pts, dtype=np.float32)
    q = q[np.all((q > 0.05) & (q < np.array([9.95, 7.95, 2.95])), axis=1)]
    assert len(q) > 5000
    sign = np.ones(len(q), dtype=np.int8)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var)
    model.set_tuning(**tuning)
    model.fit(torch.from_numpy(wl.points).cuda())
    perm = np.random.default_rng(3).permutation(len(q))
    a = model.query(torch.from_numpy(q).cuda(), torch.from_numpy(sign).cuda())
    a = {k: v.clone() for k, v in a.items()}
    b = model.query(torch.from_numpy(np.ascontiguousarray(q[perm])).cuda(),
                    torch.from_numpy(sign[perm]).cuda())
    torch.cuda.synchronize()
    pt = torch.from_numpy(perm).cuda()
    for k in a:
        assert torch.equal(a[k][pt], b[k]), f"{k} depends on the query order"
    o = oracle_run(wl, cells, q, sign, "fp32")
    rep = assert_parity({k: v.cpu().numpy() for k, v in a.items()}, o, wl.ell, "fp32", sign,
                        label=f"tied candidates {tuning}")
    print(rep, flush=True)
    model.close()
