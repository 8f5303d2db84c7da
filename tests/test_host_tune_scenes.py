"""Host logic without a GPU: the autotuner's candidate rules and cache, and the
synthetic BHM weights that stand in for a trained front-end."""
import json

import numpy as np

from paper_2603_29227_amd import scenes, tune


def test_tuner_candidate_rules():
    base = dict(query_sub=2, query_block=64, fused=0, fit_min_bucket=16, query_split=1,
                query_lanes=0, query_pairs=0, query_mfma=0)
    assert tune._valid(base, fp64=False)
    assert not tune._valid({**base, "query_split": 0, "query_lanes": 1}, fp64=False)
    assert not tune._valid({**base, "fused": 1}, fp64=False)          # split + fused
    assert not tune._valid({**base, "query_split": 0, "query_pairs": 1}, fp64=False)
    assert tune._valid({**base, "query_pairs": 1}, fp64=False)
    assert not tune._valid({**base, "query_pairs": 1}, fp64=True)
    assert not tune._valid({**base, "query_split": 0, "fit_min_bucket": 32}, fp64=True)
    assert tune._valid({**base, "query_split": 0}, fp64=True)
    assert tune._valid({**base, "query_mfma": 1}, fp64=False)
    assert not tune._valid({**base, "query_mfma": 1, "query_split": 0}, fp64=False)
    assert not tune._valid({**base, "query_mfma": 1, "query_lanes": 1}, fp64=False)
    assert not tune._valid({**base, "query_mfma": 1}, fp64=True)
    # every knob the C struct accepts is searched
    assert set(tune.KNOBS) == {"query_sub", "query_block", "fused", "fit_min_bucket",
                               "query_split", "query_lanes", "backward_lanes", "query_pairs",
                               "query_mfma"}


def test_tuner_cache_round_trip(tmp_path):
    path = str(tmp_path / "cache.json")
    tune._store(path, "sig-a", {"query_sub": 4}, 1.23456)
    tune._store(path, "sig-b", {"query_sub": 2}, 2.0)
    data = json.load(open(path))
    assert data["sig-a"] == {"tuning": {"query_sub": 4}, "ms": 1.2346}
    assert set(data) == {"sig-a", "sig-b"}
    tune._store(None, "sig-c", {}, 0.0)   # no path: nothing written


def test_bhm_weights_layout():
    wl = scenes.small_room_workload(n_queries=16)
    b = scenes.bhm_weights(wl)
    nh = b["hinges"]
    ids = b["box_bhm"][b["box_bhm"] >= 0]
    n_maps = len(ids)
    assert np.array_equal(np.sort(ids), np.arange(n_maps))           # ids are dense
    w = b["weights"].reshape(n_maps, nh ** 3 + 1)
    assert np.all(np.abs(w[:, :-1]) == 2.0) and np.all(w[:, -1] == 0.0)
    # every surface sample lies in a box that has a map
    key = np.floor((np.asarray(wl.points, np.float64) - b["origin"]) / b["box"]).astype(np.int64)
    dims = b["dims"]
    flat = (key[:, 0] * dims[1] + key[:, 1]) * dims[2] + key[:, 2]
    assert np.all(b["box_bhm"][flat] >= 0)
    assert b["gamma"] == 1.0 / (2 * 0.016 ** 2)
