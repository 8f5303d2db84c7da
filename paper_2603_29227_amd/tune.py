"""Launch-shape autotuner.

The knobs (``ksdf_tuning``): query bucketing granularity (sub-boxes per index-box
edge: 1, 2, 4), query block size (64 or 256 threads), persistent fused fit+query
launch or per-bucket fits followed by the query launch, the smallest fit m bucket
(16, 32, 64: cells below it run in the kernel sized for it), the query in one kernel
or in two with the queries regrouped by argmin cell between them, and whether each
lane reads its own cells (sparse queries) in the query and in the backward.  The
outputs do not depend on the choice.

Three calls are tuned separately, each on the caller's own data (median of a few
timed runs after a warm-up): ``tune`` the fit + query step, ``tune_query`` a query
alone, ``tune_backward`` the backward.  Results are cached in a JSON file keyed by
device (architecture and compute-unit count), the call and a workload signature
(cell count, m histogram, query count to a power of two, precision, K), so a later
process applies them without timing (``apply``).
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Optional

import numpy as np
import torch

from .ksdf import FP64

KNOBS = dict(query_sub=(1, 2, 4), query_block=(64, 256), fused=(0, 1), fit_min_bucket=(16, 32, 64),
             query_split=(0, 1), query_lanes=(0, 1), backward_lanes=(0, 1), query_pairs=(0, 1), query_mfma=(0, 1))
QUERY_KNOBS = ("query_sub", "query_block", "query_split", "query_lanes", "query_pairs",
               "query_mfma")
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def signature(model, n_queries: int, kind: str = "fit_query") -> str:
    m = np.diff(np.asarray(model.cells.offsets))
    hist = [int(np.sum(m <= 16)), int(np.sum((m > 16) & (m <= 32))), int(np.sum((m > 32) & (m <= 64))),
            int(np.sum(m > 64))]
    qb = 1 << max(int(n_queries) - 1, 0).bit_length()
    props = torch.cuda.get_device_properties(model.device)
    name = f"{props.gcnArchName.split(':')[0]}x{props.multi_processor_count}"
    prefix = "" if kind == "fit_query" else f"{kind}|"
    return (f"{prefix}{name}|cells={model.n_cells}|mhist={'/'.join(map(str, hist))}|q<={qb}|"
            f"prec={model.precision}|k={model.hyper.k_fuse}")


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: Optional[str], key: str, tuning: dict, ms: float):
    if not path:
        return
    cache = _load(path)
    cache[key] = {"tuning": tuning, "ms": round(ms, 4)}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached(model, n_queries: int, kind: str = "fit_query", cache_path: str = DEFAULT_CACHE):
    """The cached tuning for this call, or None."""
    hit = _load(cache_path).get(signature(model, n_queries, kind))
    return None if hit is None else hit["tuning"]


def apply(model, n_queries: int, kind: str = "fit_query", cache_path: str = DEFAULT_CACHE):
    """Set the cached tuning for this call on the model; None if there is none."""
    t = cached(model, n_queries, kind, cache_path)
    if t is not None:
        if not model.dense_inverse:
            t = {**t, "query_mfma": 0}   # the model has no room for the dense inverses
        model.set_tuning(**t)
    return t


def _median_ms(fn, reps: int) -> float:
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()   # warm-up for this shape
    times = []
    for _ in range(reps):
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def _valid(t: dict, fp64: bool, dense_inverse: bool = True) -> bool:
    if fp64 and (t.get("fused", 0) == 1 or t.get("fit_min_bucket", 16) != 16 or
                 t.get("query_split", 0) == 1 or t.get("query_lanes", 0) == 1):
        return False   # FP64 models fit per cell and query on the plain path
    if t.get("fused", 0) == 1 and (t.get("query_split", 0) == 1 or t.get("query_lanes", 0) == 1):
        return False   # the fused launch runs the query in one pass
    if t.get("query_lanes", 0) == 1 and t.get("query_split", 0) == 0:
        return False   # lanes apply to the two-kernel query
    if t.get("query_pairs", 0) == 1 and (t.get("query_split", 0) == 0 or fp64 or
                                         t.get("fused", 0) == 1):
        return False   # pairs apply to the two-kernel FP32 query
    if t.get("query_mfma", 0) == 1 and (t.get("query_split", 0) == 0 or fp64 or not dense_inverse or
                                        t.get("query_lanes", 0) == 1 or t.get("fused", 0) == 1):
        return False   # the matrix-core pass 2 needs wave-shared cells in the two-kernel query
                       # and a model created with room for the dense inverses
    return True


def _search(model, keys, run, reps, log):
    table = []
    base = model.tuning()
    for combo in itertools.product(*(KNOBS[k] for k in keys)):
        t = {**base, **dict(zip(keys, combo))}
        if not _valid(t, model.precision == FP64, model.dense_inverse):
            continue
        model.set_tuning(**t)
        ms = _median_ms(run, reps)
        table.append((ms, t))
        if log:
            log(f"tune {dict(zip(keys, combo))} {ms:.3f} ms")
    table.sort(key=lambda r: r[0])
    best_ms, best = table[0]
    model.set_tuning(**best)
    return best, best_ms, table


def tune(model, points: torch.Tensor, queries: torch.Tensor, sign=None, reps: int = 3,
         cache_path: Optional[str] = DEFAULT_CACHE, log=None) -> dict:
    """Time the launch shapes of this model's fit+query step; keep and cache the
    fastest.  Returns {"tuning", "ms", "table"}."""
    out = model._out(len(queries), queries.device)
    keys = ["query_sub", "query_block", "fused", "fit_min_bucket", "query_split", "query_lanes",
            "query_pairs", "query_mfma"]
    best, ms, table = _search(model, keys, lambda: model.fit_query(points, queries, sign, out=out),
                              reps, log)
    _store(cache_path, signature(model, len(queries)), best, ms)
    return {"tuning": best, "ms": round(ms, 4), "table": [{"ms": round(t, 4), **c} for t, c in table]}


def tune_query(model, queries: torch.Tensor, sign=None, reps: int = 3,
               cache_path: Optional[str] = DEFAULT_CACHE, log=None) -> dict:
    """Time the query launch shapes for this query set on the fitted model."""
    out = model._out(len(queries), queries.device)
    best, ms, table = _search(model, list(QUERY_KNOBS), lambda: model.query(queries, sign, out=out),
                              reps, log)
    q_t = {k: best[k] for k in QUERY_KNOBS}
    _store(cache_path, signature(model, len(queries), "query"), q_t, ms)
    return {"tuning": q_t, "ms": round(ms, 4), "table": [{"ms": round(t, 4), **c} for t, c in table]}


def tune_backward(model, queries: torch.Tensor, sign, cotangents: dict, argmin, reps: int = 3,
                  cache_path: Optional[str] = DEFAULT_CACHE, log=None) -> dict:
    """Time the backward launch shapes (per-lane or wave-shared cells)."""
    c = cotangents

    def run():
        model.backward(queries, sign, c.get("d_mean"), c.get("d_grad"), c.get("d_var"),
                       c.get("d_var_f"), argmin=argmin)

    best, ms, table = _search(model, ["backward_lanes"], run, reps, log)
    b_t = {"backward_lanes": best["backward_lanes"]}
    _store(cache_path, signature(model, len(queries), "backward"), b_t, ms)
    return {"tuning": b_t, "ms": round(ms, 4), "table": [{"ms": round(t, 4), **c} for t, c in table]}
