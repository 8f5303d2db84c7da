"""Launch-shape autotuner.

The knobs (``ksdf_tuning``): query bucketing granularity (sub-boxes per index-box
edge: 1, 2, 4), query block size (64 or 256 threads), persistent fused fit+query
launch or per-bucket fits followed by the query launch, the smallest fit m bucket
(16, 32, 64: cells below it run in the kernel sized for it), and the query in one
kernel or in two with the queries regrouped by argmin cell between them.  ``tune`` times every
combination on the caller's own data (the fit+query step, median of a few runs, after
a warm-up) and keeps the fastest; the outputs do not depend on the choice.  Results
are cached in a JSON file keyed by device (architecture and compute-unit count) and a
workload signature (cell count,
m histogram, query count to a power of two, precision, K), so a later process
applies them without timing (``apply``).
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
             query_split=(0, 1))
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def signature(model, n_queries: int) -> str:
    m = np.diff(np.asarray(model.cells.offsets))
    hist = [int(np.sum(m <= 16)), int(np.sum((m > 16) & (m <= 32))), int(np.sum((m > 32) & (m <= 64))),
            int(np.sum(m > 64))]
    qb = 1 << max(int(n_queries) - 1, 0).bit_length()
    props = torch.cuda.get_device_properties(model.device)
    name = f"{props.gcnArchName.split(':')[0]}x{props.multi_processor_count}"
    return (f"{name}|cells={model.n_cells}|mhist={'/'.join(map(str, hist))}|q<={qb}|"
            f"prec={model.precision}|k={model.hyper.k_fuse}")


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(model, n_queries: int, cache_path: str = DEFAULT_CACHE) -> Optional[dict]:
    """Set the cached tuning for this model and query count; None if there is none."""
    hit = _load(cache_path).get(signature(model, n_queries))
    if hit is None:
        return None
    model.set_tuning(**hit["tuning"])
    return hit["tuning"]


def _time_step(model, points, queries, sign, out, reps: int) -> float:
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    model.fit_query(points, queries, sign, out=out)  # warm-up for this shape
    times = []
    for _ in range(reps):
        e0.record(stream)
        model.fit_query(points, queries, sign, out=out)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def tune(model, points: torch.Tensor, queries: torch.Tensor, sign=None, reps: int = 3,
         cache_path: Optional[str] = DEFAULT_CACHE, log=None) -> dict:
    """Time every knob combination on this model's fit+query step; keep and cache the
    fastest.  Returns {"tuning", "ms", "table"}."""
    out = model._out(len(queries), queries.device)
    keys = list(KNOBS)
    table = []
    for combo in itertools.product(*(KNOBS[k] for k in keys)):
        t = dict(zip(keys, combo))
        if model.precision == FP64 and (t["fused"] == 1 or t["fit_min_bucket"] != 16 or
                                        t["query_split"] == 1):
            continue  # FP64 models fit per cell and query on the plain path
        if t["fused"] == 1 and t["query_split"] == 1:
            continue  # the fused launch runs the query in one pass
        model.set_tuning(**t)
        ms = _time_step(model, points, queries, sign, out, reps)
        table.append((ms, t))
        if log:
            log(f"tune {t} {ms:.3f} ms")
    table.sort(key=lambda r: r[0])
    best_ms, best = table[0]
    model.set_tuning(**best)
    res = {"tuning": best, "ms": round(best_ms, 4),
           "table": [{"ms": round(ms, 4), **t} for ms, t in table]}
    if cache_path:
        cache = _load(cache_path)
        cache[signature(model, len(queries))] = {"tuning": best, "ms": res["ms"]}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return res
