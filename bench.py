"""Benchmark: batched local-GP SDF regression on one MI355X.

One step is one pass of the whole hot path over the indoor-room workload
(10 x 8 x 3 m room, 20 boxes + 10 cylinders, 2 cm sampling, 0.25 m cells, m <= 64):
  fit + query  every cell fitted (FP32, FP64 refit of ill-conditioned cells, adjoint
               vectors for the backward) and mean + gradient + softmin variance + GP
               variance + sign at the 256^3 grid (16,777,216 points), in the fused
               persistent launch or as separate launches, as the autotuner picked;
  backward     the collision cost sum softplus(0.3 - d + sqrt(var)) over 4,096
               trajectories x 64 waypoints (262,144 points): forward query, cost
               cotangents, adjoint to the waypoints and to (length-scale, noise).
Inputs are generated once, seeded, and resident in HBM before timing.  value = query
points of one step (grid + trajectory) / step time.  Kernel durations come from HIP
events the library records around each phase's kernel on its launch stream.  The
plain per-cell FP64 GPU path is timed on the same inputs as the comparison leg, and
the FP64 CPU oracle on a bounded sample as the CPU baseline.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector peak (published, packed issue)
PEAK_VALU_TSLOTS = 39.32      # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz lane-instructions/s
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_room_grid.txt")
KERNEL_SOURCES = {
    "query_fast": ["query_fast.hip", "query_split.h", "query_split64_wave.hip",
                   "query_split64_lane.hip", "query_split256_wave.hip", "query_split256_lane.hip",
                   "query_pairs.hip",
                   "query_dev.h", "fit_dev.h", "ff.h", "ksdf_internal.h"],
    "fused": ["fused.hip", "query_dev.h", "fit_dev.h", "ff.h", "ksdf_internal.h"],
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2603_29227_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by the same counter's reading on a plain copy of
    known size); None when there is none or the kernel's sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel") != kernel or kv.get("source_hash") != source_hash(kernel):
        return None
    try:
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["copy_scale_fetch"])
        write = float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["copy_scale_write"])
    except (KeyError, ValueError):
        return None
    return fetch + write


def copy_calibration(torch, dev):
    """A plain copy of 1 GiB, launched 3 times, for scaling the HBM byte counters."""
    x = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log("copy calibration: 3 x copy of 1073741824 bytes (read 1 GiB, write 1 GiB)")
    del x, y


def query_flops(m_mean: float, k: int) -> tuple[float, float]:
    """Algorithmic work of one forward query (independent of the kernel): per sample of
    each of the K candidate cells z^2 (3 sub + 3 FMA: 9 flop), the exponent (2), exp (1),
    a e accumulation (2); at the chosen cell gradient (6 per sample), sqrt (1), softmin
    variance (8), forward substitution for the GP variance (m^2) and the recomputed k*
    (14 per sample).  Returns (flop, transcendental count)."""
    m = m_mean
    return 14 * k * m + 30 * m + m * m, (k + 2) * m + m


def backward_flops(m_mean: float) -> float:
    """One VJP point at its argmin cell: recompute k* (14 m), gradient and its Jacobian
    (20 m), the variance adjoint by a forward and a backward substitution (2 m^2), the
    hyperparameter terms (6 m)."""
    m = m_mean
    return 40 * m + 2 * m * m


def fit_flops(m: np.ndarray) -> float:
    """Per cell: assembly of the lower triangle (5 m^2), Cholesky (m^3 / 3), the two
    triangular solves for a (2 m^2)."""
    m = m.astype(np.float64)
    return float(np.sum(m ** 3 / 3 + 7 * m * m))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 GPU leg")
    ap.add_argument("--no-matern", action="store_true", help="skip the Matern 3/2 leg")
    ap.add_argument("--no-bhm", action="store_true", help="skip the BHM sign leg")
    ap.add_argument("--no-refit", action="store_true", help="skip the streaming-refit leg")
    ap.add_argument("--no-grad-var", action="store_true",
                    help="skip timing the gradient-variance output")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-tune", action="store_true", help="use the cached tuning, do not time")
    ap.add_argument("--tune-cache", default=None, help="write the autotuner's choice to this cache")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay leg")
    ap.add_argument("--serial", action="store_true",
                    help="run the trajectory query and backward after the grid query on one "
                         "stream instead of beside it on a second stream")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB copy (scale for the HBM byte counters)")
    ap.add_argument("--cpu-queries", type=int, default=1 << 20)
    ap.add_argument("--cpu-vjp", type=int, default=1 << 16)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not built)"}), flush=True)
        sys.exit(2)

    import torch
    from paper_2603_29227_amd import ksdf, scenes, tune

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    wl = scenes.room_workload("grid", grid_n=args.grid)
    tq_np, tsg_np = scenes.room_trajectories(wl)
    log(f"room workload: {len(wl.points)} samples, {len(wl.queries)} grid queries, "
        f"{len(tq_np)} trajectory points ({time.time() - t0:.1f}s)")
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    m = cells.m
    log(f"cells: {cells.n}, m mean {m.mean():.1f}, max {m.max()}")
    qbox = (np.zeros(3), np.array([10.0, 8.0, 3.0]))
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision="fp32", query_box=qbox, adjoint=True)
    info = model.info()
    pts = torch.from_numpy(wl.points).to(dev)
    q = torch.from_numpy(wl.queries).to(dev)
    sg = torch.from_numpy(wl.sign).to(dev)
    tq = torch.from_numpy(tq_np).to(dev)
    tsg = torch.from_numpy(tsg_np).to(dev)
    Q, QT = len(q), len(tq)

    out = model._out(Q, dev)
    tout = model._out(QT, dev, status=False)
    d_mean = torch.empty(QT, dtype=torch.float32, device=dev)
    d_var = torch.empty(QT, dtype=torch.float32, device=dev)

    def cotangents():
        # cost c = sum softplus(0.3 - d + sqrt(var)): dc/dd = -sigmoid(t), dc/dvar = sigmoid(t) / (2 sqrt(var))
        sd = torch.sqrt(torch.clamp_min(tout["var"], 1e-30))
        s = torch.sigmoid(0.3 - tout["mean"] + sd)
        torch.neg(s, out=d_mean)
        torch.div(s, 2 * sd, out=d_var)

    # launch shapes: the fit+query step, the trajectory query and the backward are tuned
    # (or taken from the cache) separately
    t1 = time.time()
    if args.no_tune:
        tg = tune.cached(model, Q) or {}
        model.set_tuning(**tg)
        tg = model.tuning()
        tq_t = tune.cached(model, QT, "query") or {}
        tb_t = tune.cached(model, QT, "backward") or {}
        source = "cache"
    else:
        res = tune.tune(model, pts, q, sg, reps=2, cache_path=args.tune_cache)
        tg = res["tuning"]
        log(f"autotuner fit+query: {tg} {res['ms']:.3f} ms ({len(res['table'])} candidates)")
        rq = tune.tune_query(model, tq, tsg, reps=3, cache_path=args.tune_cache)
        tq_t = rq["tuning"]
        model.query(tq, tsg, out=tout)
        cotangents()
        rb = tune.tune_backward(model, tq, tsg, dict(d_mean=d_mean, d_var=d_var), tout["argmin"],
                                reps=3, cache_path=args.tune_cache)
        tb_t = rb["tuning"]
        log(f"autotuner trajectory query: {tq_t} {rq['ms']:.3f} ms; backward: {tb_t} {rb['ms']:.3f} ms")
        source = "timed"
    t_grid = dict(tg)
    t_traj = {**t_grid, **tq_t}
    t_bwd = {**t_traj, **tb_t}
    tuned = {"source": source, "fit_query": t_grid, "trajectory_query": tq_t, "backward": tb_t,
             "seconds": round(time.time() - t1, 1)}
    fused = t_grid["fused"] == 1
    cst = torch.zeros(cells.n, dtype=torch.uint8, device=dev)
    grads = {}
    # The trajectory query and backward need only the fit: unless the fit and the grid
    # query are one fused launch, they run on a second stream (default priority) beside
    # the grid query, with their own workspace, and join before the step ends.
    overlap = not fused and not args.serial
    traj_stream = torch.cuda.Stream()
    traj_ws = model.new_workspace(QT)

    def traj_part(ws=None):
        model.set_tuning(**t_traj)
        model.query(tq, tsg, out=tout, workspace=ws)
        cotangents()
        model.set_tuning(**t_bwd)
        grads["points"], grads["hyper"] = model.backward(tq, tsg, d_mean, None, d_var, None,
                                                         argmin=tout["argmin"], workspace=ws)

    def step(mark=None, serial=not overlap):
        main = torch.cuda.current_stream()
        model.set_tuning(**t_grid)
        if serial:
            model.fit_query(pts, q, sg, cell_status=cst, out=out)
            if mark is not None:
                mark.record(main)
            traj_part()
            return
        model.fit(pts, cell_status=cst)
        traj_stream.wait_stream(main)
        with torch.cuda.stream(traj_stream):
            traj_part(traj_ws)
        model.set_tuning(**t_grid)
        model.query(q, sg, out=out)
        if mark is not None:
            mark.record(main)
        main.wait_stream(traj_stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if overlap:
        # the two-stream step must give the serial step's results bit for bit
        step(serial=True)
        torch.cuda.synchronize()
        ref = [t.clone() for t in (*out.values(), *tout.values(), grads["points"], grads["hyper"])]
        for t in (*out.values(), *tout.values()):
            t.fill_(-1)   # so that an output the two-stream step leaves unwritten shows
        step()
        torch.cuda.synchronize()
        got = (*out.values(), *tout.values(), grads["points"], grads["hyper"])
        if not all(torch.equal(a, b) for a, b in zip(ref, got)):
            raise RuntimeError("the two-stream step differs from the serial step")
        del ref
    if args.copy_calib:
        copy_calibration(torch, dev)

    # timed region: K whole steps; the library's events time each phase's kernel
    model.set_timing(True)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    step_ms, fwd_ms = [], []
    kern = {"fused": [], "fit": [], "query": [], "query_traj": [], "backward": []}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ev[0].record(stream)
        step(mark=ev[1])
        ev[2].record(stream)
        ev[2].synchronize()
        step_ms.append(ev[0].elapsed_time(ev[2]))
        fwd_ms.append(ev[0].elapsed_time(ev[1]))
        for k in ["fused"] if fused else ["fit"]:
            kern[k] += model.timer_read(k)
        # query launches in launch order: grid then trajectory, or the reverse when the
        # trajectory part is issued first on its own stream (fused: trajectory only)
        qt = model.timer_read("query")
        bt = model.timer_read("backward")
        if not fused:
            kern["query"].append(qt[-1] if overlap else qt[0])
        if not overlap:   # beside the grid query these spans include waiting for it
            kern["query_traj"].append(qt[-1])
            kern["backward"] += bt
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_start) / args.steps * 1e3
    # the trajectory query + backward alone, on one stream (beside the grid query its
    # time is hidden in the step, and its kernels' spans include waiting): the
    # trajectory part's time and its kernels' times
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    traj_list, qt, bt = [], [], []
    for _ in range(args.steps):
        e0.record(stream)
        traj_part()
        e1.record(stream)
        e1.synchronize()
        traj_list.append(e0.elapsed_time(e1))
        qt += model.timer_read("query")
        bt += model.timer_read("backward")
    traj_ms = float(np.mean(traj_list))
    if overlap:
        kern["query_traj"], kern["backward"] = qt, bt
    model.set_timing(False)
    step_avg = float(np.mean(step_ms))
    kavg = {k: float(np.mean(v)) for k, v in kern.items() if v}
    n_fp64 = int(((cst.cpu().numpy() & ksdf.C_FP64) != 0).sum())
    st = out["status"].cpu().numpy()
    log(f"step {step_avg:.3f} ms (wall {wall:.3f}; trajectory part beside the grid query: "
        f"{overlap}), grid fit+query {np.mean(fwd_ms):.3f} ms, trajectory part alone "
        f"{traj_ms:.3f} ms, "
        f"kernels {kavg}, fp64 cells {n_fp64}")

    # graph-replayed step (same work, launches captured once)
    graph = None
    if not args.no_graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        graph = round(e0.elapsed_time(e1) / args.steps, 4)
        log(f"graph replay: {graph:.3f} ms/step")
        del g

    # cost of the optional gradient-variance output (App. C), not part of the step: the
    # grid query alone, without and with it
    model.set_tuning(**{**t_grid, "fused": 0})
    gv_out = model._out(Q, dev, grad_var=True)
    gv_ms = {}
    for name, o in () if args.no_grad_var else (("query_ms", out), ("query_with_grad_var_ms", gv_out)):
        model.query(q, sg, out=o)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            model.query(q, sg, out=o)
        e1.record(stream)
        torch.cuda.synchronize()
        gv_ms[name] = round(e0.elapsed_time(e1) / 3, 4)
    del gv_out
    gv_ms = gv_ms or None
    log(f"grid query without / with grad_var: {gv_ms}")

    # streaming refit (App. G) on the fitted room model: the grid queries' argmin cells
    # counted into the query counters, a tenth of the cells marked dirty (c2 in 1..3),
    # and the training queue's highest-priority 512 cells refitted (ranking, bucketed
    # FP32 fit with the adjoint vectors, counter reset)
    refit = None
    if not args.no_refit:
        model.set_tuning(**t_grid)
        rng = np.random.default_rng(11)
        n_dirty = max(cells.n // 10, 1)
        pick = torch.from_numpy(rng.choice(cells.n, n_dirty, replace=False)).long().to(dev)
        c2 = torch.from_numpy(rng.integers(1, 4, n_dirty).astype(np.float32)).to(dev)
        qcount = torch.zeros(cells.n, dtype=torch.float32, device=dev)
        budget = min(512, cells.n)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        model.count_queries(out["argmin"], qcount)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(3):
            model.count_queries(out["argmin"], qcount)
        e1.record(stream)
        torch.cuda.synchronize()
        count_ms = e0.elapsed_time(e1) / 3
        rms = []
        for rep_ in range(4):
            dirty = torch.zeros(cells.n, dtype=torch.float32, device=dev)
            dirty[pick] = c2
            torch.cuda.synchronize()
            e0.record(stream)
            sel, nsel = model.refit(pts, dirty, qcount, 0.5, budget)
            e1.record(stream)
            torch.cuda.synchronize()
            if rep_ > 0:
                rms.append(e0.elapsed_time(e1))
        if int(nsel.item()) != min(budget, n_dirty):
            raise RuntimeError("the refit selected an unexpected number of cells")
        refit = {"dirty_cells": n_dirty, "budget": budget, "refit_ms": round(float(np.mean(rms)), 4),
                 "cells_per_s": round(budget / (float(np.mean(rms)) * 1e-3), 1),
                 "count_queries_ms": round(count_ms, 4), "counted_queries": Q}
        log(f"streaming refit: {refit}")

    # the Matern 3/2 variant (Table I) on the same room and grid, its own FP32 model:
    # float-float fit as for the RBF, the plain one-thread-per-query kernel in FP32
    matern = None
    if not args.no_matern:
        mat = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell,
                         noise_var=wl.noise_var, precision="fp32", query_box=qbox,
                         kernel="matern32")
        mout = mat._out(Q, dev)
        mat.fit(pts)
        mat.query(q, sg, out=mout)
        torch.cuda.synchronize()
        mat.set_timing(True)
        mf, mq = [], []
        for _ in range(2):
            mat.fit(pts)
            mat.query(q, sg, out=mout)
            torch.cuda.synchronize()
            mf += mat.timer_read("fit")
            mq += mat.timer_read("query")
        mat.set_timing(False)
        mst = mout["status"].cpu().numpy()
        matern = {"fit_ms": round(float(np.mean(mf)), 4), "query_ms": round(float(np.mean(mq)), 4),
                  "query_qps": round(Q / (float(np.mean(mq)) * 1e-3), 1),
                  "no_valid_queries": int(((mst & 1) != 0).sum())}
        log(f"matern32: {matern}")
        del mout
        mat.close()

    # SDF sign from local BHM weights (synthetic weights from the scene's free-space
    # test; paper's indoor box, hinge count and kernel scale), for the grid and the
    # trajectory points
    bhm = None
    if not args.no_bhm:
        b = scenes.bhm_weights(wl)
        bargs = (b["origin"], b["box"], b["dims"], b["hinges"], b["gamma"],
                 torch.from_numpy(b["box_bhm"]).to(dev), torch.from_numpy(b["weights"]).to(dev))
        bhm = {"maps": int((b["box_bhm"] >= 0).sum()), "hinges": b["hinges"]}
        for name, pts_ in (("grid", q), ("trajectory", tq)):
            ksdf.bhm_sign(pts_, *bargs)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                sgn = ksdf.bhm_sign(pts_, *bargs)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            bhm[f"{name}_sign_ms"] = round(ms, 4)
            bhm[f"{name}_sign_qps"] = round(len(pts_) / (ms * 1e-3), 1)
        del bargs
        log(f"bhm sign: {bhm}")

    # roofline of the dominant kernel (algorithmic flops over its measured duration)
    k_fuse = int(model.hyper.k_fuse)
    fq, tr = query_flops(float(m.mean()), k_fuse)
    if fused:
        dom, dom_ms, flops = "fused", kavg["fused"], fq * Q + fit_flops(m)
    else:
        dom, dom_ms, flops = "query_fast", kavg["query"], fq * Q
    achieved = flops / (dom_ms * 1e-3) / 1e12
    slots = (fq / 2 + tr * 4) * Q   # FMA-slot equivalents; a transcendental takes 4 slots
    traffic = measured_traffic(dom)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": None if traffic is None else round(traffic),
                "kernel": dom, "kernel_ms": round(dom_ms, 4), "flop_per_launch": round(flops),
                "issue_frac": round(slots / (kavg["query" if not fused else "fused"] * 1e-3)
                                    / (PEAK_VALU_TSLOTS * 1e12), 4)}
    bflops = backward_flops(float(m.mean())) * QT
    roof_bwd = {"kernel": "bwd_wave", "kernel_ms": round(kavg["backward"], 4),
                "achieved": round(bflops / (kavg["backward"] * 1e-3) / 1e12, 3),
                "frac": round(bflops / (kavg["backward"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)}

    result = {
        "metric": "SDF queries/s (mean+grad+var) + backward queries/s vs plain path, at tolerance",
        "value": round((Q + QT) / (step_avg * 1e-3), 1),
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_avg, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"indoor room 10x8x3 m, 20 boxes + 10 cylinders, 2 cm sampling, "
                               f"{len(wl.points)} samples, {cells.n} cells (h 0.25 m, m<=64); "
                               f"{args.grid}^3 grid queries + backward of the softplus collision "
                               f"cost at 4096 x 64 trajectory points", "grid_queries": Q,
                   "trajectory_points": QT, "k_fuse": k_fuse, "ell": wl.ell,
                   "noise_var": wl.noise_var, "tuning": tuned,
                   "streams": 2 if overlap else 1},
        "fwd_qps": round(Q / (np.mean(fwd_ms) * 1e-3), 1),
        "bwd_qps": round(QT / (traj_ms * 1e-3), 1),
        "trajectory_part_ms": round(traj_ms, 4),
        "kernel_ms": {k: round(v, 4) for k, v in kavg.items()},
        "graph_ms_per_step": graph,
        "fp64_cells": n_fp64, "no_valid_queries": int(((st & 1) != 0).sum()),
        "model_device_bytes": info["device_bytes"],
        "roofline": roofline, "roofline_backward": roof_bwd,
        "grad_var_cost": gv_ms,
        "matern32": matern,
        "bhm_sign": bhm,
        "streaming_refit": refit,
    }

    if not args.no_plain:
        # the plain per-cell FP64 GPU path: one thread per query, every candidate cell in
        # FP64, the plain backward; same inputs
        plain = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell,
                           noise_var=wl.noise_var, precision="fp64", query_box=qbox, adjoint=True)
        p64, q64, tq64 = pts.double(), q.double(), tq.double()
        pout = plain._out(Q, dev)
        ptout = plain._out(QT, dev, status=False)
        dm64, dv64 = d_mean.double(), d_var.double()

        def plain_step(ev=None):
            if ev:
                ev[0].record(stream)
            plain.fit(p64)
            plain.query(q64, sg, out=pout)
            if ev:
                ev[1].record(stream)
            plain.query(tq64, tsg, out=ptout)
            plain.backward(tq64, tsg, dm64, None, dv64, None, argmin=ptout["argmin"])
            if ev:
                ev[2].record(stream)

        plain_step()
        torch.cuda.synchronize()
        pe = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        plain_step(pe)
        torch.cuda.synchronize()
        pf, pb = pe[0].elapsed_time(pe[1]), pe[1].elapsed_time(pe[2])
        ours_b = traj_ms
        result["plain_fp64"] = {"fit_query_ms": round(pf, 3), "traj_query_backward_ms": round(pb, 3),
                                "step_ms": round(pf + pb, 3),
                                "value": round((Q + QT) / ((pf + pb) * 1e-3), 1),
                                "speedup_step": round((pf + pb) / step_avg, 2),
                                "speedup_grid_fit_query": round(pf / float(np.mean(fwd_ms)), 2),
                                "speedup_trajectory_query_backward": round(pb / ours_b, 2)}
        log(f"plain fp64: grid fit+query {pf:.3f} ms, trajectory query+backward {pb:.3f} ms")
        plain.close()

    if not args.no_cpu:
        import oracle
        nthreads = oracle.threads()
        rng = np.random.default_rng(0)
        sel = np.sort(rng.choice(Q, size=min(args.cpu_queries, Q), replace=False))
        tsel = np.sort(rng.choice(QT, size=min(args.cpu_vjp, QT), replace=False))
        oc = oracle.Cells(cells.offsets, cells.samples, cells.keys,
                          np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)
        t1 = time.perf_counter()
        f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var)
        t2 = time.perf_counter()
        oracle.query(wl.points, oc, f, wl.queries[sel], wl.ell, wl.noise_var, cand_prec=32,
                     sign=wl.sign[sel])
        t3 = time.perf_counter()
        # the VJP refits every cell with dual numbers (its hyperparameter derivative), a
        # fixed cost per call: two sample sizes separate it from the per-point cost
        small = tsel[:64]
        oracle.vjp(wl.points, oc, tq_np[small], wl.ell, wl.noise_var, cand_prec=32,
                   sign=tsg_np[small], mode=1)
        t4 = time.perf_counter()
        oracle.vjp(wl.points, oc, tq_np[tsel], wl.ell, wl.noise_var, cand_prec=32,
                   sign=tsg_np[tsel], mode=1)
        t5 = time.perf_counter()
        per_vjp = max((t5 - t4) - (t4 - t3), 0.0) / (len(tsel) - len(small))
        fixed_vjp = max((t4 - t3) - per_vjp * len(small), 0.0)
        cpu_step = (t2 - t1) + (t3 - t2) / len(sel) * Q + fixed_vjp + per_vjp * QT
        result["cpu_baseline"] = {
            "value": round((Q + QT) / cpu_step, 1), "unit": "queries/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"full FP64 fit of {cells.n} cells ({t2 - t1:.2f} s), {len(sel)} seeded grid "
                      f"queries ({t3 - t2:.2f} s), trajectory VJPs of the softplus cost at "
                      f"{len(small)} and {len(tsel)} points ({t4 - t3:.2f} s, {t5 - t4:.2f} s: "
                      f"dual-number refit {fixed_vjp:.2f} s + {per_vjp * 1e3:.3f} ms/point); "
                      f"step time = fit + grid queries + refit + trajectory points, scaled to "
                      f"{Q} grid and {QT} trajectory points"}
        log(f"cpu oracle: fit {t2 - t1:.2f}s, {len(sel)} queries {t3 - t2:.2f}s, "
            f"vjps {t4 - t3:.2f}s / {t5 - t4:.2f}s, {nthreads} threads")
    model.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
