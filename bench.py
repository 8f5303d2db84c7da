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
points of one step (grid + trajectory) / median step time.  Kernel durations come from
HIP events the library records around each phase's kernels on their launch stream.
The plain per-cell FP64 GPU path is timed on the same inputs as the comparison leg.
Further legs, each timed the same way with its own roofline and plain-path ratio: the
uneven-m batch (room with per-object densities, m on [8, 128], fit + 4,194,304 random
queries as the autotuner picks, the persistent fused launch among the choices) and the
outdoor terrain (256^3 grid + the backward at 16,384 x 64 trajectory points).  The FP64
CPU oracle runs on bounded samples as the CPU baseline, and its outputs give the
parity statistics (max and 99.99th-percentile errors, bound use, FP64-fallback
fraction).  Prints one JSON line.
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
PEAK_FP64_TFLOPS = 78.6       # MI355X FP64 vector peak (published)
PEAK_VALU_TSLOTS = 39.32      # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz lane-instructions/s
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_room_grid.txt")
KERNEL_SOURCES = {
    "query": ["query_fast.hip", "query_split.h", "query_split64_wave.hip",
              "query_split64_lane.hip", "query_split256_wave.hip", "query_split256_lane.hip",
              "query_pairs.hip", "query_dev.h", "fit_dev.h", "ff.h", "ksdf_internal.h"],
    "fused": ["fused.hip", "query_dev.h", "fit_dev.h", "ff.h", "ksdf_internal.h"],
}
ROOM_BOX = (np.zeros(3), np.array([10.0, 8.0, 3.0]))
TERRAIN_BOX = (np.zeros(3), np.array([100.0, 100.0, 25.0]))


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


def backward_flops(m_mean: float, var_f: bool) -> float:
    """One VJP point at its argmin cell, as the launched variant computes it: recompute
    k* and the scaled kernel values (14 m), the mean and gradient adjoints (12 m), the
    softmin variance adjoint (10 m), the hyperparameter terms (4 m); with a var_f
    cotangent also the forward and backward substitution for A^{-1} k* (2 m^2)."""
    m = m_mean
    return 40 * m + (2 * m * m if var_f else 0.0)


def fit_flops(m: np.ndarray) -> float:
    """Per cell: assembly of the lower triangle (5 m^2), Cholesky (m^3 / 3), the two
    triangular solves for a (2 m^2)."""
    m = m.astype(np.float64)
    return float(np.sum(m ** 3 / 3 + 7 * m * m))


def med(xs):
    return float(np.median(xs)) if len(xs) else None


def r4(x):
    return None if x is None else round(float(x), 4)


class Timer:
    """HIP events on the current stream around a callable, per repetition."""

    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, reps):
        torch = self.torch
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return med(ms), ms


COST_MARGIN, COST_KVAR = 0.3, 1.0   # c = sum softplus(0.3 - d + 1.0 sqrt(var))


def softplus_cotangents(torch, out, d_mean, d_var):
    # cost c = sum softplus(0.3 - d + sqrt(var)): dc/dd = -sigmoid(t), dc/dvar = sigmoid(t) / (2 sqrt(var))
    sd = torch.sqrt(torch.clamp_min(out["var"], 1e-30))
    s = torch.sigmoid(0.3 - out["mean"] + sd)
    torch.neg(s, out=d_mean)
    torch.div(s, 2 * sd, out=d_var)


def roofline_query(flop_q, tr_q, Q, kernel_ms, kernel, extra_flop=0.0, traffic=None):
    flops = flop_q * Q + extra_flop
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    slots = (flop_q / 2 + tr_q * 4) * Q + extra_flop / 2
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": None if traffic is None else round(traffic), "kernel": kernel,
            "kernel_ms": round(kernel_ms, 4), "flop_per_launch": round(flops),
            "issue_frac": round(slots / (kernel_ms * 1e-3) / (PEAK_VALU_TSLOTS * 1e12), 4)}


def roofline_backward(m_mean, QT, kernel_ms, var_f, fp64_arith=False):
    """The backward kernel of an FP32 model computes in FP32 (float-float differences and
    kernel exponents, compensated sums): scored at the algorithmic flop count against the
    FP32 vector peak."""
    flops = backward_flops(m_mean, var_f) * QT
    peak = PEAK_FP64_TFLOPS if fp64_arith else PEAK_FP32_TFLOPS
    ach = flops / (kernel_ms * 1e-3) / 1e12
    return {"kernel": "bwd_wave_kernel<%s, *>" % ("true" if var_f else "false"),
            "arith": "f64" if fp64_arith else "f32", "kernel_ms": round(kernel_ms, 4),
            "flop_per_launch": round(flops), "achieved": round(ach, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(ach / peak, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 GPU legs")
    ap.add_argument("--no-matern", action="store_true", help="skip the Matern 3/2 leg")
    ap.add_argument("--no-bhm", action="store_true", help="skip the BHM sign leg")
    ap.add_argument("--no-refit", action="store_true", help="skip the streaming-refit leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-m batch leg")
    ap.add_argument("--no-terrain", action="store_true", help="skip the outdoor terrain leg")
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
    ap.add_argument("--parity-sample", type=int, default=16384)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not built)"}), flush=True)
        sys.exit(2)

    import torch
    from paper_2603_29227_amd import ksdf, scenes, tune

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    timer = Timer(torch)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    wl = scenes.room_workload("grid", grid_n=args.grid)
    tq_np, tsg_np = scenes.room_trajectories(wl)
    log(f"room workload: {len(wl.points)} samples, {len(wl.queries)} grid queries, "
        f"{len(tq_np)} trajectory points ({time.time() - t0:.1f}s)")
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    m = cells.m
    log(f"cells: {cells.n}, m mean {m.mean():.1f}, max {m.max()}")
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision="fp32", query_box=ROOM_BOX, adjoint=True, dense_inverse=True)
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
        softplus_cotangents(torch, tout, d_mean, d_var)

    # launch shapes: the fit+query step, the trajectory query and the backward are tuned
    # (or taken from the cache) separately
    t1 = time.time()
    if args.no_tune:
        tune.apply(model, Q)
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
        # the softplus margin cost's gradient, its cotangents formed inside the backward
        model.set_tuning(**t_traj)
        model.query(tq, tsg, out=tout, workspace=ws)
        model.set_tuning(**t_bwd)
        grads["points"], grads["hyper"] = model.cost_backward(
            tq, tsg, tout["mean"], tout["var"], argmin=tout["argmin"], margin=COST_MARGIN,
            kvar=COST_KVAR, workspace=ws)

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

    # timed region: K whole steps; the library's events time each phase's kernels
    model.set_timing(True)
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
    traj_list, qt, bt = [], [], []
    for _ in range(args.steps):
        ms, _ = timer(traj_part, 1)
        traj_list.append(ms)
        qt += model.timer_read("query")
        bt += model.timer_read("backward")
    traj_ms = med(traj_list)
    if overlap:
        kern["query_traj"], kern["backward"] = qt, bt
    model.set_timing(False)
    step_med = med(step_ms)
    kmed = {k: med(v) for k, v in kern.items() if v}
    n_fp64 = int(((cst.cpu().numpy() & ksdf.C_FP64) != 0).sum())
    st = out["status"].cpu().numpy()
    log(f"step median {step_med:.3f} ms (mean {np.mean(step_ms):.3f}, wall {wall:.3f}; trajectory "
        f"part beside the grid query: {overlap}), grid fit+query {med(fwd_ms):.3f} ms, trajectory "
        f"part alone {traj_ms:.3f} ms, kernels {kmed}, fp64 cells {n_fp64}")
    # the room's GPU outputs of the timed step, for the parity statistics
    room_gpu = {k: v.cpu().numpy() for k, v in out.items()}
    room_traj = dict(dp=grads["points"].cpu().numpy(), am=tout["argmin"].cpu().numpy())

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
        graph, _ = timer(g.replay, args.steps)
        graph = round(graph, 4)
        log(f"graph replay: {graph:.3f} ms/step (median)")
        del g

    # cost of the optional gradient-variance output (App. C), not part of the step: the
    # grid query alone, without and with it
    gv_ms = None
    if not args.no_grad_var:
        model.set_tuning(**{**t_grid, "fused": 0})
        gv_out = model._out(Q, dev, grad_var=True)
        gv_ms = {}
        for name, o in (("query_ms", out), ("query_with_grad_var_ms", gv_out)):
            model.query(q, sg, out=o)
            ms, _ = timer(lambda: model.query(q, sg, out=o), 3)
            gv_ms[name] = round(ms, 4)
        del gv_out
        log(f"grid query without / with grad_var: {gv_ms}")
    model.set_tuning(**t_grid)

    # streaming refit (App. G) on the fitted room model: the grid queries' argmin cells
    # counted into the query counters, a tenth of the cells marked dirty (c2 in 1..3),
    # and the training queue's highest-priority 512 cells refitted (ranking, bucketed
    # FP32 fit with the adjoint vectors, counter reset)
    refit = None
    if not args.no_refit:
        rng = np.random.default_rng(11)
        n_dirty = max(cells.n // 10, 1)
        pick = torch.from_numpy(rng.choice(cells.n, n_dirty, replace=False)).long().to(dev)
        c2 = torch.from_numpy(rng.integers(1, 4, n_dirty).astype(np.float32)).to(dev)
        qcount = torch.zeros(cells.n, dtype=torch.float32, device=dev)
        budget = min(512, cells.n)
        model.count_queries(out["argmin"], qcount)
        torch.cuda.synchronize()
        count_ms, _ = timer(lambda: model.count_queries(out["argmin"], qcount), 3)
        rms = []
        for rep_ in range(4):
            dirty = torch.zeros(cells.n, dtype=torch.float32, device=dev)
            dirty[pick] = c2
            torch.cuda.synchronize()
            ms, _ = timer(lambda: model.refit(pts, dirty, qcount, 0.5, budget), 1)
            if rep_ > 0:
                rms.append(ms)
        refit = {"dirty_cells": n_dirty, "budget": budget, "refit_ms": r4(med(rms)),
                 "cells_per_s": round(budget / (med(rms) * 1e-3), 1),
                 "count_queries_ms": r4(count_ms), "counted_queries": Q}
        log(f"streaming refit: {refit}")

    # the Matern 3/2 variant (Table I) on the same room and grid, its own FP32 model:
    # float-float fit as for the RBF, and the RBF's wave-shared two-kernel query with the
    # Matern cell value, launch shapes of the grid's tuning (no matrix-core variance:
    # the dense inverses are an RBF option)
    matern = None
    if not args.no_matern:
        mat = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell,
                         noise_var=wl.noise_var, precision="fp32", query_box=ROOM_BOX,
                         kernel="matern32")
        mat.set_tuning(**{**t_grid, "fused": 0, "query_mfma": 0, "query_pairs": 0})
        mout = mat._out(Q, dev)
        mat.fit(pts)
        mat.query(q, sg, out=mout)
        torch.cuda.synchronize()
        mat.set_timing(True)
        mf, mq = [], []
        for _ in range(5):
            mat.fit(pts)
            mat.query(q, sg, out=mout)
            torch.cuda.synchronize()
            mf += mat.timer_read("fit")
            mq += mat.timer_read("query")
        mat.set_timing(False)
        mst = mout["status"].cpu().numpy()
        matern = {"fit_ms": r4(med(mf)), "query_ms": r4(med(mq)),
                  "query_qps": round(Q / (med(mq) * 1e-3), 1),
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
            ms, _ = timer(lambda: ksdf.bhm_sign(pts_, *bargs), 3)
            bhm[f"{name}_sign_ms"] = round(ms, 4)
            bhm[f"{name}_sign_qps"] = round(len(pts_) / (ms * 1e-3), 1)
        del bargs
        log(f"bhm sign: {bhm}")

    # roofline of the dominant kernel (algorithmic flops over its measured duration)
    k_fuse = int(model.hyper.k_fuse)
    fq, tr = query_flops(float(m.mean()), k_fuse)
    split = t_grid.get("query_split", 0) == 1
    if fused:
        roofline = roofline_query(fq, tr, Q, kmed["fused"], "fused_kernel (fit + query)",
                                  extra_flop=fit_flops(m), traffic=measured_traffic("fused"))
    else:
        name = ("query phase: query_p1_kernel + query_regroup_kernel + query_p2_kernel" if split
                else "query_fast_kernel")
        roofline = roofline_query(fq, tr, Q, kmed["query"], name, traffic=measured_traffic("query"))
    roof_bwd = roofline_backward(float(m.mean()), QT, kmed["backward"], var_f=False)
    fit_roof = None
    if not fused:
        ff = fit_flops(m)
        fit_roof = {"kernel": "fit32_kernel (all m buckets) + FP64 refits", "kernel_ms": r4(kmed["fit"]),
                    "flop_per_launch": round(ff),
                    "achieved": round(ff / (kmed["fit"] * 1e-3) / 1e12, 3), "peak": PEAK_FP32_TFLOPS,
                    "frac": round(ff / (kmed["fit"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 5)}

    result = {
        "metric": "SDF queries/s (mean+grad+var) + backward queries/s vs plain path, at tolerance",
        "value": round((Q + QT) / (step_med * 1e-3), 1),
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_med, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"indoor room 10x8x3 m, 20 boxes + 10 cylinders, 2 cm sampling, "
                               f"{len(wl.points)} samples, {cells.n} cells (h 0.25 m, m<=64); "
                               f"{args.grid}^3 grid queries + backward of the softplus collision "
                               f"cost at 4096 x 64 trajectory points", "grid_queries": Q,
                   "trajectory_points": QT, "k_fuse": k_fuse, "ell": wl.ell,
                   "noise_var": wl.noise_var, "tuning": tuned,
                   "streams": 2 if overlap else 1, "ms_per_step_is": "median of the timed steps"},
        "step_ms_all": [round(x, 4) for x in step_ms],
        "fwd_qps": round(Q / (med(fwd_ms) * 1e-3), 1),
        "bwd_qps": round(QT / (traj_ms * 1e-3), 1),
        "trajectory_part_ms": r4(traj_ms),
        "kernel_ms": {k: r4(v) for k, v in kmed.items()},
        "graph_ms_per_step": graph,
        "fp64_cells": n_fp64, "fp64_fraction": round(n_fp64 / max(cells.n, 1), 6),
        "no_valid_queries": int(((st & 1) != 0).sum()),
        "model_device_bytes": info["device_bytes"],
        "roofline": roofline, "roofline_backward": roof_bwd, "roofline_fit": fit_roof,
        "grad_var_cost": gv_ms,
        "matern32": matern,
        "bhm_sign": bhm,
        "streaming_refit": refit,
    }

    if not args.no_plain:
        # the plain per-cell FP64 GPU path: one thread per query, every candidate cell in
        # FP64, the plain backward; same inputs; medians of 3 runs
        plain = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell,
                           noise_var=wl.noise_var, precision="fp64", query_box=ROOM_BOX, adjoint=True)
        p64, q64, tq64 = pts.double(), q.double(), tq.double()
        pout = plain._out(Q, dev)
        ptout = plain._out(QT, dev, status=False)
        softplus_cotangents(torch, tout, d_mean, d_var)   # the plain path takes them as inputs
        dm64, dv64 = d_mean.double(), d_var.double()

        def plain_grid():
            plain.fit(p64)
            plain.query(q64, sg, out=pout)

        def plain_traj():
            plain.query(tq64, tsg, out=ptout)
            plain.backward(tq64, tsg, dm64, None, dv64, None, argmin=ptout["argmin"])

        plain_grid()
        plain_traj()
        torch.cuda.synchronize()
        pf, _ = timer(plain_grid, 3)
        pb, _ = timer(plain_traj, 3)
        result["plain_fp64"] = {"fit_query_ms": round(pf, 3), "traj_query_backward_ms": round(pb, 3),
                                "step_ms": round(pf + pb, 3),
                                "value": round((Q + QT) / ((pf + pb) * 1e-3), 1),
                                "speedup_step": round((pf + pb) / step_med, 2),
                                "speedup_grid_fit_query": round(pf / med(fwd_ms), 2),
                                "speedup_trajectory_query_backward": round(pb / traj_ms, 2),
                                "runs": "medians of 3"}
        log(f"plain fp64: grid fit+query {pf:.3f} ms, trajectory query+backward {pb:.3f} ms")
        plain.close()
        del p64, q64, tq64, pout, ptout

    model.close()
    del pts, q, sg, out, tout, traj_ws

    batch = None if args.no_batch else leg_batch(args, torch, dev, ksdf, scenes, tune, timer)
    terrain = None if args.no_terrain else leg_terrain(args, torch, dev, ksdf, scenes, tune, timer)
    result["batch_uneven_m"] = batch and batch["report"]
    result["terrain"] = terrain and terrain["report"]

    if not args.no_cpu:
        cpu_leg(args, result, wl, cells, room_gpu, room_traj, tq_np, tsg_np, batch, terrain)
    print(json.dumps(result), flush=True)


def leg_batch(args, torch, dev, ksdf, scenes, tune, timer):
    """Uneven-m batch: the room with per-object densities x logU[0.1, 4] and per-cell caps
    logU[8, 128], fit + 4,194,304 random queries in the launch shape the autotuner picks
    (the persistent fused fit+query launch among the choices)."""
    t0 = time.time()
    wl = scenes.room_workload("batch")
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    m = cells.m
    log(f"batch: {len(wl.points)} samples, {cells.n} cells, m {m.min()}..{m.max()} mean {m.mean():.1f} "
        f"({time.time() - t0:.1f}s)")
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision="fp32", query_box=ROOM_BOX, dense_inverse=True)
    pts = torch.from_numpy(wl.points).to(dev)
    q = torch.from_numpy(wl.queries).to(dev)
    sg = torch.from_numpy(wl.sign).to(dev)
    Q = len(q)
    if args.no_tune:
        tune.apply(model, Q)
        source = "cache"
    else:
        res = tune.tune(model, pts, q, sg, reps=2, cache_path=args.tune_cache)
        log(f"batch autotuner: {res['tuning']} {res['ms']:.3f} ms ({len(res['table'])} candidates)")
        source = "timed"
    t = model.tuning()
    out = model._out(Q, dev)
    cst = torch.zeros(cells.n, dtype=torch.uint8, device=dev)
    for _ in range(2):
        model.fit_query(pts, q, sg, cell_status=cst, out=out)
    torch.cuda.synchronize()
    model.set_timing(True)
    step_ms, kf, kq, ku = [], [], [], []
    for _ in range(args.steps):
        ms, _ = timer(lambda: model.fit_query(pts, q, sg, cell_status=cst, out=out), 1)
        step_ms.append(ms)
        if t["fused"]:
            ku += model.timer_read("fused")
        else:
            kf += model.timer_read("fit")
            kq += model.timer_read("query")
    model.set_timing(False)
    model.check()
    step = med(step_ms)
    fq, tr = query_flops(float(m.mean()), int(model.hyper.k_fuse))
    if t["fused"]:
        roof = roofline_query(fq, tr, Q, med(ku), "fused_kernel (fit + query)", extra_flop=fit_flops(m))
    else:
        roof = roofline_query(fq, tr, Q, med(kq),
                              "query phase (two kernels)" if t["query_split"] else "query_fast_kernel")
    n_fp64 = int(((cst.cpu().numpy() & ksdf.C_FP64) != 0).sum())
    rep = {"workload": f"room, per-object density x logU[0.1,4], per-cell m cap logU[8,128]: "
                       f"{len(wl.points)} samples, {cells.n} cells, m {int(m.min())}..{int(m.max())} "
                       f"(mean {m.mean():.1f}); fit + {Q} random queries",
           "tuning": {**t, "source": source}, "step_ms": r4(step),
           "qps_fit_query": round(Q / (step * 1e-3), 1),
           "kernel_ms": {"fused": r4(med(ku)), "fit": r4(med(kf)), "query": r4(med(kq))},
           "roofline": roof, "fp64_cells": n_fp64, "fp64_fraction": round(n_fp64 / cells.n, 6),
           "no_valid_queries": int(((out["status"].cpu().numpy() & 1) != 0).sum())}
    if not args.no_plain:
        plain = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                           precision="fp64", query_box=ROOM_BOX)
        p64, q64 = pts.double(), q.double()
        pout = plain._out(Q, dev)
        plain.fit_query(p64, q64, sg, out=pout)
        torch.cuda.synchronize()
        pms, _ = timer(lambda: plain.fit_query(p64, q64, sg, out=pout), 3)
        rep["plain_fp64"] = {"fit_query_ms": round(pms, 3), "speedup": round(pms / step, 2),
                             "runs": "medians of 3"}
        plain.close()
        del p64, q64, pout
    log(f"batch: {rep}")
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    model.close()
    return {"report": rep, "wl": wl, "cells": cells, "gpu": gpu}


def leg_terrain(args, torch, dev, ksdf, scenes, tune, timer):
    """Large outdoor terrain (value-noise heightfield, 500 boxes and cylinders, 3 cm
    sampling, 0.5 m cells, uneven m): fit + 256^3 grid query, then the softplus-cost
    backward at 16,384 x 64 trajectory points (1,048,576)."""
    t0 = time.time()
    wl = scenes.terrain_workload(grid_n=args.grid)
    tq_np, tsg_np = scenes.terrain_trajectories(wl)
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                             wl.m_cap_grid, wl.key_lo)
    m = cells.m
    log(f"terrain: {len(wl.points)} samples, {cells.n} cells, m {m.min()}..{m.max()} mean "
        f"{m.mean():.1f}, {len(tq_np)} trajectory points ({time.time() - t0:.1f}s)")
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                       precision="fp32", query_box=TERRAIN_BOX, adjoint=True, dense_inverse=True)
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
    cst = torch.zeros(cells.n, dtype=torch.uint8, device=dev)
    model.set_tuning(fused=0)
    model.fit(pts, cell_status=cst)
    if args.no_tune:
        tg = {**(tune.cached(model, Q, "query") or {}), "fused": 0}
        tqt = tune.cached(model, QT, "query") or {}
        tbt = tune.cached(model, QT, "backward") or {}
    else:
        tg = {**tune.tune_query(model, q, sg, reps=2, cache_path=args.tune_cache)["tuning"], "fused": 0}
        tqt = tune.tune_query(model, tq, tsg, reps=2, cache_path=args.tune_cache)["tuning"]
        model.query(tq, tsg, out=tout)
        softplus_cotangents(torch, tout, d_mean, d_var)
        tbt = tune.tune_backward(model, tq, tsg, dict(d_mean=d_mean, d_var=d_var), tout["argmin"],
                                 reps=2, cache_path=args.tune_cache)["tuning"]

    def grid():
        model.set_tuning(**tg)
        model.fit(pts, cell_status=cst)
        model.query(q, sg, out=out)

    def traj():
        model.set_tuning(**{**tg, **tqt})
        model.query(tq, tsg, out=tout)
        model.set_tuning(**{**tg, **tqt, **tbt})
        return model.cost_backward(tq, tsg, tout["mean"], tout["var"], argmin=tout["argmin"],
                                   margin=COST_MARGIN, kvar=COST_KVAR)

    grid()
    traj()
    torch.cuda.synchronize()
    model.set_timing(True)
    g_ms, t_ms, kf, kq, kqt, kb = [], [], [], [], [], []
    for _ in range(max(3, args.steps // 2)):
        ms, _ = timer(grid, 1)
        g_ms.append(ms)
        kf += model.timer_read("fit")
        kq += model.timer_read("query")
        ms, _ = timer(traj, 1)
        t_ms.append(ms)
        kqt += model.timer_read("query")
        kb += model.timer_read("backward")
    model.set_timing(False)
    torch.cuda.synchronize()
    gm, tm = med(g_ms), med(t_ms)
    fq, tr = query_flops(float(m.mean()), int(model.hyper.k_fuse))
    ff = fit_flops(m)
    n_fp64 = int(((cst.cpu().numpy() & ksdf.C_FP64) != 0).sum())
    rep = {"workload": f"terrain 100x100x20 m, 250 boxes + 250 cylinders, 3 cm sampling: "
                       f"{len(wl.points)} samples, {cells.n} cells (h 0.5 m, m {int(m.min())}.."
                       f"{int(m.max())}, mean {m.mean():.1f}); {args.grid}^3 grid + backward at "
                       f"{QT} trajectory points",
           "tuning": {"grid": tg, "trajectory": tqt, "backward": tbt},
           "grid_fit_query_ms": r4(gm), "grid_qps": round(Q / (gm * 1e-3), 1),
           "trajectory_query_backward_ms": r4(tm), "bwd_qps": round(QT / (tm * 1e-3), 1),
           "value": round((Q + QT) / ((gm + tm) * 1e-3), 1),
           "kernel_ms": {"fit": r4(med(kf)), "query": r4(med(kq)), "query_traj": r4(med(kqt)),
                         "backward": r4(med(kb))},
           "roofline": roofline_query(fq, tr, Q, med(kq), "query phase (grid)"),
           "roofline_fit": {"kernel_ms": r4(med(kf)), "flop_per_launch": round(ff),
                            "achieved": round(ff / (med(kf) * 1e-3) / 1e12, 3),
                            "frac": round(ff / (med(kf) * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 5)},
           "roofline_backward": roofline_backward(float(m.mean()), QT, med(kb), var_f=False),
           "fp64_cells": n_fp64, "fp64_fraction": round(n_fp64 / cells.n, 6),
           "no_valid_queries": int(((out["status"].cpu().numpy() & 1) != 0).sum())}
    if not args.no_plain:
        plain = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var,
                           precision="fp64", query_box=TERRAIN_BOX, adjoint=True)
        p64, q64, tq64 = pts.double(), q.double(), tq.double()
        pout = plain._out(Q, dev)
        ptout = plain._out(QT, dev, status=False)
        softplus_cotangents(torch, tout, d_mean, d_var)   # the plain path takes them as inputs
        dm64, dv64 = d_mean.double(), d_var.double()

        def pgrid():
            plain.fit(p64)
            plain.query(q64, sg, out=pout)

        def ptraj():
            plain.query(tq64, tsg, out=ptout)
            plain.backward(tq64, tsg, dm64, None, dv64, None, argmin=ptout["argmin"])

        pgrid()
        ptraj()
        torch.cuda.synchronize()
        pg, _ = timer(pgrid, 3)
        pt, _ = timer(ptraj, 3)
        rep["plain_fp64"] = {"grid_fit_query_ms": round(pg, 3), "trajectory_query_backward_ms": round(pt, 3),
                             "speedup_grid": round(pg / gm, 2), "speedup_trajectory": round(pt / tm, 2),
                             "speedup_total": round((pg + pt) / (gm + tm), 2), "runs": "medians of 3"}
        plain.close()
        del p64, q64, tq64, pout, ptout
    log(f"terrain: {rep}")
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    model.close()
    return {"report": rep, "wl": wl, "cells": cells, "gpu": gpu}


def cpu_leg(args, result, wl, cells, room_gpu, room_traj, tq_np, tsg_np, batch, terrain):
    """The FP64 CPU oracle: timed on a bounded sample of the room step (the CPU
    baseline), and its outputs on seeded samples compared with the GPU's (the parity
    statistics of this run)."""
    import oracle
    from tests import parity
    Q, QT = len(wl.queries), len(tq_np)
    nthreads = oracle.threads()
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(Q, size=min(args.cpu_queries, Q), replace=False))
    tsel = np.sort(rng.choice(QT, size=min(args.cpu_vjp, QT), replace=False))
    oc = oracle.Cells(cells.offsets, cells.samples, cells.keys,
                      np.asarray(wl.origin) + (cells.keys + 0.5) * wl.h)
    t1 = time.perf_counter()
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var)
    t2 = time.perf_counter()
    oracle.query(wl.points, oc, f, wl.queries[sel], wl.ell, wl.noise_var, sign=wl.sign[sel])
    t3 = time.perf_counter()
    # the VJP refits every cell with dual numbers (its hyperparameter derivative), a
    # fixed cost per call: two sample sizes separate it from the per-point cost
    small = tsel[:64]
    oracle.vjp(wl.points, oc, tq_np[small], wl.ell, wl.noise_var, sign=tsg_np[small], mode=1)
    t4 = time.perf_counter()
    oracle.vjp(wl.points, oc, tq_np[tsel], wl.ell, wl.noise_var, sign=tsg_np[tsel], mode=1)
    t5 = time.perf_counter()
    per_vjp = max((t5 - t4) - (t4 - t3), 0.0) / (len(tsel) - len(small))
    fixed_vjp = max((t4 - t3) - per_vjp * len(small), 0.0)
    cpu_step = (t2 - t1) + (t3 - t2) / len(sel) * Q + fixed_vjp + per_vjp * QT
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    result["cpu_baseline"] = {
        "value": round((Q + QT) / cpu_step, 1), "unit": "queries/s", "cores": nthreads,
        "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model,
        "sample": f"full FP64 fit of {cells.n} cells ({t2 - t1:.2f} s), {len(sel)} seeded grid "
                  f"queries ({t3 - t2:.2f} s), trajectory VJPs of the softplus cost at "
                  f"{len(small)} and {len(tsel)} points ({t4 - t3:.2f} s, {t5 - t4:.2f} s: "
                  f"dual-number refit {fixed_vjp:.2f} s + {per_vjp * 1e3:.3f} ms/point); "
                  f"step time = fit + grid queries + refit + trajectory points, scaled to "
                  f"{Q} grid and {QT} trajectory points; {nthreads} OpenMP threads"}
    log(f"cpu oracle: fit {t2 - t1:.2f}s, {len(sel)} queries {t3 - t2:.2f}s, "
        f"vjps {t4 - t3:.2f}s / {t5 - t4:.2f}s, {nthreads} threads")

    def sample(mean, n, seed):
        rng_ = np.random.default_rng(seed)
        uni = rng_.choice(len(mean), size=min(3 * n // 4, len(mean)), replace=False)
        near = np.where(np.abs(mean) < 0.05)[0]
        near = rng_.choice(near, size=min(n // 4, len(near)), replace=False) if len(near) else near
        return np.unique(np.concatenate([uni, near]))

    def fwd_stats(w, ocells, fit_, gpu, n, seed):
        idx = sample(gpu["mean"], n, seed)
        o = oracle.query(w.points, ocells, fit_, w.queries[idx], w.ell, w.noise_var,
                         sign=w.sign[idx], all_candidates=True)
        rep = parity.compare({k: v[idx] for k, v in gpu.items()}, o, w.ell, "fp32")
        keep = ("n", "near_tie", "cand_tie", "grad_unconstrained", "grad_err_over_bound_max",
                "mean_err_max", "mean_err_p9999", "grad_err_max", "grad_err_p9999",
                "var_relerr_max", "var_relerr_p9999", "var_f_err_max", "var_f_err_p9999")
        s = {k: rep[k] for k in keep if k in rep}
        s["failures"] = rep["failures"]
        return s

    par = {"room_grid": fwd_stats(wl, oc, f, room_gpu, args.parity_sample, 20)}
    # the step's backward at the first 1,024 trajectory points (a point's VJP does not
    # depend on the batch it is in; d_hyper sums the whole set and is left to the tests)
    n = 1024
    vr = parity.vjp_report(room_traj["dp"][:n], None, room_traj["am"][:n], wl, oc, tq_np[:n],
                           tsg_np[:n], "fp32", mode=1)
    vr.pop("_worst", None)
    par["room_trajectory_vjp"] = vr
    if batch is not None:
        w, c = batch["wl"], batch["cells"]
        ocb = oracle.Cells(c.offsets, c.samples, c.keys, np.asarray(w.origin) + (c.keys + 0.5) * w.h)
        fb = oracle.fit(w.points, ocb, w.ell, w.noise_var)
        par["batch_uneven_m"] = fwd_stats(w, ocb, fb, batch["gpu"], args.parity_sample // 2, 21)
    if terrain is not None:
        w, c = terrain["wl"], terrain["cells"]
        oct_ = oracle.Cells(c.offsets, c.samples, c.keys, np.asarray(w.origin) + (c.keys + 0.5) * w.h)
        ft = oracle.fit(w.points, oct_, w.ell, w.noise_var)
        par["terrain_grid"] = fwd_stats(w, oct_, ft, terrain["gpu"], args.parity_sample // 2, 22)
    par["fp64_fallback_fraction"] = {"room": result.get("fp64_fraction"),
                                     "batch_uneven_m": batch and batch["report"]["fp64_fraction"],
                                     "terrain": terrain and terrain["report"]["fp64_fraction"]}
    par["contract"] = ("tests/parity.py: mean 1e-4 relative (floor 1 m, square-root zone), "
                       "grad within max(1e-4, ratio (3e-7 + 3e-7 |u|)), var 1e-3 relative, "
                       "var_f 1e-3 absolute, VJP per point within max(1e-3, 2 cond_2 2^-24); "
                       "argmin cells accepted by readings R6 and R7")
    result["parity"] = par
    log(f"parity: {par}")


if __name__ == "__main__":
    main()
