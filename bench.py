#!/usr/bin/env python3
"""Training-iteration benchmark of the differentiable Gaussian rasterizer.

One step = forward render of every view of the batch, L1 loss against the
target images (fused into the compositing epilogue), backward to all
Gaussian parameters and a dense Adam update (fused into the per-Gaussian
backward), all in the HIP library, replayed as
one captured HIP graph.  Default workload: the 6-camera 1600x900 ring rig in
a street corridor with 1M Gaussians (SH degree 3).

Prints one JSON line (rank 0).  Besides the throughput it reports:
  roofline      achieved vs peak of the dominant kernel, its duration taken
                from HIP events recorded around it on the library's stream
                during an eager pass of the same steps
  cpu_baseline  the FP64 CPU oracle timed on a bounded pixel sample, one
                single-threaded worker process per host core (at most 15)
  step_ms_spread  p10 / median / p90 of 30 single replays (HIP events)
  hbm_copy_gbs  achievable HBM bandwidth (the library's streaming copy of
                1 GiB), and the step's algorithmic bytes as a fraction of it
  per_view      batched against plain per-view launches, both arranged the
                same way (forward with the fused loss, backward to dense
                gradients, one Adam step) and graph-captured (per-view also
                eager)
  window        the same comparison, and the fused step, on the 40-view
                uneven keyframe window (2M Gaussians)
  pose          the same step with each view's camera-pose gradient and its
                rig chain (central pose per frame, relative transform per
                camera) added, as a second captured graph
  freq          the frequency-based scheduling pass on the step's renders:
                X of every view (batched 2D FFT) and one scheduling step,
                timed with HIP events, with its bytes against HBM peak
  insert        the LoG-based insertion step over all views (seeded
                structured ground truth, render and depth of the views'
                sizes), timed with HIP events, bytes against HBM peak
  merge         the per-camera merge of the scene's Gaussians with view 0's
                samples from that insertion, timed with HIP events
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd iterations/s and Mpix/s, 6-cam 1600x900 rig, 1M Gaussians; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# Non-packed FP32 VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Lane operations of one (pixel, Gaussian) evaluation, counted from the
# formulas (each add, mul, fma, min, compare, exp2 and rcp is one op; loads,
# control flow and the per-record wave reductions are not counted):
#   forward : box test 4, offsets 4, u 1, q 4, exp2 1, opacity and cap 2,
#             alpha test 1, T update 2, stop test 1, weight 1, colour 3  = 24
#   backward: the above up to alpha (box 4 + in-front test 1, 13), rcp and
#             T recovery 3, weight 1, colour grads 3, suffix differences 3,
#             dL/dalpha 4, suffix update 3, cap test 1, opacity grad 1,
#             dq 1, conic grads 5, offset grads 5                        = 48
FWD_OPS_PER_EVAL = 24
BWD_OPS_PER_EVAL = 48


def stage_work(stage, n, n_u, pg, views, px, rec, pairs, tiles, evals):
    """(algorithmic HBM bytes, algorithmic lane ops) of one stage: every array
    the method needs read or written once (ideal one-pass sort, Adam state
    read and written once), and the compositing evaluations."""
    if stage == "preprocess":   # params in (visible ones whole), records out; visibility scan
        return 12 * n + 4 * (pg - 3) * n_u + 4 * views * n + 48 * rec + 8 * views * n, 0
    if stage == "binning":      # records in, (key, value) pairs out; tile ranges
        return 24 * rec + 12 * pairs + 8 * pairs + 8 * tiles, 0
    if stage == "sort":         # (key, value) pairs in and out
        return 24 * pairs, 0
    if stage == "raster_fwd":   # lists + records in; image, T, last, count out; the fused L1 loss:
        return 40 * pairs + 20 * px + 24 * px, FWD_OPS_PER_EVAL * evals  # target in, gradient out
    if stage == "loss":         # the final sum of the fused loss's per-workgroup partials
        return 4 * tiles, 0
    if stage == "raster_bwd":   # lists, records, dL/dC, T, last in
        return 40 * pairs + 20 * px, BWD_OPS_PER_EVAL * evals
    if stage == "reduce":       # per-record 2D gradients out and back in
        return 72 * rec, 0
    if stage == "pre_bwd":      # 2D grads in; Adam fused: each parameter read once, its moments
        return 36 * rec + 24 * pg * n + 4 * n, 0  # read, all three written (no gradient array)
    return 0, 0


STEP_STAGES = ("preprocess", "binning", "sort", "raster_fwd", "loss", "raster_bwd", "reduce", "pre_bwd")
STAGE_KERNEL = {"raster_bwd": "k_raster_bwd16", "raster_fwd": "k_raster_fwd16", "preprocess": "k_pre_write<3>",
                "pre_bwd": "k_pre_bwd<3,true>"}


def source_hash(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# HBM traffic of a kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# recorded under profiles/ with the hash of the kernel's sources; reported
# only while the sources are unchanged.
TRAFFIC_SOURCES = {"k_raster_bwd16": ["paper_2512_08498_amd/csrc/raster_bwd.hip", "paper_2512_08498_amd/csrc/raster.hpp",
                                      "paper_2512_08498_amd/csrc/util.hpp", "paper_2512_08498_amd/csrc/common.hpp"]}


def recorded_traffic(kernel, workload):
    import re

    srcs = TRAFFIC_SOURCES.get(kernel)
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not srcs or not os.path.exists(path):
        return None
    text = open(path).read()
    m_h = re.search(r"source hash: `([0-9a-f]+)`", text)
    m_b = re.search(r"HBM bytes per launch: ([0-9.e+]+)", text)
    if not m_h or not m_b or m_h.group(1) != source_hash(srcs):
        return None
    return float(m_b.group(1))


# --- CPU baseline: the oracle on pixel windows, one single-threaded worker
# process per host core of the GPU's share (at most 15 besides this one) -----
_ORACLE_STATE = {}


def _oracle_worker_init():
    """Each worker runs single-threaded (NumPy's and torch's pools at one
    thread), so the process count is the core count."""
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except ImportError:
        pass


def _oracle_windows(task):
    """Worker: forward + FP64 autograd backward of the oracle on random
    win x win windows of the workload for budget_s seconds (scene generation
    not timed).  Returns (pixels, windows, seconds)."""
    config, scale, worker, budget_s, win, seed = task
    import torch

    torch.set_num_threads(1)
    from oracle.grad64 import grad64
    from oracle.project64 import to_params64
    from oracle.render64 import render_view
    from workloads import make_config, make_target

    key = (config, scale)
    if key not in _ORACLE_STATE:
        scene, cams = make_config(config, scale)
        targets = make_target(config, cams)
        _ORACLE_STATE[key] = (scene, cams, targets, to_params64(scene.arrays()),
                              sum(c.width * c.height for c in cams))
    scene, cams, targets, p64, total_px = _ORACLE_STATE[key]
    arrays = scene.arrays()
    rng = np.random.default_rng(seed + 7919 * worker)
    done_px = n_win = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        v = (worker + n_win) % len(cams)
        c = cams[v]
        x0 = int(rng.integers(0, c.width - win + 1))
        y0 = int(rng.integers(0, c.height - win + 1))
        w = (x0, x0 + win, y0, y0 + win)
        fwd = render_view(arrays, scene.sh_degree, c, window=w, p64=p64)
        cot = np.zeros((3, c.height, c.width))
        cot[:, y0:y0 + win, x0:x0 + win] = np.sign(fwd["image"] - targets[v][:, y0:y0 + win, x0:x0 + win]) / (
            3.0 * total_px)
        grad64(scene, [c], [cot], windows=[w])
        done_px += win * win
        n_win += 1
    return done_px, n_win, time.perf_counter() - t0


def oracle_workers():
    """Worker count: the host cores this process may use, at most 15, so
    that with this process the run stays within one GPU's share of the host
    (16 processes, which the GPU hosts enforce per process tree)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(15, avail))


def start_oracle_pool(n):
    """The worker pool, forked before this process touches the GPU."""
    import multiprocessing as mp

    return mp.get_context("fork").Pool(n, initializer=_oracle_worker_init)


def cpu_baseline(pool, n_workers, config, scale, total_px, budget_s=15.0, win=32, seed=3003):
    """The oracle timed on all workers at once: each renders and
    differentiates random windows for budget_s seconds; the rate is the
    pixels done over the wall time of the slowest worker, scaled to one full
    iteration of total_px pixels."""
    res = pool.map(_oracle_windows, [(config, scale, w, budget_s, win, seed) for w in range(n_workers)])
    px = sum(r[0] for r in res)
    n_win = sum(r[1] for r in res)
    wall = max(r[2] for r in res)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    mpix = px / wall / 1e6
    return {"value": mpix * 1e6 / total_px, "unit": "it/s", "mpix_per_s": mpix, "cores": n_workers,
            "kind": "oracle", "host_cpus": os.cpu_count(), "cpu_model": model, "extrapolated": True,
            "sample": f"{n_win} windows of {win}x{win} px across the views (FP64 forward + autograd backward), "
                      f"{n_workers} single-threaded worker processes for {wall:.1f} s; rate extrapolated "
                      f"linearly to one full iteration of {total_px} px"}


def batching_comparison(scene, cams, target, params, rast, dev, steps, warmup, replayable, timed, ms_fused):
    """Batched launch against plain per-view launches with the same loss and
    optimiser arrangement: each view's forward with the fused L1 loss, its
    dL/dC rescaled from the view's mean to the batch mean (one torch
    multiply), its backward accumulated into dense gradients, then one Adam
    step; and the batched step arranged the same way (forward with the
    loss, backward to gradients, Adam).  Both are timed as captured graphs;
    the per-view step also eagerly."""
    import torch

    from paper_2512_08498_amd import FusedAdam, Rasterizer

    tun = rast.tuning()
    grads = {k: torch.zeros_like(v) for k, v in params.items()}
    opt2 = FusedAdam(rast, params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    out = rast.new_fwd_out()
    dl = torch.empty_like(out["image"])

    def step_b():
        rast.forward_l1(params, target, out=out, loss_out=loss, dl_out=dl, check=False)
        rast.backward(params, out, dl, grads=grads)
        opt2.apply(grads)

    run_b = replayable(step_b, [rast])
    b_ms = timed(run_b, steps) / steps * 1e3

    rs = []
    for c in cams:
        r = Rasterizer([c], scene.n, scene.sh_degree, tile_size=tun["tile_size"], long_list=tun["long_list"],
                       persistent=tun["persistent"], device=dev, capacity_records=max(scene.n // 4, 65536), capacity_pairs=max(scene.n, 262144))
        r.forward(params)
        rr, pp, _ = r.required_capacity()
        r._plan(int(rr * 1.5) + 4096, int(pp * 1.5) + 65536)
        rs.append(r)
    outs = [r.new_fwd_out() for r in rs]
    tv = [target[3 * rast.pix_off[v]:3 * rast.pix_off[v + 1]] for v in range(len(cams))]
    dls = [torch.empty_like(o["image"]) for o in outs]
    frac = [(rast.pix_off[v + 1] - rast.pix_off[v]) / rast.total_px for v in range(len(cams))]

    def step_pv():
        for v, r in enumerate(rs):
            r.forward_l1(params, tv[v], out=outs[v], loss_out=loss, dl_out=dls[v], check=False)
            dls[v].mul_(frac[v])
            r.backward(params, outs[v], dls[v], grads=grads, accumulate=v > 0)
        opt2.apply(grads)

    n_pv = max(5, steps // 4)
    pv_eager_ms = timed(step_pv, n_pv) / n_pv * 1e3
    for r in rs:
        r.check()
    run_pv = replayable(step_pv, rs)
    pv_ms = timed(run_pv, n_pv) / n_pv * 1e3
    for r in rs:
        r.check()
    del rs, outs, dls
    return {"batched_it_s": 1e3 / b_ms, "batched_ms": b_ms, "per_view_it_s": 1e3 / pv_ms, "per_view_ms": pv_ms,
            "per_view_eager_it_s": 1e3 / pv_eager_ms, "per_view_eager_ms": pv_eager_ms,
            "speedup_batching": pv_ms / b_ms, "speedup_headline_step": pv_ms / ms_fused,
            "arrangement": "forward with fused L1, backward to dense gradients, one Adam step; per-view dL/dC "
                           "rescaled to the batch mean; both legs graph-captured (per-view also eager)",
            "tuning": tun}


def window_leg(args, dev, replayable, timed):
    """The uneven keyframe window (8 rig frames x 5 cameras at mixed
    resolutions, 2M Gaussians): the fused training step, autotuned and
    graph-captured, and the batched vs per-view comparison on it."""
    import torch

    from paper_2512_08498_amd import FusedAdam, Rasterizer
    from workloads import config_names, make_config, make_target

    t0 = time.perf_counter()
    scene, cams = make_config(4, args.scale)
    targets = make_target(4, cams)
    params = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.arrays().items()}
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in targets])).to(dev)
    del targets
    r = Rasterizer(cams, scene.n, scene.sh_degree, device=dev, capacity_records=len(cams) * scene.n // 4,
                   capacity_pairs=len(cams) * scene.n)
    r.forward(params)
    rec, pairs, _ = r.required_capacity()
    r._plan(int(rec * 1.5) + 4096, int(pairs * 1.5) + 65536)
    tuning = r.autotune(params, repeats=5)
    r.forward(params)
    rec, pairs, _ = r.required_capacity()
    r._plan(int(rec * 1.5) + 4096, int(pairs * 1.5) + 65536)
    log(f"window: {scene.n} Gaussians, {len(cams)} views, {r.total_px} px, tuning {tuning} "
        f"({time.perf_counter() - t0:.1f} s set-up)")
    opt = FusedAdam(r, params)
    out = r.new_fwd_out()
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    dl = torch.empty_like(out["image"])

    def step():
        r.forward_l1(params, target, out=out, loss_out=loss, dl_out=dl, check=False)
        r.backward_adam(params, out, dl, opt)

    run = replayable(step, [r])
    ms = timed(run, args.steps) / args.steps * 1e3
    r.check()
    cmp = batching_comparison(scene, cams, target, params, r, dev, args.steps, args.warmup, replayable, timed, ms)
    res = {"workload": config_names()[4], "views": len(cams), "gaussians": scene.n, "pixels": r.total_px,
           "it_s": 1e3 / ms, "ms_per_step": ms, "mpix_per_s": r.total_px / ms / 1e3, **cmp}
    log(f"window: {res['it_s']:.2f} it/s fused; batched (same arrangement) {cmp['batched_it_s']:.2f} it/s, "
        f"per-view {cmp['per_view_it_s']:.2f} it/s graph ({cmp['per_view_eager_it_s']:.2f} eager): batching "
        f"{cmp['speedup_batching']:.2f}x")
    del r, opt, out, dl, params, target
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--tile-size", type=int, default=0, help="8, 16 or 32; 0 (default) = autotune on the workload")
    ap.add_argument("--persistent", type=int, default=0, choices=(0, 1),
                    help="with --tile-size: 1 = persistent compositing launches (the autotuner chooses otherwise)")
    ap.add_argument("--long-list", type=int, default=1024,
                    help="with --tile-size 16: lists this long are walked by a whole workgroup (the autotuner "
                         "chooses otherwise)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-window", action="store_true",
                    help="skip the batched vs per-view comparison on the 40-view uneven keyframe window")
    ap.add_argument("--no-pose", action="store_true")
    ap.add_argument("--no-freq", action="store_true")
    ap.add_argument("--no-insert", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer three times (the reference kernel for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the rasterizer path is built and timed on a single GPU (sharding "
              "by view across GPUs is a design note, not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the oracle's worker processes are forked now, before this process
    # touches the GPU; they stay idle until the GPU timing is done
    pool, n_workers = None, 0
    if not args.no_cpu_baseline and not args.copy_calibration:
        n_workers = oracle_workers()
        pool = start_oracle_pool(n_workers)

    import torch

    from paper_2512_08498_amd import FusedAdam, Frequency, Rasterizer, device_copy
    from workloads import RIG_LAYOUT, config_names, make_config, make_insert_inputs, make_target

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n_el = args.copy_calibration * 2**20 // 4
        src = torch.ones(n_el, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize(dev)
        print(json.dumps({"copy_bytes": n_el * 4, "repeats": 3}), flush=True)
        return
    t_setup = time.perf_counter()
    scene, cams = make_config(args.config, args.scale)
    targets = make_target(args.config, cams)
    log(f"workload {config_names()[args.config]}: {scene.n} Gaussians, {len(cams)} views "
        f"({time.perf_counter() - t_setup:.1f} s to generate)")
    params = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.arrays().items()}
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in targets])).to(dev)

    cap_rec = max(len(cams) * scene.n // 4, 65536)
    rast = Rasterizer(cams, scene.n, scene.sh_degree, tile_size=args.tile_size or 16, device=dev,
                      capacity_records=cap_rec, capacity_pairs=4 * cap_rec, persistent=bool(args.persistent),
                      long_list=args.long_list)
    out = rast.forward(params)  # re-plans on capacity overflow
    rec, pairs, tiles = rast.required_capacity()
    # headroom for the scene to move during training
    rast._plan(int(rec * 1.5) + 4096, int(pairs * 1.5) + 65536)
    tuning = None
    if args.tile_size == 0:
        t_tune = time.perf_counter()
        tuning = rast.autotune(params, repeats=5)
        out = rast.forward(params)
        rec, pairs, tiles = rast.required_capacity()
        rast._plan(int(rec * 1.5) + 4096, int(pairs * 1.5) + 65536)
        log(f"autotuned in {time.perf_counter() - t_tune:.1f} s: {tuning}")
    out = rast.new_fwd_out()
    log(f"records {rec}, pairs {pairs}, tiles {tiles}, workspace {rast.ws_bytes / 2**30:.2f} GiB")
    opt = FusedAdam(rast, params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    dl = torch.empty_like(out["image"])

    def step():
        rast.forward_l1(params, target, out=out, loss_out=loss, dl_out=dl, check=False)
        rast.backward_adam(params, out, dl, opt)

    def replayable(fn, rasts=None):
        fn()
        for r in (rasts if rasts is not None else [rast]):
            r.check()
        if args.no_graph:
            return fn
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream(dev).wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn()
        return graph.replay

    def timed(run, steps):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize(dev)
        return time.perf_counter() - t0

    run = replayable(step)
    log(f"timing {args.steps} steps")
    elapsed = timed(run, args.steps)
    rast.check()
    it_s = args.steps / elapsed
    ms = elapsed / args.steps * 1e3
    total_px = rast.total_px
    rec, pairs, tiles = rast.required_capacity()
    log(f"{it_s:.2f} it/s, {ms:.3f} ms/step, loss {loss.item():.5f}")

    # spread of single steps: HIP events around each of 30 more replays, on
    # the stream the replays run on
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(30)]
    for a, b in evs:
        a.record()
        run()
        b.record()
    torch.cuda.synchronize(dev)
    t_each = np.array([a.elapsed_time(b) for a, b in evs])
    spread = {"replays": len(t_each), "p10": float(np.percentile(t_each, 10)), "median": float(np.median(t_each)),
              "p90": float(np.percentile(t_each, 90))}
    log(f"single steps: median {spread['median']:.3f} ms (p10 {spread['p10']:.3f}, p90 {spread['p90']:.3f})")

    # achievable HBM bandwidth: the library's streaming copy of 1 GiB, read +
    # write bytes
    src = torch.ones(2**28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    device_copy(dst, src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        device_copy(dst, src)
    c1.record()
    torch.cuda.synchronize(dev)
    copy_gbs = 2 * src.numel() * 4 * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    log(f"streaming copy: {copy_gbs:.0f} GB/s ({copy_gbs / HBM_PEAK_GBS:.1%} of the 8 TB/s peak)")

    # per-stage durations from HIP events around each stage (eager steps)
    rast.profile(True)
    rast.profile_read(reset=True)
    for _ in range(args.profile_steps):
        step()
    stages = rast.profile_read(reset=True)
    rast.profile(False)
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    log("stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items() if v > 0))
    if min(stage_ms[st] for st in STEP_STAGES) <= 0.0:
        raise SystemExit("stage timing needs --profile-steps >= 1")
    k_sh = (scene.sh_degree + 1) ** 2
    pg = 11 + 3 * k_sh
    keys, vals, _ = rast.debug_binning()
    n_u = int(np.unique(vals).size)  # Gaussians visible in at least one view
    del keys, vals
    evals = rast.count_evaluations(out)
    composited = int(out["n_contrib"].sum().item())
    work = {st: stage_work(st, scene.n, n_u, pg, len(cams), total_px, rec, pairs, tiles, evals) for st in STEP_STAGES}
    stages = {}
    for st in STEP_STAGES:
        b, ops = work[st]
        t = stage_ms[st] * 1e-3
        e = {"ms": stage_ms[st], "bytes": b, "hbm_frac": b / t / (HBM_PEAK_GBS * 1e9) if t else None}
        if ops:
            e.update(ops=ops, alu_frac=ops / t / (VALU_PEAK_TOPS * 1e12) if t else None)
        stages[st] = e
    dom = max(STEP_STAGES, key=lambda k: stage_ms[k])
    b_dom, ops_dom = work[dom]
    t_dom = stage_ms[dom] * 1e-3
    kernel = STAGE_KERNEL.get(dom, dom) if rast.tile_size == 16 else dom
    workload = config_names()[args.config]
    traffic = recorded_traffic(kernel, workload) if args.scale == 1.0 else None
    if ops_dom:
        achieved = ops_dom / t_dom / 1e12
        roofline = {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": VALU_PEAK_TOPS,
                    "unit": "Tops/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                    "algorithmic_ops": ops_dom, "ops_per_evaluation": BWD_OPS_PER_EVAL if dom == "raster_bwd"
                    else FWD_OPS_PER_EVAL, "evaluations": evals, "duration_ms": stage_ms[dom],
                    "algorithmic_bytes": b_dom, "hbm_frac": b_dom / t_dom / (HBM_PEAK_GBS * 1e9)}
    else:
        achieved = b_dom / t_dom / 1e9
        roofline = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes": b_dom,
                    "duration_ms": stage_ms[dom]}
    total_b = sum(w[0] for w in work.values())
    # each stage at the slower of its two bounds, over the measured step
    ideal_s = sum(max(w[0] / (HBM_PEAK_GBS * 1e9), w[1] / (VALU_PEAK_TOPS * 1e12)) for w in work.values())
    log(f"dominant {kernel}: {roofline['achieved']:.2f} {roofline['unit']} = {roofline['frac']:.1%} of peak; "
        f"evaluations {evals} ({composited} composited); step HBM fraction {total_b / (ms * 1e-3) / 8e12:.1%}, "
        f"combined roofline fraction {ideal_s / (ms * 1e-3):.1%}")

    per_view = None
    if not args.no_per_view and len(cams) > 1:
        per_view = batching_comparison(scene, cams, target, params, rast, dev, args.steps, args.warmup, replayable,
                                       timed, ms)
        log(f"batched (same arrangement) {per_view['batched_it_s']:.2f} it/s, per-view plain launches "
            f"{per_view['per_view_it_s']:.2f} it/s as a graph ({per_view['per_view_eager_it_s']:.2f} eager): "
            f"batching {per_view['speedup_batching']:.2f}x")

    pose = None
    if not args.no_pose:
        # the rig of the workload: views frame-major; central pose = the
        # frame's camera 0, relative transforms from frame 0
        n_fr, n_cam = RIG_LAYOUT[args.config]
        frame = np.arange(len(cams)) // n_cam
        camid = np.arange(len(cams)) % n_cam
        rast.set_rig(frame, camid, n_fr, n_cam)
        T = np.zeros((len(cams), 4, 4))
        for v, c in enumerate(cams):
            T[v, :3, :3] = np.asarray(c.R, np.float64).reshape(3, 3)
            T[v, :3, 3] = np.asarray(c.t, np.float64)
            T[v, 3, 3] = 1.0
        central = np.stack([np.concatenate([T[f * n_cam, :3, :3].reshape(-1), T[f * n_cam, :3, 3]])
                            for f in range(n_fr)])
        rel = [np.linalg.inv(T[0]) @ T[k] for k in range(n_cam)]
        relative = np.stack([np.concatenate([r[:3, :3].reshape(-1), r[:3, 3]]) for r in rel])
        c_dev = torch.from_numpy(central.astype(np.float32)).to(dev)
        r_dev = torch.from_numpy(relative.astype(np.float32)).to(dev)
        camg = torch.empty(len(cams), 12, dtype=torch.float32, device=dev)
        rig_out = rast.rig_gradients(c_dev, r_dev, camg.zero_())

        def step_pose():
            rast.forward_l1(params, target, out=out, loss_out=loss, dl_out=dl, check=False)
            rast.backward_adam(params, out, dl, opt, cam_grads=camg)
            rast.rig_gradients(c_dev, r_dev, camg, out=rig_out)

        run_pose = replayable(step_pose)
        pose_s = timed(run_pose, args.steps)
        rast.check()
        pose_ms = pose_s / args.steps * 1e3
        rast.profile(True)
        rast.profile_read(reset=True)
        for _ in range(args.profile_steps):
            step_pose()
        st_pose = rast.profile_read(reset=True)
        rast.profile(False)
        pre_pose = st_pose["pre_bwd"][0] / max(st_pose["pre_bwd"][1], 1)
        pose = {"it_s": 1e3 / pose_ms, "ms_per_step": pose_ms, "overhead_ms": pose_ms - ms,
                "pre_bwd_ms": pre_pose, "pre_bwd_ms_without": stage_ms["pre_bwd"],
                "rig": {"frames": n_fr, "cameras": n_cam},
                "per_record_bytes": 48 + 48 + 4}
        log(f"with pose gradients: {1e3 / pose_ms:.2f} it/s ({pose_ms - ms:+.3f} ms/step; per-Gaussian stage "
            f"{pre_pose:.3f} ms vs {stage_ms['pre_bwd']:.3f} ms)")

    freq = None
    if not args.no_freq:
        fq = Frequency(rast.sizes, device=dev)
        x_gt = fq.significance(target)
        x_r = torch.empty_like(x_gt)
        levels = torch.zeros(len(cams), dtype=torch.int32, device=dev)
        u = torch.rand(len(cams), generator=torch.Generator(device=dev).manual_seed(5), device=dev)
        for _ in range(3):
            fq.significance(out["image"], out=x_r)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        reps = 20
        e0.record()
        for _ in range(reps):
            fq.significance(out["image"], out=x_r)
        e1.record()
        for _ in range(reps):
            fq.schedule(x_gt, x_r, x_gt_level=x_gt, levels=levels, uniforms=u)
        e2.record()
        torch.cuda.synchronize(dev)
        x_ms = e0.elapsed_time(e1) / reps
        s_ms = e1.elapsed_time(e2) / reps
        # image read once, half spectra written and read once
        fbytes = sum(12 * w * h + 2 * 24 * (w // 2 + 1) * h for w, h in rast.sizes)
        freq = {"significance_ms": x_ms, "schedule_ms": s_ms, "bytes": fbytes,
                "hbm_frac": fbytes / (x_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), "images": len(cams)}
        log(f"frequency significance of {len(cams)} views: {x_ms:.3f} ms ({freq['hbm_frac']:.1%} of HBM peak), "
            f"schedule step {s_ms:.3f} ms")

    ins = None
    if not args.no_insert:
        gts, rds, depths = make_insert_inputs(rast.sizes, 7000 + args.config)
        flat = lambda arrs: torch.from_numpy(np.concatenate([a.reshape(-1) for a in arrs])).to(dev)  # noqa: E731
        g_d, r_d, z_d = flat(gts), flat(rds), flat(depths)
        del gts, rds, depths
        res = rast.log_insert(g_d, r_d, z_d)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        reps = 20
        ev[0].record()
        for _ in range(reps):
            res = rast.log_insert(g_d, r_d, z_d)
        ev[1].record()
        torch.cuda.synchronize(dev)
        i_ms = ev[0].elapsed_time(ev[1]) / reps
        n_ins = int(res["count"].item())
        # both images read, P(I) and the mask written, the mask read twice;
        # per inserted pixel P(I) and z read, index, scale and centre written
        ibytes = total_px * (12 + 12 + 4 + 1 + 2) + n_ins * (8 + 20)
        ins = {"ms": i_ms, "bytes": ibytes, "hbm_frac": ibytes / (i_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
               "inserted": n_ins, "pixels": total_px}
        log(f"LoG insertion over {len(cams)} views: {i_ms:.3f} ms ({ins['hbm_frac']:.1%} of HBM peak), "
            f"{n_ins} pixels insert")
        mres = rast.merge(params, 0, g_d, res, tau_d=50.0)
        ev[0].record()
        for _ in range(reps):
            mres = rast.merge(params, 0, g_d, res, tau_d=50.0, out=mres)
        ev[1].record()
        torch.cuda.synchronize(dev)
        m_ms = ev[0].elapsed_time(ev[1]) / reps
        k0 = int((res["pix"][:n_ins] < rast.pix_off[1]).sum().item())
        # per Gaussian: mean and DC colour read twice, log-scale once, match
        # written and read, keep, colour and re-aligned mean written; per
        # sample of the view: its pixel read twice, slot and group (count,
        # colour and distance sums, winner key) written, its colour and centre
        # read, keep, colour and centre written
        mbytes = scene.n * (2 * 24 + 12 + 8 + 1 + 12 + 12) + k0 * (8 + 4 + 4 + 24 + 8 + 8 + 12 + 12 + 1 + 12 + 12)
        ins["merge"] = {"ms": m_ms, "bytes": mbytes, "hbm_frac": mbytes / (m_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                        "removed": int((mres["keep"][:scene.n] == 0).sum().item())}
        log(f"merge of {scene.n} Gaussians with view 0's samples: {m_ms:.3f} ms "
            f"({ins['merge']['hbm_frac']:.1%} of HBM peak)")

    window = None
    if not args.no_window and not args.no_per_view and args.config != 4:
        window = window_leg(args, dev, replayable, timed)

    cpu = None
    if pool is not None:
        log(f"timing the CPU oracle on pixel windows ({n_workers} worker processes)")
        cpu = cpu_baseline(pool, n_workers, args.config, args.scale, total_px, budget_s=args.cpu_budget)
        pool.close()
        pool.join()
        log(f"oracle: {cpu['mpix_per_s']:.5f} Mpix/s on {n_workers} cores")

    res = {
        "metric": METRIC,
        "value": it_s,
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": config_names()[args.config], "views": len(cams), "gaussians": scene.n,
                   "sh_degree": scene.sh_degree, "pixels": total_px, "tile_size": rast.tile_size,
                   "tuning": rast.tuning() if tuning is None else tuning,
                   "graph": not args.no_graph, "batched": True},
        "mpix_per_s": total_px * it_s / 1e6,
        "records": rec,
        "pairs": pairs,
        "evaluations": evals,
        "composited": composited,
        "visible_gaussians": n_u,
        "stages": stages,
        "step_hbm_bytes": total_b,
        "step_hbm_frac": total_b / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "step_ms_spread": spread,
        "hbm_copy_gbs": copy_gbs,
        "step_hbm_frac_of_copy": total_b / (ms * 1e-3) / (copy_gbs * 1e9),
        "combined_roofline_frac": ideal_s / (ms * 1e-3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_view": per_view,
        "window": window,
        "pose": pose,
        "freq": freq,
        "insert": ins,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
