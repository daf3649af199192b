#!/usr/bin/env python3
"""Training-iteration benchmark of the differentiable Gaussian rasterizer.

One step = forward render of every view of the batch, L1 loss against the
target images, backward to all Gaussian parameters and a dense Adam update
(fused into the per-Gaussian backward), all in the HIP library, replayed as
one captured HIP graph.  Default workload: the 6-camera 1600x900 ring rig in
a street corridor with 1M Gaussians (SH degree 3).

Prints one JSON line (rank 0).  Besides the throughput it reports:
  roofline      achieved vs peak of the dominant kernel, its duration taken
                from HIP events recorded around it on the library's stream
                during an eager pass of the same steps
  cpu_baseline  the FP64 CPU oracle timed on a bounded pixel sample
  per_view      the same step issued as plain per-view launches (no batching,
                no graph), for comparison
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


def algorithmic_bytes(stage, n, k_sh, views, px, rec, pairs, fused_adam=True):
    """Bytes each stage must move at least once (see the design notes):
    parameters read, records / pairs written and read, images, Adam state."""
    pg = 11 + 3 * k_sh  # parameters per Gaussian
    if stage == "preprocess":
        return 4 * pg * n + 64 * rec + 24 * rec          # params in; payload + meta out
    if stage == "binning":
        return 24 * rec + 8 * pairs                       # meta in; entries out
    if stage == "sort":
        return 8 * pairs + 4 * pairs                      # entries in; sorted records out
    if stage == "raster_fwd":
        return 4 * pairs + 64 * rec + 24 * px             # lists + payload in; image, T, last, count out
    if stage == "loss":
        return 36 * px                                    # image + target in; gradient out
    if stage == "raster_bwd":
        return 4 * pairs + 64 * rec + 20 * px + 36 * pairs  # lists, payload, dL/dC, T, last in; partials out
    if stage == "reduce":
        return 36 * pairs + 36 * rec
    if stage == "pre_bwd":
        b = 4 * (pg * n) + 36 * rec                       # params + record grads in
        return b + (24 * pg * n if fused_adam else 4 * pg * n)  # Adam: m, v in/out, p out
    if stage == "adam":
        return 28 * pg * n
    return 0


def cpu_baseline(scene, cams, targets, total_px, budget_s=15.0, win=32, seed=3003):
    """The oracle (forward + gradients) on random win x win pixel windows."""
    import torch

    from oracle.grad64 import grad64
    from oracle.render64 import render_view
    from oracle.project64 import to_params64

    arrays = scene.arrays()
    p64 = to_params64(arrays)
    rng = np.random.default_rng(seed)
    done_px, n_win = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n_win < 64:
        v = n_win % len(cams)
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
    dt = time.perf_counter() - t0
    mpix = done_px / dt / 1e6
    return {"value": mpix * 1e6 / total_px, "unit": "it/s", "mpix_per_s": mpix, "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n_win} windows of {win}x{win} px across the views (forward + FP64 autograd backward), "
                      f"{dt:.1f} s; rate scaled to one full iteration of {total_px} px"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--tile-size", type=int, default=16)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the rasterizer path is single-GPU (multi-GPU sharding by view is "
              "described in DESIGN.md but not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2512_08498_amd import FusedAdam, Rasterizer
    from workloads import config_names, make_config, make_target

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t_setup = time.perf_counter()
    scene, cams = make_config(args.config, args.scale)
    targets = make_target(args.config, cams)
    log(f"workload {config_names()[args.config]}: {scene.n} Gaussians, {len(cams)} views "
        f"({time.perf_counter() - t_setup:.1f} s to generate)")
    params = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.arrays().items()}
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in targets])).to(dev)

    rast = Rasterizer(cams, scene.n, scene.sh_degree, tile_size=args.tile_size, device=dev)
    out = rast.forward(params)  # re-plans on capacity overflow
    rec, pairs, tiles = rast.required_capacity()
    # headroom for the scene to move during training
    rast._plan(int(rec * 1.5) + 4096, int(pairs * 1.5) + 65536)
    out = rast.new_fwd_out()
    log(f"records {rec}, pairs {pairs}, tiles {tiles}, workspace {rast.ws_bytes / 2**30:.2f} GiB")
    opt = FusedAdam(rast, params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    dl = torch.empty_like(out["image"])

    def step():
        rast.forward(params, out=out, check=False)
        rast.l1_loss(out["image"], target, loss, dl)
        rast.backward_adam(params, out, dl, opt)

    step()
    rast.check()
    run = step
    if not args.no_graph:
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream(dev).wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        run = graph.replay
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize(dev)
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t0
    rast.check()
    it_s = args.steps / elapsed
    ms = elapsed / args.steps * 1e3
    total_px = rast.total_px
    rec, pairs, tiles = rast.required_capacity()
    log(f"{it_s:.2f} it/s, {ms:.3f} ms/step, loss {loss.item():.5f}")

    # per-stage durations from HIP events around each stage (eager steps)
    rast.profile(True)
    rast.profile_read(reset=True)
    for _ in range(args.profile_steps):
        step()
    stages = rast.profile_read(reset=True)
    rast.profile(False)
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    log("stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items() if v > 0))
    k_sh = (scene.sh_degree + 1) ** 2
    dom = max(stage_ms, key=stage_ms.get)
    b = algorithmic_bytes(dom, scene.n, k_sh, len(cams), total_px, rec, pairs)
    achieved = b / (stage_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": b,
                "duration_ms": stage_ms[dom]}
    total_b = sum(algorithmic_bytes(s, scene.n, k_sh, len(cams), total_px, rec, pairs)
                  for s in ("preprocess", "binning", "sort", "raster_fwd", "loss", "raster_bwd", "reduce", "pre_bwd"))

    per_view = None
    if not args.no_per_view and len(cams) > 1:
        rs = [Rasterizer([c], scene.n, scene.sh_degree, tile_size=args.tile_size, device=dev) for c in cams]
        outs = []
        for r in rs:
            o = r.forward(params)
            rr, pp, _ = r.required_capacity()
            r._plan(int(rr * 1.5) + 4096, int(pp * 1.5) + 65536)
            outs.append(r.new_fwd_out())
        grads = {k: torch.zeros_like(v) for k, v in params.items()}
        tv = [target[3 * rast.pix_off[v]:3 * rast.pix_off[v + 1]] for v in range(len(cams))]
        dls = [torch.empty_like(o["image"]) for o in outs]
        opt2 = FusedAdam(rast, params)

        def step_pv():
            for v, r in enumerate(rs):
                r.forward(params, out=outs[v], check=False)
                r.l1_loss(outs[v]["image"], tv[v], loss, dls[v])
                dls[v].mul_(1.0 / len(cams))
                r.backward(params, outs[v], dls[v], grads=grads, accumulate=v > 0)
            opt2.apply(grads)

        for _ in range(3):
            step_pv()
        torch.cuda.synchronize(dev)
        n_pv = max(5, args.steps // 4)
        t1 = time.perf_counter()
        for _ in range(n_pv):
            step_pv()
        torch.cuda.synchronize(dev)
        pv_ms = (time.perf_counter() - t1) / n_pv * 1e3
        per_view = {"it_s": 1e3 / pv_ms, "ms_per_step": pv_ms, "speedup_batched": pv_ms / ms}
        log(f"per-view plain launches: {1e3 / pv_ms:.2f} it/s")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a pixel sample")
        cpu = cpu_baseline(scene, cams, targets, total_px, budget_s=args.cpu_budget)

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
                   "sh_degree": scene.sh_degree, "pixels": total_px, "tile_size": args.tile_size,
                   "graph": not args.no_graph, "batched": True},
        "mpix_per_s": total_px * it_s / 1e6,
        "records": rec,
        "pairs": pairs,
        "stage_ms": stage_ms,
        "whole_step_hbm_frac": total_b / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_view": per_view,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
