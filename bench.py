#!/usr/bin/env python3
"""Benchmark of the VEG rasterizer's training step on one MI355X.

Workload (the configuration the headline metric is quoted on): 1,000,000 shell-clustered
Gaussians (70% on 5 spherical shells, 30% uniform; scales log-uniform [0.002, 0.03]),
16 orbit views x 3 random transfer functions = 48 frames at 1024x1024, L1 loss against
targets rendered from a perturbed copy (rendered before timing).  One step = forward +
L1 + backward + parameter gradients for all 48 frames, processed in groups of frames
with the forward recomputed per group (only one group's key lists are alive).

Prints ONE JSON line.  ``value`` = forward+backward megapixels per second of the whole
step (48 * 1024^2 * steps / seconds), inputs resident in HBM.  ``roofline`` covers the
kernel with the largest share of the step, timed with HIP events on the library's stream.
``cpu_baseline`` times the float64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd & fwd+bwd Mpix/s at 1M Gaussians; serve p50/p99 ms vs plain render loop"

# Per-unit algorithmic work of the blend kernels (one unit = one Gaussian-pixel
# evaluation visited before the pixel stops): ~20 VALU lane-operations forward, 2.5x that
# backward.  Peak: 256 CUs x 64 lanes x 2.4 GHz of non-packed FP32 issue.
FWD_OPS_PER_EVAL = 20.0
BWD_OPS_PER_EVAL = 50.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12          # 39.32 T lane-ops/s
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_inputs(args):
    import numpy as np
    import torch

    import synth
    from paper_2504_13339_amd import render as R
    from paper_2504_13339_amd import veg as V

    w = synth.workload(2, n_override=args.n, views_override=args.views, tfs_override=args.tfs,
                       res_override=args.res)
    g = V.Gaussians.from_numpy(w.gaussians)
    gt = V.Gaussians.from_numpy(w.target_gaussians)
    luts = [torch.as_tensor(t).cuda() for t in w.tfs]
    F = len(w.frames)
    H = W = w.width
    targets = torch.empty((F, 3, H, W), dtype=torch.float32, device="cuda")
    for f0 in range(0, F, args.group):
        fr = w.frames[f0:f0 + args.group]
        st = R.render(gt, [w.cameras[c] for c, _ in fr], [luts[t] for _, t in fr], w.opts)
        targets[f0:f0 + len(fr)] = st.image
        del st
    torch.cuda.synchronize()
    return w, g, luts, targets


def eval_counts(st, t_min):
    """Visited Gaussian-pixel evaluations of one group, from the forward's per-pixel state:
    forward = entries from the tile start through the stop entry (or the whole list when
    the pixel never stops); backward = entries from the tile start through n_last."""
    import torch
    proj, bins = st.proj, st.bins
    F, H, W = st.t_final.shape
    tx_n, ty_n = int(proj.struct.tiles_x), int(proj.struct.tiles_y)
    ys = torch.arange(H, device="cuda").view(1, H, 1) // 16
    xs = torch.arange(W, device="cuda").view(1, 1, W) // 16
    fs = torch.arange(F, device="cuda").view(F, 1, 1)
    tile = (fs * (tx_n * ty_n) + ys * tx_n + xs).reshape(-1).long()
    rg = bins.ranges.view(-1, 2).long()
    start = rg[tile, 0]
    end = rg[tile, 1]
    nl = st.n_last.reshape(-1).long()
    stopped = st.t_final.reshape(-1) < t_min
    bwd = torch.where(nl >= 0, nl - start + 1, torch.zeros_like(nl))
    fwd = torch.where(stopped, nl - start + 1, end - start)
    return int(fwd.sum()), int(bwd.sum())


def cpu_baseline(w, n_pixels, seed=5):
    """The oracle (float64 brute force + autograd adjoint) on ``n_pixels`` sampled pixels of
    the first frame of the workload, forward and backward."""
    import numpy as np
    import torch

    import oracle
    import synth
    cores = torch.get_num_threads()
    rng = synth.rng_for(2, 100 + seed)
    ci, ti = w.frames[0]
    cam = w.cameras[ci]
    px = synth.sample_pixels(rng, cam.width, cam.height, n_pixels)
    d = rng.standard_normal((n_pixels, 3))
    t0 = time.perf_counter()
    oracle.gradients(w.gaussians, cam, w.tfs[ti], w.opts, d, pixels=px)
    dt = time.perf_counter() - t0
    return {"value": n_pixels / dt / 1e6, "unit": "Mpix/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n_pixels} sampled pixels of frame 0 (1024x1024, {w.gaussians.n} Gaussians), "
                      f"float64 projection of every Gaussian + brute-force forward + autograd backward, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--group", type=int, default=16, help="frames per recompute group")
    ap.add_argument("--n", type=int, default=None, help="override Gaussian count (testing only)")
    ap.add_argument("--views", type=int, default=None)
    ap.add_argument("--tfs", type=int, default=None)
    ap.add_argument("--res", type=int, default=None)
    ap.add_argument("--cpu-pixels", type=int, default=48)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(frames would be split across GPUs with one gradient all-reduce; not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_13339_amd import render as R

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("bench: building inputs")
    w, g, luts, targets = build_inputs(args)
    F = len(w.frames)
    H = W = w.width
    grads = R.Grads.zeros(g)
    loss_acc = torch.empty(1, dtype=torch.float64, device="cuda")
    t_min = float(w.opts["t_min"])

    # warm-up; the first warm-up step also counts the visited evaluations per group
    counts = {"fwd": 0, "bwd": 0}

    def count_group(f0, st):
        a, b = eval_counts(st, t_min)
        counts["fwd"] += a
        counts["bwd"] += b

    for k in range(args.warmup):
        res = R.train_step_l1(g, w.cameras, luts, w.frames, targets, grads, args.group, w.opts, loss_acc=loss_acc,
                              on_group=count_group if k == 0 else None)
        log(f"bench: warm-up step {k} loss {res.loss:.6f} entries {res.n_entries}")
    if args.warmup == 0:
        R.train_step_l1(g, w.cameras, luts, w.frames, targets, grads, args.group, w.opts, loss_acc=loss_acc,
                        on_group=count_group)

    # timed steps
    timer = R.EventTimer()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = R.train_step_l1(g, w.cameras, luts, w.frames, targets, grads, args.group, w.opts, loss_acc=loss_acc,
                              timer=timer)
        log(f"bench: step {k} loss {res.loss:.6f}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    value = F * H * W * args.steps / dt / 1e6

    times = timer.totals_ms()
    per_step = {k: sum(v) / args.steps for k, v in times.items()}
    launches = {k: len(v) // args.steps for k, v in times.items()}

    # forward-only throughput (project + bin + blend for all frames, no backward)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        for f0 in range(0, F, args.group):
            fr = w.frames[f0:f0 + args.group]
            st = R.render(g, [w.cameras[c] for c, _ in fr], [luts[t] for _, t in fr], w.opts)
            del st
    torch.cuda.synchronize()
    fwd_mpix = F * H * W * args.steps / (time.perf_counter() - t1) / 1e6

    # roofline of the dominant kernel (blend forward or backward: VALU-bound)
    dom = max(("blend_bwd", "blend_fwd"), key=lambda k: per_step.get(k, 0.0))
    evals = counts["bwd"] if dom == "blend_bwd" else counts["fwd"]
    ops = BWD_OPS_PER_EVAL if dom == "blend_bwd" else FWD_OPS_PER_EVAL
    n_launch = launches[dom]
    avg_ms = per_step[dom] / n_launch
    ach = evals / n_launch * ops / (avg_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TFLOP/s", "frac": round(ach / VALU_PEAK_TOPS, 4), "traffic": None,
            "avg_launch_ms": round(avg_ms, 4), "evals_per_launch": evals // n_launch,
            "ops_per_eval": ops, "note": "T lane-ops/s (FMA = 1 op), non-packed FP32 issue peak"}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "gaussians": w.gaussians.n, "frames": F, "width": W, "height": H,
                   "group": args.group},
        "fwd_mpix_s": round(fwd_mpix, 2),
        "geval_s": {"fwd": round(counts["fwd"] * args.steps / dt / 1e9, 3),
                    "bwd": round(counts["bwd"] * args.steps / dt / 1e9, 3)},
        "kernel_ms_per_step": {k: round(v, 3) for k, v in sorted(per_step.items(), key=lambda kv: -kv[1])},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
