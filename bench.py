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
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd & fwd+bwd Mpix/s at 1M Gaussians; serve p50/p99 ms vs plain render loop"

# Algorithmic FLOPs of the blend kernels, counted from the definition (each add, multiply,
# compare, min and exp counts 1):
#   every visited Gaussian-pixel pair (both passes): d = p - mu' (2), the quadratic form
#     sigma = 1/2 (a dx^2 + 2b dx dy + c dy^2) (8), a = A exp(-sigma) (2), skip test (1) = 13
#   every blended pair, forward: alpha = min (1), w = alpha T (1), C += w c (6),
#     T *= 1 - alpha (2), stop test (1) = 11
#   every blended pair, backward: alpha, 1 - alpha, T / (1 - alpha), w (4), dL/dc (6),
#     dL/dalpha (9), colour-behind update (6), dL/dA and dL/dsigma (3), dL/dconic (10),
#     dL/dmu' (10) = 48
# Peak: 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s of non-packed FP32 (the build
# disables packed FP32; the packed figure, 157.3, is reported beside it).
FLOPS_VISIT = 13.0
FLOPS_BLEND_FWD = 11.0
FLOPS_BLEND_BWD = 48.0
VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12    # 78.64
VALU_PACKED_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "train-1M-1024px-16x3_hbm_traffic.md")
BLEND_SOURCES = ("paper_2504_13339_amd/csrc/veg_blend.hip", "paper_2504_13339_amd/csrc/veg_internal.h")
PROFILE_KERNEL = {"blend_bwd": "void blend_bwd_kernel<true>", "blend_fwd": "void blend_fwd_kernel<false, true, {shared}>"}


def profiled_traffic(name, shared=True):
    """HBM bytes per launch of a blend kernel from the committed counter summary (FETCH_SIZE
    and WRITE_SIZE passes calibrated on a plain copy), or None when the blend sources have
    changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for p in BLEND_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    m = re.search(r"sha256\(veg_blend\.hip \+ veg_internal\.h\): ([0-9a-f]{64})", text)
    if not m or m.group(1) != h.hexdigest():
        return None
    kernel = PROFILE_KERNEL[name].format(shared="true" if shared else "false")
    row = re.search(r"^\| `" + re.escape(kernel) + r"` \|([^\n]*)$", text, flags=re.M)
    if not row:
        return None
    return float(row.group(1).split("|")[-2])


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
    K = max(1, int(proj.struct.tfs_per_view))      # frames sharing a list walk their view's tiles
    fs = (torch.arange(F, device="cuda") // K).view(F, 1, 1)
    tile = (fs * (tx_n * ty_n) + ys * tx_n + xs).reshape(-1).long()
    rg = bins.ranges.view(-1, 2).long()
    start = rg[tile, 0]
    end = rg[tile, 1]
    nl = st.n_last.reshape(-1).long()
    stopped = st.t_final.reshape(-1) < t_min
    bwd = torch.where(nl >= 0, nl - start + 1, torch.zeros_like(nl))
    fwd = torch.where(stopped, nl - start + 1, end - start)
    blended = int(st.n_contrib.long().sum()) if st.n_contrib is not None else 0
    return int(fwd.sum()), int(bwd.sum()), blended


def opacity_guided_bench(steps, warmup=2):
    """The opacity-guided training family (500k shell-clustered Gaussians, 8 views x 10 tent
    opacity maps, 800x800, targets from a perturbed copy): L1 training steps over all 80
    frames with a view's ten frames on one shared list, with neighbouring maps sharing in
    pairs, and with every frame on its own list."""
    import torch

    import synth
    from paper_2504_13339_amd import render as R
    from paper_2504_13339_amd import veg as V
    w = synth.workload(5)
    g = V.Gaussians.from_numpy(w.gaussians)
    gt = V.Gaussians.from_numpy(w.target_gaussians)
    luts = [torch.as_tensor(t).cuda() for t in w.tfs]
    F = len(w.frames)
    K = R.views_of(w.frames)
    st = R.render(gt, w.cameras, [luts[t] for _, t in w.frames], w.opts, shared=True, hits=False)
    targets = st.image.clone()
    del st
    grads = R.Grads.zeros(g)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    out = {"workload": w.name, "frames": F, "tables_per_view": K, "width": w.width, "height": w.height}
    for shared in (True, 2, False):
        def step(**kw):
            return R.train_step(g, w.cameras, luts, w.frames, targets, grads, F, w.opts, loss_acc=loss, shared=shared,
                                **kw)
        cap = max(step().n_entries)   # lists sized ahead, as in the main timed loop
        for _ in range(warmup):
            step(capacity=cap)
        stat = []
        gc.collect()
        gc.disable()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            stat.append(step(capacity=cap, read_loss=False).status)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        gc.enable()
        for st in stat:
            R.check_status(st, cap)
        key = "shared" if shared is True else "pairs_shared" if shared else "own_lists"
        out[key + "_mpix_s"] = round(F * w.width * w.height * steps / dt / 1e6, 2)
        out[key + "_ms_per_step"] = round(dt * 1e3 / steps, 3)
    del grads, targets, g, gt
    torch.cuda.empty_cache()
    return out


def workload_step_bench(index, steps, warmup=1, group=None, shared=True):
    """Forward + backward Mpix/s of another configuration's whole L1 training step (all its
    frames, targets from a perturbed copy, lists sized from the last warm-up step): the
    multi-TF workload (200k Gaussians, 8 views x 4 tables, 800x800) or the stress workload
    (4M Gaussians, 32 views x 4 tables, 2048x2048)."""
    import torch

    import synth
    from paper_2504_13339_amd import render as R
    from paper_2504_13339_amd import veg as V
    w = synth.workload(index)
    g = V.Gaussians.from_numpy(w.gaussians)
    gt = V.Gaussians.from_numpy(w.target_gaussians)
    luts = [torch.as_tensor(t).cuda() for t in w.tfs]
    F, H, W = len(w.frames), w.height, w.width
    group = group or F
    K = R.views_of(w.frames) if shared else 1
    targets = torch.empty((F, 3, H, W), dtype=torch.float32, device="cuda")
    for f0 in range(0, F, group):
        fr = w.frames[f0:f0 + group]
        cams = [w.cameras[c] for c, _ in (fr[::K] if K > 1 else fr)]
        st = R.render(gt, cams, [luts[t] for _, t in fr], w.opts, hits=False, shared=K > 1)
        targets[f0:f0 + len(fr)] = st.image
        del st
    grads = R.Grads.zeros(g)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    # one zeroed g2d buffer for every group, left zero by each group's projection backward
    g2d = torch.zeros(9 * w.gaussians.n * min(F, max(group, K)), dtype=torch.float32, device="cuda")

    def step(**kw):
        return R.train_step(g, w.cameras, luts, w.frames, targets, grads, group, w.opts, loss_acc=loss,
                            shared=shared, g2d=g2d, **kw)
    res = step()
    cap = int(max(res.n_entries) * 1.05) + 4096
    for _ in range(warmup):
        R.check_status(step(capacity=cap, read_loss=False).status, cap)
    stat = []
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stat.append(step(capacity=cap, read_loss=False).status)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gc.enable()
    for st in stat:
        R.check_status(st, cap)
    out = {"workload": w.name, "gaussians": w.gaussians.n, "frames": F, "width": W, "height": H, "group": group,
           "shared_views": bool(shared), "max_entries_per_group": int(max(res.n_entries)),
           "mpix_s": round(F * H * W * steps / dt / 1e6, 2), "ms_per_step": round(dt * 1e3 / steps, 3)}
    del grads, targets, g, gt, g2d
    torch.cuda.empty_cache()
    return out


def stress_serve_bench(n_frames=64, max_batch=8, n_streams=2):
    """The stress workload's serving leg: a batch of ``n_frames`` 2048x2048 frames of the 4M-
    Gaussian model, each with its own camera (the workload's views) and one of its transfer
    functions, submitted at once to a server (continuous batching, captured graphs) and,
    for comparison, rendered one after another by the plain stateless loop; Mpix/s of the
    whole batch and latency from submission."""
    import numpy as np
    import torch

    import synth
    from paper_2504_13339_amd import render as R
    from paper_2504_13339_amd import veg as V
    from paper_2504_13339_amd.serve import Server
    w = synth.workload(4)
    g = V.Gaussians.from_numpy(w.gaussians)
    frames = [(f % len(w.cameras), f % len(w.tfs)) for f in range(n_frames)]
    res = w.width
    srv = Server(max_gaussians=w.gaussians.n, max_entries=1 << 29, max_batch=max_batch, n_streams=n_streams,
                 use_graphs=True, max_width=res, max_height=res, max_tf_k=256)
    mid = srv.add_model(g)
    outs = [torch.empty((3, res, res), device="cuda") for _ in range(n_frames)]

    def serve_once():
        srv.reset_stats()
        t0 = time.perf_counter()
        ids = [srv.submit(mid, w.cameras[c], w.tfs[t], outs[i], t_arrival=t0) for i, (c, t) in enumerate(frames)]
        for rid in ids:
            srv.wait(rid)
        return time.perf_counter() - t0, srv.stats()
    serve_once()                                   # graph capture
    dt, st = serve_once()
    luts = [torch.as_tensor(t).cuda() for t in w.tfs]
    R.render(g, [w.cameras[0]], [luts[0]], w.opts, hits=False)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for c, t in frames:
        st_p = R.render(g, [w.cameras[c]], [luts[t]], w.opts, hits=False)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
        del st_p
    dtp = time.perf_counter() - t0
    srv.close()
    px = n_frames * res * res
    return {"workload": w.name + "-serve", "frames": n_frames, "width": res, "height": res,
            "server": {"mpix_s": round(px / dt / 1e6, 2), "seconds": round(dt, 4), "p50_ms": round(st["p50_ms"], 3),
                       "p99_ms": round(st["p99_ms"], 3), "mean_batch": round(st["mean_batch"], 3),
                       "retries": int(st["retries"])},
            "plain": {"mpix_s": round(px / dtp / 1e6, 2), "seconds": round(dtp, 4),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3)}}


def cpu_baseline(w, n_pixels, seed=5, one_core_pixels=64):
    """The oracle (float64 brute force + autograd adjoint) on the host's cores: forward and
    backward of ``n_pixels`` sampled pixels of the first frame of the workload on every core
    of this process's affinity set, the same on one core with ``one_core_pixels`` pixels,
    and a whole 64x64 frame of the 1k-Gaussian workload (forward + backward) on all cores
    and on one."""
    import numpy as np
    import torch

    import oracle
    import synth
    cores = len(os.sched_getaffinity(0))
    threads0 = torch.get_num_threads()
    rng = synth.rng_for(2, 100 + seed)
    ci, ti = w.frames[0]
    cam = w.cameras[ci]
    px = synth.sample_pixels(rng, cam.width, cam.height, n_pixels)
    d = rng.standard_normal((n_pixels, 3))

    def timed(threads, fn):
        torch.set_num_threads(threads)
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    dt = timed(cores, lambda: oracle.gradients(w.gaussians, cam, w.tfs[ti], w.opts, d, pixels=px))
    k1 = min(one_core_pixels, n_pixels)
    dt1 = timed(1, lambda: oracle.gradients(w.gaussians, cam, w.tfs[ti], w.opts, d[:k1], pixels=px[:k1]))
    w0 = synth.workload(0)
    cam0 = w0.cameras[0]
    d0 = rng.standard_normal((cam0.width * cam0.height, 3))
    f_all = timed(cores, lambda: oracle.gradients(w0.gaussians, cam0, w0.tfs[0], w0.opts, d0))
    f_one = timed(1, lambda: oracle.gradients(w0.gaussians, cam0, w0.tfs[0], w0.opts, d0))
    torch.set_num_threads(threads0)
    npx0 = cam0.width * cam0.height
    return {"value": n_pixels / dt / 1e6, "unit": "Mpix/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n_pixels} sampled pixels of frame 0 ({cam.width}x{cam.height}, {w.gaussians.n} Gaussians), "
                      f"float64 projection of every Gaussian + brute-force forward + autograd backward, "
                      f"{dt:.1f} s on {cores} threads",
            "one_core": {"value": k1 / dt1 / 1e6, "unit": "Mpix/s", "cores": 1,
                         "sample": f"{k1} of the same pixels, {dt1:.1f} s"},
            "full_frame_1k_64px": {"seconds_all_cores": round(f_all, 3), "seconds_one_core": round(f_one, 3),
                                   "mpix_s_all_cores": npx0 / f_all / 1e6, "mpix_s_one_core": npx0 / f_one / 1e6,
                                   "sample": f"a whole {cam0.width}x{cam0.height} frame of {w0.gaussians.n} "
                                             f"Gaussians, forward + backward"}}


def serve_bench(rates, min_requests=2000, max_seconds=30.0, max_batch=8, n_streams=3, budget_gb=64.0,
                saturate=2.0):
    """Serving workload: 4 resident shell-clustered models (100k, 500k, 1M, 3M Gaussians),
    open-loop Poisson arrivals, each request a random model, camera on a sphere of radius
    2.5-4, fresh random 256-entry TF and a resolution from {512^2, 1024^2, 1920x1080}; an
    HBM admission budget of ``budget_gb``.  Each rate serves min(``min_requests``, rate x
    ``max_seconds``) requests, then one more rate ``saturate`` times the plain loop's measured
    capacity.  The server (continuous batching) and the plain loop (stateless API, one
    request at a time in arrival order) serve the same trace; for both, latency = completion
    - scheduled arrival and throughput = requests / (last completion - first arrival)."""
    import numpy as np
    import torch

    import synth
    from paper_2504_13339_amd import render as R
    from paper_2504_13339_amd import veg as V
    from paper_2504_13339_amd.serve import Server

    models_np, _ = synth.serve_trace(1.0, 1)
    models = [V.Gaussians.from_numpy(m) for m in models_np]
    opts = synth.DEFAULT_OPTS
    results = {"models": [m.n for m in models], "resolutions": ["512x512", "1024x1024", "1920x1080"],
               "max_batch": max_batch, "streams": n_streams, "graphs": True, "budget_gb": budget_gb, "rates": {}}
    srv = Server(max_gaussians=max(m.n for m in models), max_entries=64_000_000, max_batch=max_batch,
                 n_streams=n_streams, use_graphs=True, max_width=1920, max_height=1080, max_tf_k=256,
                 budget_bytes=int(budget_gb * 1e9))
    results["arena_gb"] = round(srv.arena_bytes / 1e9, 2)
    mids = [srv.add_model(m) for m in models]
    RING = 256
    ring = {}

    def run_server(reqs):
        srv.reset_stats()
        users = {}
        t0 = time.perf_counter() + 0.05
        ids = []
        for r in reqs:
            target = t0 + r.arrival_s
            while time.perf_counter() < target:   # the same busy-wait pacing as the plain loop
                pass
            key = (r.camera.width, r.camera.height)
            bufs = ring.get(key)
            if bufs is None:   # (allocated once per resolution, not on every request)
                bufs = ring[key] = [torch.empty((3, key[1], key[0]), device="cuda") for _ in range(RING)]
            used = users.setdefault(key, [])
            k = len(used) % RING
            if len(used) >= RING and used[len(used) - RING] is not None:
                srv.wait(used[len(used) - RING])       # the buffer's previous request is done with it
                used[len(used) - RING] = None
            rid = srv.submit(mids[r.model], r.camera, r.tf, bufs[k], t_arrival=target)
            used.append(rid)
            ids.append(rid)
        for lst in users.values():
            for rid in lst:
                if rid is not None:
                    srv.wait(rid)
        return srv.stats()

    def run_plain(reqs):
        luts = [torch.as_tensor(r.tf).cuda() for r in reqs]
        torch.cuda.synchronize()
        lat, service = [], []
        t0 = time.perf_counter() + 0.05
        for i, r in enumerate(reqs):
            target = t0 + r.arrival_s
            while time.perf_counter() < target:
                pass
            ts = time.perf_counter()
            st = R.render(models[r.model], [r.camera], [luts[i]], opts, hits=False)   # forward only
            torch.cuda.synchronize()
            te = time.perf_counter()
            lat.append((te - target) * 1e3)
            service.append(te - ts)
            del st
        span = te - (t0 + reqs[0].arrival_s)
        lat = np.sort(np.asarray(lat))
        pix = sum(r.camera.width * r.camera.height for r in reqs)
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(lat[-1]), "throughput_rps": len(reqs) / span, "mpix_per_s": pix / span / 1e6,
                "mean_service_ms": float(np.mean(service) * 1e3)}

    def one_rate(label, rate, n, seed):
        _, reqs = synth.serve_trace(float(rate), int(n), build_models=False, seed_sub=seed)
        log(f"bench: serving {len(reqs)} requests at {rate:.0f} req/s")
        st = run_server(reqs)
        pl = run_plain(reqs)
        results["rates"][label] = {
            "rate": round(float(rate), 1), "requests": len(reqs),
            "server": {k2: round(float(st[k2]), 3) for k2 in ("p50_ms", "p99_ms", "max_ms", "throughput_rps",
                                                              "mpix_per_s", "mean_batch", "gpu_busy_frac")} |
                      {"completed": int(st["completed"]), "retries": int(st["retries"]),
                       "peak_gb": round(st["peak_bytes"] / 1e9, 2), "graphs_captured": int(st["graphs_captured"])},
            "plain": {k2: round(v, 3) for k2, v in pl.items()}}
        return pl

    # warm-up: graph capture for the common batch shapes, allocator
    _, warm = synth.serve_trace(2000.0, 400, build_models=False, seed_sub=99)
    run_server(warm)
    run_plain(warm[:16])
    cap = None
    for k, rate in enumerate(rates):
        n = max(1, min(int(min_requests), int(math.ceil(rate * max_seconds))))
        pl = one_rate(str(rate), rate, n, k)
        cap = 1e3 / pl["mean_service_ms"]
    if saturate and cap:
        one_rate("saturating", saturate * cap, int(min_requests), len(rates))
        results["plain_capacity_rps"] = round(cap, 1)
    srv.close()
    return results


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--group", type=int, default=48, help="frames per recompute group")
    ap.add_argument("--no-shared", dest="shared", action="store_false",
                    help="give every frame its own projection and key list (veg_project) instead of sharing "
                         "them between the frames of one camera (veg_project_views)")
    ap.add_argument("--n", type=int, default=None, help="override Gaussian count (testing only)")
    ap.add_argument("--views", type=int, default=None)
    ap.add_argument("--tfs", type=int, default=None)
    ap.add_argument("--res", type=int, default=None)
    ap.add_argument("--cpu-pixels", type=int, default=640)
    ap.add_argument("--lit-steps", type=int, default=5,
                    help="timed steps of the same workload with lighting attributes (0 to skip)")
    ap.add_argument("--og-steps", type=int, default=5,
                    help="timed training steps of the opacity-guided family (8 views x 10 tent opacity maps, "
                         "800x800, 500k Gaussians), shared and own lists (0 to skip)")
    ap.add_argument("--full-steps", type=int, default=5,
                    help="timed whole training iterations: L1 + SSIM loss, densification statistics, Adam (0 to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c1-steps", type=int, default=5,
                    help="timed training steps of the multi-TF workload (200k, 8 x 4 frames, 800x800; 0 to skip)")
    ap.add_argument("--c4-steps", type=int, default=2,
                    help="timed training steps of the stress workload (4M, 32 x 4 frames, 2048x2048; 0 to skip)")
    ap.add_argument("--c4-serve", type=int, default=64,
                    help="frames of the stress workload's 2048x2048 serving batch (0 to skip)")
    ap.add_argument("--serve-rates", default="50,100,200,400",
                    help="comma-separated arrival rates (req/s), each followed by a rate twice the plain loop's "
                         "capacity; '' to skip")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per rate (fewer when the rate reaches them only after --serve-seconds)")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 3 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(args.calibrate_copy // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": a.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(frames would be split across GPUs with one gradient all-reduce; not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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

    K = R.views_of(w.frames) if args.shared else 1
    group_frames = max(K, args.group // K * K)
    # one zeroed g2d buffer for every group of every step: each group's projection backward
    # reads its records and leaves them zero (no clear per group)
    # (the counting step's groups, on own lists, are not rounded to whole views)
    g2d_buf = torch.zeros(9 * w.gaussians.n * min(F, max(args.group, group_frames)), dtype=torch.float32,
                          device="cuda")

    # warm-up; the first warm-up step also counts the visited evaluations per group
    counts = {"fwd": 0, "bwd": 0, "blended": 0}

    def count_group(f0, st):
        a, b, c = eval_counts(st, t_min)
        counts["fwd"] += a
        counts["bwd"] += b
        counts["blended"] += c

    # the counting pass is an extra (untimed) step that also asks the forward for n_contrib
    def l1_step(gm, gr, shared=args.shared, **kw):
        return R.train_step(gm, w.cameras, luts, w.frames, targets, gr, args.group, w.opts, loss_acc=loss_acc,
                            shared=shared, g2d=g2d_buf, **kw)

    # Visits are counted on every frame's own list (the algorithm's work); a frame on a
    # shared list visits the same entries and drops the rest at staging.
    res = l1_step(g, grads, shared=False, on_group=count_group, want_contrib=True)
    log(f"bench: counting step loss {res.loss:.6f} entries {res.n_entries}")
    for k in range(args.warmup):
        res = l1_step(g, grads)
        log(f"bench: warm-up step {k} loss {res.loss:.6f}")

    # Timed steps.  The key lists are sized from the last warm-up step (the model does not
    # change between these steps, so neither do the lists), so a step needs no host
    # synchronisation: each one's loss and key-list flags are copied aside on the device
    # and read once after the loop, where an overflow would fail the run.  Step times are
    # the intervals between events recorded at the step boundaries.  Python's cycle
    # collector is paused (a collection stalls the host).
    cap = max(res.n_entries)
    timer = R.EventTimer()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    step_loss = torch.empty(args.steps, dtype=torch.float64, device="cuda")
    status = []
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record()
    for k in range(args.steps):
        res = l1_step(g, grads, timer=timer, capacity=cap, read_loss=False)
        step_loss[k:k + 1].copy_(loss_acc)
        status.append(res.status)
        marks[k + 1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gc.enable()
    for st in status:
        R.check_status(st, cap)
    step_ms = [marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps)]
    for k, v in enumerate(step_loss.cpu().tolist()):
        if k % 10 == 0 or k == args.steps - 1:
            log(f"bench: step {k} loss {v:.6f}")
    ms_step = dt * 1e3 / args.steps
    value = F * H * W * args.steps / dt / 1e6

    times = timer.totals_ms()
    per_step = {k: sum(v) / args.steps for k, v in times.items()}
    launches = {k: len(v) // args.steps for k, v in times.items()}

    # forward-only throughput (project + bin + blend for all frames, no backward), lists
    # sized as in the timed steps
    n_groups = (F + group_frames - 1) // group_frames
    fstat = torch.empty((args.steps, n_groups, 2), dtype=torch.int64, device="cuda")
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        for f0 in range(0, F, group_frames):
            fr = w.frames[f0:f0 + group_frames]
            cams = [w.cameras[c] for c, _ in (fr[::K] if args.shared else fr)]
            st = R.render(g, cams, [luts[t] for _, t in fr], w.opts, hits=False, shared=args.shared,
                          capacity=cap, status=fstat[k, f0 // group_frames])
            del st
    torch.cuda.synchronize()
    fwd_mpix = F * H * W * args.steps / (time.perf_counter() - t1) / 1e6
    gc.enable()
    R.check_status(fstat.view(-1, 2), cap)

    # the same training step with Blinn-Phong lighting attributes on every Gaussian
    lit_mpix = None
    if args.lit_steps > 0:
        import synth
        from paper_2504_13339_amd import veg as V
        sh = synth.random_shading(synth.rng_for(2, 90), w.gaussians.n)
        gl = V.Gaussians(g.means, g.log_scales, g.quats, g.scalars, g.weights,
                         **{k: torch.as_tensor(getattr(sh, k)).cuda() for k in V.LIGHTING})
        grads_l = R.Grads.zeros(gl)
        l1_step(gl, grads_l)
        lstat = []
        gc.collect()
        gc.disable()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for k in range(args.lit_steps):
            lstat.append(l1_step(gl, grads_l, capacity=cap, read_loss=False).status)
        torch.cuda.synchronize()
        lit_mpix = F * H * W * args.lit_steps / (time.perf_counter() - t2) / 1e6
        gc.enable()
        for st in lstat:
            R.check_status(st, cap)
        del grads_l, gl

    # a whole training iteration: the (1 - 0.2) L1 + 0.2 (1 - SSIM) loss, densification
    # statistics and the Adam update of every parameter tensor (this changes the model, so
    # it runs after the other measurements that use it)
    full = None
    if args.full_steps > 0:
        dens = R.DensifyStats.zeros(w.gaussians.n)
        lrs = [(g.means, 1.6e-4), (g.log_scales, 5e-3), (g.quats, 1e-3), (g.scalars, 2.5e-4)]
        if g.weights is not None:
            lrs.append((g.weights, 2.5e-2))
        opt = R.Adam(lrs)

        # Adam moves the model, so the lists may grow a little: 50% headroom, checked after
        fcap = int(cap * 1.5) + 4096

        def full_iter(timer=R.NO_TIMER):
            grads.zero_()
            r = R.train_step(g, w.cameras, luts, w.frames, targets, grads, args.group, w.opts, ssim_lambda=0.2,
                             shared=args.shared, capacity=fcap, g2d=g2d_buf,
                             loss_acc=loss_acc, densify=dens, timer=timer, read_loss=False)
            with timer("adam"):
                opt.step([grads.d_means, grads.d_log_scales, grads.d_quats, grads.d_scalars] +
                         ([grads.d_weights] if g.weights is not None else []))
            return r
        R.check_status(full_iter().status, fcap)
        ftimer = R.EventTimer()
        fst = []
        gc.collect()
        gc.disable()
        t3 = time.perf_counter()
        for k in range(args.full_steps):
            fst.append(full_iter(ftimer).status)
        torch.cuda.synchronize()
        fdt = time.perf_counter() - t3
        gc.enable()
        for st in fst:
            R.check_status(st, fcap)
        ft = {k: round(sum(v) / args.full_steps, 3) for k, v in ftimer.totals_ms().items()
              if k in ("image_loss", "project_bwd", "adam")}
        full = {"mpix_s": round(F * H * W * args.full_steps / fdt / 1e6, 2),
                "ms_per_step": round(fdt * 1e3 / args.full_steps, 3), "ssim_lambda": 0.2, "kernel_ms_per_step": ft}
        del dens, opt

    # roofline of the dominant kernel (blend forward or backward: VALU-bound)
    def blend_roof(name):
        visits = counts["bwd"] if name == "blend_bwd" else counts["fwd"]
        blend_flops = FLOPS_BLEND_BWD if name == "blend_bwd" else FLOPS_BLEND_FWD
        n_launch = launches[name]
        avg_ms = per_step[name] / n_launch
        flops = (visits * FLOPS_VISIT + counts["blended"] * blend_flops) / n_launch
        ach = flops / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "kernel": name, "achieved": round(ach, 3), "peak": round(VALU_PEAK_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(ach / VALU_PEAK_TFLOPS, 4), "traffic": profiled_traffic(name, args.shared),
                "traffic_unit": "HBM bytes per launch",
                "avg_launch_ms": round(avg_ms, 4), "visited_pairs_per_launch": visits // n_launch,
                "blended_pairs_per_launch": counts["blended"] // n_launch,
                "flops_per_launch": flops, "frac_of_packed_peak": round(ach / VALU_PACKED_PEAK_TFLOPS, 4)}
    dom = max(("blend_bwd", "blend_fwd"), key=lambda k: per_step.get(k, 0.0))
    roof = blend_roof(dom)
    other = blend_roof("blend_fwd" if dom == "blend_bwd" else "blend_bwd")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "step_ms_p10_p50_p90": [round(float(x), 3) for x in np.percentile(step_ms, [10, 50, 90])],
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "gaussians": w.gaussians.n, "frames": F, "width": W, "height": H,
                   "group": group_frames, "shared_views": bool(args.shared)},
        "fwd_mpix_s": round(fwd_mpix, 2),
        "lit_mpix_s": None if lit_mpix is None else round(lit_mpix, 2),
        "full_iteration": full,
        "geval_s": {"fwd": round(counts["fwd"] * args.steps / dt / 1e9, 3),
                    "bwd": round(counts["bwd"] * args.steps / dt / 1e9, 3)},
        "kernel_ms_per_step": {k: round(v, 3) for k, v in sorted(per_step.items(), key=lambda kv: -kv[1])},
        "roofline": roof,
        "roofline_other_blend": other,
    }
    if args.og_steps > 0:
        del grads, targets
        torch.cuda.empty_cache()
        log("bench: opacity-guided family")
        out["opacity_guided"] = opacity_guided_bench(args.og_steps)
        grads = targets = None
    if args.c1_steps > 0 or args.c4_steps > 0 or args.c4_serve > 0:
        del grads, targets
        grads = targets = None
        torch.cuda.empty_cache()
    if args.c1_steps > 0:
        log("bench: multi-TF workload step")
        out["multi_tf_step"] = workload_step_bench(1, args.c1_steps, shared=True)
    if args.c4_steps > 0:
        log("bench: stress workload step")
        out["stress_step"] = workload_step_bench(4, args.c4_steps, group=64, shared=True)
    if args.c4_serve > 0:
        log("bench: stress workload serving batch")
        out["stress_serve"] = stress_serve_bench(args.c4_serve)
    if args.serve_rates:
        del grads, targets
        torch.cuda.empty_cache()
        out["serve"] = serve_bench([float(r) for r in args.serve_rates.split(",")], args.serve_requests,
                                   args.serve_seconds)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
