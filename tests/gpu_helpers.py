"""Shared helpers for the GPU parity tests: run the HIP path and the oracle on the same
seeded inputs and line their outputs up."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import synth


def hip():
    from paper_2504_13339_amd import render as R
    from paper_2504_13339_amd import veg as V
    return V, R


def to_dev(g):
    V, _ = hip()
    return V.Gaussians.from_numpy(g)


def luts_to_dev(tfs):
    return [torch.as_tensor(np.ascontiguousarray(t, np.float32)).cuda() for t in tfs]


def image_pixels(img_chw):
    """[3,H,W] tensor -> [H*W,3] numpy in row-major pixel order (pixel index y*W + x)."""
    return img_chw.permute(1, 2, 0).reshape(-1, 3).detach().cpu().numpy().astype(np.float64)


def all_pixels(W, H):
    ys, xs = np.mgrid[0:H, 0:W]
    return np.stack([xs.reshape(-1), ys.reshape(-1)], 1)


def stratified_pixels(rng, fp, cam, n):
    """[n,2] (x, y) sample pixels of a frame, stratified so that the hottest tiles are in:
    all 256 pixels of the fullest tile (by the oracle's own tile occupancy), then half of
    the rest in tiles drawn with probability proportional to their list length, one random
    pixel each, and the other half uniform over the image."""
    occ = oracle.tile_occupancy(fp, cam)
    ty, tx = np.unravel_index(int(np.argmax(occ)), occ.shape)
    ys, xs = np.mgrid[16 * ty:min(16 * ty + 16, cam.height), 16 * tx:min(16 * tx + 16, cam.width)]
    hot = np.stack([xs.reshape(-1), ys.reshape(-1)], 1)
    rest = max(0, n - hot.shape[0])
    nw = rest // 2
    p = occ.reshape(-1).astype(np.float64)
    t = rng.choice(p.size, size=nw, p=p / p.sum()) if p.sum() > 0 else rng.integers(0, p.size, nw)
    wx = np.minimum((t % occ.shape[1]) * 16 + rng.integers(0, 16, nw), cam.width - 1)
    wy = np.minimum((t // occ.shape[1]) * 16 + rng.integers(0, 16, nw), cam.height - 1)
    ux = rng.integers(0, cam.width, rest - nw)
    uy = rng.integers(0, cam.height, rest - nw)
    px = np.concatenate([hot, np.stack([wx, wy], 1), np.stack([ux, uy], 1)])[:n]
    return px.astype(np.int32), int(occ.max())


# Largest fraction of compared pixels allowed a decision-margin flag: twice the worst
# fraction measured over every parity case of the GPU suite (0.0078, 1024 stratified pixels
# of a 1M-Gaussian frame, where the fullest tile's pixels carry many near-threshold
# evaluations).  Tests report theirs in the session summary (PARITY_STATS).
MAX_FLAG_FRAC = 1.6e-2

# One record per image comparison: (test id, pixels, unflagged max-abs, flagged fraction,
# largest slack, largest error on a flagged pixel); printed at the end of the session.
PARITY_STATS = []


def compare_image(gpu_px, res, tol=1e-4, max_flag_frac=MAX_FLAG_FRAC):
    """Every pixel: |gpu - oracle| <= tol + slack, where slack (from the oracle) bounds what
    near-threshold skip/stop decisions may legitimately change; pixels without a flag
    (slack below a quarter of tol) must meet tol itself.  The flagged fraction is bounded
    and returned; the comparison's figures are recorded in PARITY_STATS."""
    import os
    ref = res.color.detach().numpy()
    err = np.abs(gpu_px - ref).max(1)
    ok = ~res.flag
    assert ok.any()
    emax = err[ok].max()
    frac = float(res.flag.mean())
    eflag = float(err[res.flag].max()) if res.flag.any() else 0.0
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    PARITY_STATS.append((test, int(err.shape[0]), float(emax), frac, float(res.slack.max()), eflag))
    assert emax <= tol, f"unflagged max-abs {emax:.3g} > {tol}"
    worst = (err - (tol + res.slack)).max()
    assert worst <= 0, f"a flagged pixel exceeds tol + slack by {worst:.3g}"
    assert frac <= max_flag_frac, f"flagged fraction {frac:.3g}"
    return emax, frac


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
