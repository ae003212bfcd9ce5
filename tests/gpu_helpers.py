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


def compare_image(gpu_px, res, tol=1e-4, max_flag_frac=5e-2):
    """Every pixel: |gpu - oracle| <= tol + slack, where slack (from the oracle) bounds what
    near-threshold skip/stop decisions may legitimately change; pixels without a flag
    (slack below a quarter of tol) must meet tol itself.  The flagged fraction is bounded
    and returned."""
    ref = res.color.detach().numpy()
    err = np.abs(gpu_px - ref).max(1)
    ok = ~res.flag
    assert ok.any()
    emax = err[ok].max()
    assert emax <= tol, f"unflagged max-abs {emax:.3g} > {tol}"
    worst = (err - (tol + res.slack)).max()
    assert worst <= 0, f"a flagged pixel exceeds tol + slack by {worst:.3g}"
    frac = res.flag.mean()
    assert frac <= max_flag_frac, f"flagged fraction {frac:.3g}"
    return emax, frac


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
