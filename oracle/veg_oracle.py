"""CPU oracle for the VEG splatting rasterizer.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this module.  It shares no code with the HIP library and never calls it.

What the rasterizer computes (paper, section "Rendering of VEGs", Eq. 1): each Gaussian
carries position mu, scale S, rotation R and a scalar v (plus an optional trainable weight w).
The transfer function is applied first, per Gaussian: colour c = C(v), opacity
A = O(v) * w, with C and O linearly interpolated between the table's control points.
The 3D covariance R S S^T R^T is projected to a 2D screen covariance with Zwicker's EWA
linearisation; each pixel evaluates the 2D Gaussian at its centre and composites the
Gaussians front to back, C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j).  Tiling and
sorting only make this faster, so the oracle computes the definition by brute force.
Optionally each Gaussian also carries Blinn-Phong lighting attributes (normal, ambient,
diffuse and specular coefficients, shininess; Eq. 2-3), which turn C(v) into the shaded
colour under a headlight before compositing.

Three parts:

* O1 ``footprint_f32`` / ``key_list`` -- the integer decisions of the tiled renderer
  (cull, depth key, 16x16 tile rectangle, tile count, the sorted (tile, depth, index) key
  list and per-tile ranges).  A float decides each of these integers, so this part takes
  the decisions in the kernel's precision: float32 for covariance and extent, float64 for
  the projected centre, each operation rounded in the order stated next to the code (no
  fused multiply-add).  exp and log here are float32 functions built from Cody-Waite range
  reduction and truncated series (``exp32``, ``log32``).
* O2 ``project_f64`` / ``render_pixels`` -- float64 brute force: every kept Gaussian is
  evaluated at every requested pixel, in O1's depth order, with no tiles.  It also
  returns per-pixel decision-margin flags (pixels where an alpha-skip or a stop test lies
  within rounding distance of its threshold, so float32 and float64 may legitimately
  decide differently).
* O3 ``gradients`` -- the gradient of a linear functional of O2's image, by torch
  autograd in float64 on the CPU.
* ``vq_decode`` -- attributes stored as codebook indices, expanded into the model arrays.
* ``densify_plan`` / ``densify_apply`` -- adaptive density control: clone, split or prune
  decisions from the densification statistics and the model they produce.
* ``footprint_shared_f32`` -- the key list of frames that share a camera (several transfer
  functions over one view, as in opacity-guided training): the footprint at the largest
  opacity over the frames' tables, which contains each frame's own footprint.  The images
  and gradients of such frames are still O2 / O3 per frame.
* The training-loop neighbours of section "Training": ``l1_loss`` (the L1 term and its
  gradient), ``ssim_map`` / ``ssim_loss`` (the
  SSIM term of the image loss, Gaussian 11-tap window, float64, gradient by autograd),
  ``adam_step`` (the optimizer update) and ``densify_stats`` (per-Gaussian accumulated
  screen-space gradient norm and visibility count that drive densification).

Readings where the paper is silent (tile size, thresholds, footprint rule, low-pass,
guard band, near plane, stop semantics, knot derivative, light direction) follow the
renderer options and the headlight of the paper's evaluation (light and view direction =
the unit vector from the camera centre to the Gaussian):
alpha clamp 0.99, skip alpha < 1/255, stop once T < 1e-4 after blending the Gaussian that
crossed it, low-pass 0.3 px^2, guard 1.3, near 0.2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

__all__ = [
    "TILE", "QNORM2_MIN", "exp32", "log32", "footprint_f32", "footprint_shared_f32", "key_list", "tile_occupancy", "project_f64",
    "render_pixels", "render_image", "gradients", "quat_to_rot_f64", "OracleProjection",
    "depth_order", "frame_pairs", "l1_loss", "ssim_window_1d", "ssim_map", "ssim_loss", "adam_step", "densify_stats",
    "SSIM_C1", "SSIM_C2", "SSIM_WINDOW", "SSIM_SIGMA", "vq_decode", "densify_plan", "densify_apply",
    "KEEP", "CLONE", "SPLIT", "PRUNE", "SPLIT_SHRINK",
]

TILE = 16
QNORM2_MIN = np.float32(1e-24)   # |q|^2 below this (or non-finite) culls the Gaussian

_f = np.float32
_LOG2E = _f(float.fromhex("0x1.715476p+0"))
_LN2_HI = _f(0.693359375)                        # few significant bits: k*_LN2_HI is exact
_LN2_LO = _f(float.fromhex("-0x1.bd0106p-13"))   # ln2 - _LN2_HI
_SQRT2 = _f(float.fromhex("0x1.6a09e6p+0"))
_EXP_HI = _f(88.0)
_EXP_LO = _f(-87.0)


# ---------------------------------------------------------------------------------------
# O1: float32 exp / log (Cody & Waite range reduction + truncated series)
# ---------------------------------------------------------------------------------------

def exp32(x):
    """exp(x) in float32.  x = k ln2 + r with k = floor(x log2e + 1/2) and the reduction
    done in two parts (Cody & Waite); exp(r) by its Taylor series up to r^7 (Horner, with
    coefficients 1/n! rounded to float32); the result scaled by 2^k exactly.
    Domain clamps: x >= 88 gives +inf, x < -87 gives 0 (no subnormal results)."""
    x = np.asarray(x, dtype=np.float32)
    k = np.floor(x * _LOG2E + _f(0.5)).astype(np.float32)
    r = (x - k * _LN2_HI) - k * _LN2_LO
    p = _f(1.0) / _f(5040.0)
    for fac in (720.0, 120.0, 24.0, 6.0, 2.0, 1.0, 1.0):
        p = p * r + _f(1.0) / _f(fac)
    ki = np.clip(k, -126, 127).astype(np.int32)
    scale = ((ki + 127).astype(np.uint32) << np.uint32(23)).view(np.float32)
    out = (p * scale).astype(np.float32)
    out = np.where(x >= _EXP_HI, _f(np.inf), out)
    out = np.where(x < _EXP_LO, _f(0.0), out)
    return out.astype(np.float32)


def log32(x):
    """log(x) in float32 for positive normal x.  x = m 2^e with m in [sqrt(1/2), sqrt(2));
    log m = 2 atanh(u), u = (m-1)/(m+1), by the odd series up to u^9 (Horner in u^2,
    coefficients 1/(2j+1) rounded to float32); log x = e*ln2_hi + (e*ln2_lo + log m)."""
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32)
    e = (bits >> np.uint32(23)).astype(np.int32) - 127
    m = ((bits & np.uint32(0x7FFFFF)) | np.uint32(0x3F800000)).view(np.float32)
    big = m > _SQRT2
    m = np.where(big, m * _f(0.5), m).astype(np.float32)
    e = np.where(big, e + 1, e)
    u = (m - _f(1.0)) / (m + _f(1.0))
    u2 = u * u
    p = _f(1.0) / _f(9.0)
    for d in (7.0, 5.0, 3.0):
        p = p * u2 + _f(1.0) / _f(d)
    s = p * u2
    t = u + u * s
    logm = t + t
    ef = e.astype(np.float32)
    return (ef * _LN2_HI + (ef * _LN2_LO + logm)).astype(np.float32)


# ---------------------------------------------------------------------------------------
# O1: footprint in the kernel's precision
# ---------------------------------------------------------------------------------------

@dataclass
class Footprint:
    keep: np.ndarray        # [n] bool
    depth: np.ndarray       # [n] float32 camera-space z (computed for every Gaussian)
    depth_bits: np.ndarray  # [n] uint32
    rect: np.ndarray        # [n,4] int32 tile rectangle (x0, y0, x1, y1), inclusive
    count: np.ndarray       # [n] int64 tiles covered (0 when culled)
    mx: np.ndarray          # [n] float64 projected centre
    my: np.ndarray
    ex: np.ndarray          # [n] float32 half extents of the alpha >= alpha_min ellipse
    ey: np.ndarray
    A: Optional[np.ndarray] = None   # [n] float32 peak opacity O(v) w (before the cull)
    cov: Optional[np.ndarray] = None  # [n,3] float32 screen covariance (S00, S01, S11) as rounded above
    det: Optional[np.ndarray] = None  # [n] float32 determinant of that covariance, as computed above


def _finite_rows(*arrs):
    ok = None
    for a in arrs:
        if a is None:
            continue
        a2 = a.reshape(a.shape[0], -1)
        r = np.isfinite(a2).all(axis=1)
        ok = r if ok is None else ok & r
    return ok


def footprint_f32(g, cam, lut, opts) -> Footprint:
    """Cull, depth key and tile rectangle per Gaussian, in the kernel's precision.

    Order of operations (each line rounds once, no fused multiply-add):
      t     = ((V0 mu_x + V1 mu_y) + V2 mu_z) + V3 per row, float64
      depth = float32(t_z); cull unless depth > near
      xn = t_x / t_z, yn = t_y / t_z, mx = fx xn + cx, my = fy yn + cy, float64
      TF:   vc = clamp(v,0,1); t = vc (K-1); i = min(floor t, K-2); f = t - i;
            X = L[i] (1-f) + L[i+1] f; A = O w
      cull unless A >= alpha_min, unless |q|^2 >= 1e-24
      q normalised by 1/sqrt(|q|^2); R(q); s = exp32(log s)
      Q = Vr R; P = Q diag(s); J from float32 depth and clamped float32 xn, yn;
      G = J P; S = G G^T + lowpass I; det = |G0 x G1|^2 + lowpass (|G0|^2 + |G1|^2) + lowpass^2
      (cull unless > 0)
      tau = 2 log32(A / alpha_min); ex = sqrt(tau S00), ey = sqrt(tau S11)
      pixel range x in [ceil(mx - ex - 0.5), floor(mx + ex - 0.5)] (float64), clipped to the
      image; tile rectangle = pixel range // 16; count = its area.
    """
    f32 = np.float32
    n = g.means.shape[0]
    V = np.asarray(cam.view, np.float32).reshape(3, 4)
    Vd = V.astype(np.float64)
    mu = g.means.astype(np.float64)
    t = [((Vd[r, 0] * mu[:, 0] + Vd[r, 1] * mu[:, 1]) + Vd[r, 2] * mu[:, 2]) + Vd[r, 3] for r in range(3)]
    tx, ty, tz = t
    with np.errstate(all="ignore"):
        depth = tz.astype(np.float32)
        fx, fy, cx, cy = (f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy))
        W, H = int(cam.width), int(cam.height)
        xn = tx / tz
        yn = ty / tz
        mx = float(fx) * xn + float(cx)
        my = float(fy) * yn + float(cy)

        sh = getattr(g, "shading", None)
        finite = _finite_rows(g.means, g.log_scales, g.quats, g.scalars[:, None],
                              None if g.weights is None else g.weights[:, None])
        if sh is not None:
            finite = finite & _finite_rows(sh.normals, sh.k_ambient[:, None], sh.k_diffuse[:, None],
                                           sh.k_specular[:, None], sh.shininess[:, None])
            nn = np.asarray(sh.normals, np.float32)
            nrm2 = ((nn[:, 0] * nn[:, 0] + nn[:, 1] * nn[:, 1]) + nn[:, 2] * nn[:, 2])
            finite = finite & (nrm2 >= QNORM2_MIN)
        # transfer function
        K = lut.shape[0]
        v = g.scalars.astype(np.float32)
        v = np.where(np.isfinite(v), v, f32(0))
        vc = np.where(v < f32(0), f32(0), np.where(v > f32(1), f32(1), v)).astype(np.float32)
        tpos = vc * f32(K - 1)
        i = np.minimum(np.floor(tpos).astype(np.int64), K - 2)
        fr = tpos - i.astype(np.float32)
        om = f32(1) - fr
        O = lut[i, 3] * om + lut[i + 1, 3] * fr
        A = O if g.weights is None else O * g.weights.astype(np.float32)

        q = g.quats.astype(np.float32)
        n2 = ((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3]
        inv = f32(1) / np.sqrt(n2)
        w_, x_, y_, z_ = (q[:, 0] * inv, q[:, 1] * inv, q[:, 2] * inv, q[:, 3] * inv)
        two = f32(2)
        one = f32(1)
        R = np.empty((n, 3, 3), np.float32)
        R[:, 0, 0] = one - two * (y_ * y_ + z_ * z_)
        R[:, 0, 1] = two * (x_ * y_ - w_ * z_)
        R[:, 0, 2] = two * (x_ * z_ + w_ * y_)
        R[:, 1, 0] = two * (x_ * y_ + w_ * z_)
        R[:, 1, 1] = one - two * (x_ * x_ + z_ * z_)
        R[:, 1, 2] = two * (y_ * z_ - w_ * x_)
        R[:, 2, 0] = two * (x_ * z_ - w_ * y_)
        R[:, 2, 1] = two * (y_ * z_ + w_ * x_)
        R[:, 2, 2] = one - two * (x_ * x_ + y_ * y_)
        s = exp32(g.log_scales.astype(np.float32))

        Q = np.empty((n, 3, 3), np.float32)
        for j in range(3):
            for k in range(3):
                Q[:, j, k] = (V[j, 0] * R[:, 0, k] + V[j, 1] * R[:, 1, k]) + V[j, 2] * R[:, 2, k]
        P = Q * s[:, None, :]

        limx = f32(opts["guard"]) * ((f32(0.5) * f32(W)) / fx)
        limy = f32(opts["guard"]) * ((f32(0.5) * f32(H)) / fy)
        xnf = xn.astype(np.float32)
        ynf = yn.astype(np.float32)
        xc = np.minimum(np.maximum(xnf, -limx), limx)
        yc = np.minimum(np.maximum(ynf, -limy), limy)
        J00 = fx / depth
        J02 = -(fx * xc) / depth
        J11 = fy / depth
        J12 = -(fy * yc) / depth
        G0 = J00[:, None] * P[:, 0, :] + J02[:, None] * P[:, 2, :]
        G1 = J11[:, None] * P[:, 1, :] + J12[:, None] * P[:, 2, :]
        lp = f32(opts["lowpass"])
        g00 = (G0[:, 0] * G0[:, 0] + G0[:, 1] * G0[:, 1]) + G0[:, 2] * G0[:, 2]
        g11 = (G1[:, 0] * G1[:, 0] + G1[:, 1] * G1[:, 1]) + G1[:, 2] * G1[:, 2]
        S00 = g00 + lp
        S01 = (G0[:, 0] * G1[:, 0] + G0[:, 1] * G1[:, 1]) + G0[:, 2] * G1[:, 2]
        S11 = g11 + lp
        # det(S) = |G0 x G1|^2 + lp (|G0|^2 + |G1|^2) + lp^2 (Cauchy-Binet), no cancellation
        x0 = G0[:, 1] * G1[:, 2] - G0[:, 2] * G1[:, 1]
        x1 = G0[:, 2] * G1[:, 0] - G0[:, 0] * G1[:, 2]
        x2 = G0[:, 0] * G1[:, 1] - G0[:, 1] * G1[:, 0]
        det = (((x0 * x0 + x1 * x1) + x2 * x2) + lp * (g00 + g11)) + lp * lp

        amin = f32(opts["alpha_min"])
        keep = finite & (depth > f32(opts["near_z"])) & (A >= amin) & (n2 >= QNORM2_MIN) & (det > f32(0))
        ratio = np.where(keep, A / amin, f32(1))
        tau = two * log32(ratio)
        ex = np.sqrt(tau * S00).astype(np.float32)
        ey = np.sqrt(tau * S11).astype(np.float32)
        xlo = np.ceil((mx - ex.astype(np.float64)) - 0.5)
        xhi = np.floor((mx + ex.astype(np.float64)) - 0.5)
        ylo = np.ceil((my - ey.astype(np.float64)) - 0.5)
        yhi = np.floor((my + ey.astype(np.float64)) - 0.5)
        xlo = np.maximum(xlo, 0.0)
        ylo = np.maximum(ylo, 0.0)
        xhi = np.minimum(xhi, float(W - 1))
        yhi = np.minimum(yhi, float(H - 1))
        keep = keep & (xlo <= xhi) & (ylo <= yhi)
    rect = np.zeros((n, 4), np.int32)
    kk = keep
    rect[kk, 0] = xlo[kk].astype(np.int64) // TILE
    rect[kk, 1] = ylo[kk].astype(np.int64) // TILE
    rect[kk, 2] = xhi[kk].astype(np.int64) // TILE
    rect[kk, 3] = yhi[kk].astype(np.int64) // TILE
    count = np.where(kk, (rect[:, 2] - rect[:, 0] + 1).astype(np.int64) * (rect[:, 3] - rect[:, 1] + 1), 0)
    return Footprint(keep=keep, depth=depth, depth_bits=depth.view(np.uint32).copy(), rect=rect,
                     count=count, mx=mx, my=my, ex=ex, ey=ey, A=np.asarray(A, np.float32),
                     cov=np.stack([S00, S01, S11], 1).astype(np.float32), det=np.asarray(det, np.float32))


def footprint_shared_f32(g, cam, luts, opts) -> Footprint:
    """Footprint of one camera whose frames (one per table in ``luts``) share a key list.

    Everything in ``footprint_f32`` except A is independent of the transfer function, and
    the ellipse where A exp(-sigma) >= alpha_min grows with A, so the frames' footprints
    are all contained in the footprint at the largest A over the tables.  The shared list
    is built from exactly that footprint: per Gaussian, the fields of the table with the
    largest A (non-finite A never wins; ties give identical fields).  A Gaussian is in the
    list when that table keeps it.  A frame blends only the Gaussians its own footprint
    keeps, and skips pixel by pixel what its own A puts below alpha_min, so every frame's
    image is the one of its own footprint."""
    fps = [footprint_f32(g, cam, lut, opts) for lut in luts]
    with np.errstate(invalid="ignore"):
        a = np.stack([np.where(np.isfinite(fp.A), fp.A, -np.inf) for fp in fps])
    k = np.argmax(a, axis=0)
    idx = np.arange(k.shape[0])

    def pick(name):
        return np.stack([getattr(fp, name) for fp in fps])[k, idx]
    return Footprint(keep=pick("keep"), depth=fps[0].depth, depth_bits=fps[0].depth_bits, rect=pick("rect"),
                     count=pick("count"), mx=fps[0].mx, my=fps[0].my, ex=pick("ex"), ey=pick("ey"), A=pick("A"),
                     cov=fps[0].cov, det=fps[0].det)


def tiles_of(cam):
    return (cam.width + TILE - 1) // TILE, (cam.height + TILE - 1) // TILE


def key_list(fps, cams):
    """Sorted key list over several frames.

    ``fps[f]`` is frame f's Footprint (all frames over the same n Gaussians), ``cams[f]``
    its camera.  Global tile id = tile_base[f] + ty * tiles_x + tx with tile_base the
    prefix sum of the frames' tile counts; pair id = f * n + i.  Entries are sorted by
    (global tile, depth bits, pair id).  Returns (tile_ids, depth_bits, pair_ids) of the
    sorted list and ranges[total_tiles, 2] = [start, end)."""
    n = fps[0].keep.shape[0]
    tiles, depths, pairs = [], [], []
    tile_base = 0
    bases = []
    for f, (fp, cam) in enumerate(zip(fps, cams)):
        tx_n, ty_n = tiles_of(cam)
        bases.append(tile_base)
        idx = np.nonzero(fp.count > 0)[0]
        cnt = fp.count[idx]
        rep = np.repeat(idx, cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        local = np.arange(rep.shape[0], dtype=np.int64) - start
        r = fp.rect[rep]
        wdt = (r[:, 2] - r[:, 0] + 1).astype(np.int64)
        txs = r[:, 0] + local % wdt
        tys = r[:, 1] + local // wdt
        tiles.append(tile_base + tys * tx_n + txs)
        depths.append(fp.depth_bits[rep])
        pairs.append(f * n + rep)
        tile_base += tx_n * ty_n
    tiles = np.concatenate(tiles) if tiles else np.zeros(0, np.int64)
    depths = np.concatenate(depths) if depths else np.zeros(0, np.uint32)
    pairs = np.concatenate(pairs) if pairs else np.zeros(0, np.int64)
    order = np.lexsort((pairs, depths, tiles))
    tiles, depths, pairs = tiles[order], depths[order], pairs[order]
    ranges = np.zeros((tile_base, 2), np.int64)
    if tiles.shape[0]:
        starts = np.searchsorted(tiles, np.arange(tile_base), side="left")
        ends = np.searchsorted(tiles, np.arange(tile_base), side="right")
        ranges[:, 0] = np.where(ends > starts, starts, 0)
        ranges[:, 1] = np.where(ends > starts, ends, 0)
    return tiles, depths, pairs, ranges, np.asarray(bases, np.int64)


def tile_occupancy(fp: Footprint, cam) -> np.ndarray:
    """[tiles_y, tiles_x] number of Gaussians whose tile rectangle covers each tile (the
    length of each tile's key list), by a 2D difference array over the rectangles."""
    tx_n, ty_n = tiles_of(cam)
    diff = np.zeros((ty_n + 1, tx_n + 1), np.int64)
    r = fp.rect[fp.count > 0].astype(np.int64)
    np.add.at(diff, (r[:, 1], r[:, 0]), 1)
    np.add.at(diff, (r[:, 1], r[:, 2] + 1), -1)
    np.add.at(diff, (r[:, 3] + 1, r[:, 0]), -1)
    np.add.at(diff, (r[:, 3] + 1, r[:, 2] + 1), 1)
    return diff.cumsum(0).cumsum(1)[:ty_n, :tx_n]


def frame_pairs(n, n_frames):
    return n * n_frames


def depth_order(fp: Footprint, kept: np.ndarray) -> np.ndarray:
    """Indices of ``kept`` Gaussians ordered front to back by (float32 depth bits, index)."""
    idx = np.nonzero(kept)[0]
    return idx[np.lexsort((idx, fp.depth_bits[idx]))]


# ---------------------------------------------------------------------------------------
# O2: float64 brute force
# ---------------------------------------------------------------------------------------

def quat_to_rot_f64(q):
    """Rotation matrix of unit quaternions (w, x, y, z), [n,4] -> [n,3,3] (torch)."""
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


@dataclass
class OracleProjection:
    mean2d: torch.Tensor   # [n,2] pixel coordinates of the projected centre
    conic: torch.Tensor    # [n,3] (a, b, c) of the inverse 2D covariance [[a,b],[b,c]]
    cov2d: torch.Tensor    # [n,3] (S00, S01, S11)
    rgb: torch.Tensor      # [n,3] C(v)
    A: torch.Tensor        # [n]   O(v) * w
    depth: torch.Tensor    # [n]   camera-space z
    kept: np.ndarray       # [n]   bool (float64 decisions)


def _t64(a):
    if isinstance(a, torch.Tensor):
        return a.to(torch.float64)
    return torch.as_tensor(np.asarray(a, np.float64))


def project_f64(means, log_scales, quats, scalars, weights, cam, lut, opts, shading=None) -> OracleProjection:
    """Per-Gaussian quantities in float64 (torch, differentiable).

    TF first (paper: colour and opacity from the transfer function before rasterizing;
    alpha = O(v) w; linear interpolation between control points), then the 3D covariance
    Sigma = R S S^T R^T, then Zwicker's EWA projection Sigma' = J W Sigma W^T J^T + lowpass I
    with J the Jacobian of the pinhole map at the camera-space centre (its x/z, y/z clamped
    to the guard band), conic = Sigma'^-1.

    ``shading`` = (normals, k_ambient, k_diffuse, k_specular, shininess) applies the
    Blinn-Phong colour of Eq. 2-3 with a headlight: light and view direction both the unit
    vector l from the camera centre to the Gaussian, so the half vector is l and, with
    s = |n^ . l| (n^ the normalised normal),
        c = C(v) (k_a + k_d s) + k_s s^beta (white),  the specular term 0 when s = 0.
    """
    means, log_scales, quats, scalars = map(_t64, (means, log_scales, quats, scalars))
    weights = None if weights is None else _t64(weights)
    lut = _t64(lut)
    V = _t64(np.asarray(cam.view, np.float32)).reshape(3, 4)
    Wr, b = V[:, :3], V[:, 3]
    fx, fy, cx, cy = (float(np.float32(cam.fx)), float(np.float32(cam.fy)),
                      float(np.float32(cam.cx)), float(np.float32(cam.cy)))
    t = means @ Wr.T + b
    tx, ty, tz = t.unbind(-1)

    K = lut.shape[0]
    vc = scalars.clamp(0.0, 1.0)
    tpos = vc * (K - 1)
    with torch.no_grad():
        i = torch.floor(tpos).clamp(max=K - 2).long()
    fr = (tpos - i.to(tpos.dtype))[:, None]
    rgba = lut[i] * (1 - fr) + lut[i + 1] * fr
    rgb = rgba[:, :3]
    A = rgba[:, 3] if weights is None else rgba[:, 3] * weights
    if shading is not None:
        nrm, k_a, k_d, k_s, beta = map(_t64, shading)
        campos = -(Wr.T @ b)                                # camera centre: W campos + b = 0
        dvec = means - campos
        ldir = dvec / torch.sqrt((dvec * dvec).sum(-1))[:, None]
        nhat = nrm / torch.sqrt((nrm * nrm).sum(-1))[:, None]
        sabs = (nhat * ldir).sum(-1).abs()
        pos = sabs > 0
        spec = torch.where(pos, k_s * torch.where(pos, sabs, torch.ones_like(sabs)) ** beta, torch.zeros_like(sabs))
        rgb = rgb * (k_a + k_d * sabs)[:, None] + spec[:, None]

    qn2 = (quats * quats).sum(-1)
    qhat = quats / torch.sqrt(qn2)[:, None]
    R = quat_to_rot_f64(qhat)
    s2 = torch.exp(2 * log_scales)
    Sigma = (R * s2[:, None, :]) @ R.transpose(-1, -2)
    Sigma_c = Wr @ Sigma @ Wr.T

    W_img, H_img = int(cam.width), int(cam.height)
    limx = float(opts["guard"]) * (0.5 * W_img / fx)
    limy = float(opts["guard"]) * (0.5 * H_img / fy)
    xn, yn = tx / tz, ty / tz
    xc, yc = xn.clamp(-limx, limx), yn.clamp(-limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * xc / tz], -1),
                     torch.stack([zero, fy / tz, -fy * yc / tz], -1)], -2)
    S2 = J @ Sigma_c @ J.transpose(-1, -2) + float(opts["lowpass"]) * torch.eye(2, dtype=torch.float64)
    S00, S01, S11 = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
    det = S00 * S11 - S01 * S01
    conic = torch.stack([S11 / det, -S01 / det, S00 / det], -1)
    mean2d = torch.stack([fx * xn + cx, fy * yn + cy], -1)

    with torch.no_grad():
        def fin(x):
            return torch.isfinite(x.reshape(x.shape[0], -1)).all(1)
        ok = fin(means) & fin(log_scales) & fin(quats) & torch.isfinite(scalars)
        if weights is not None:
            ok &= torch.isfinite(weights)
        if shading is not None:
            ok &= fin(nrm) & torch.isfinite(k_a) & torch.isfinite(k_d) & torch.isfinite(k_s) & torch.isfinite(beta)
            ok &= (nrm * nrm).sum(-1) >= float(QNORM2_MIN)
        amin = float(np.float32(opts["alpha_min"]))
        ok &= (tz > float(np.float32(opts["near_z"]))) & (A >= amin) & (qn2 >= float(QNORM2_MIN)) & (det > 0)
        ok &= torch.isfinite(conic).all(1) & torch.isfinite(mean2d).all(1)
    return OracleProjection(mean2d=mean2d, conic=conic, cov2d=torch.stack([S00, S01, S11], -1),
                            rgb=rgb, A=A, depth=tz, kept=ok.numpy().copy())


@dataclass
class PixelResult:
    color: torch.Tensor      # [P,3] C + T bg
    T: torch.Tensor          # [P]   final transmittance
    last: np.ndarray         # [P]   position in ``order`` of the last blended Gaussian, -1 if none
    n_eval: np.ndarray       # [P]   Gaussians visited up to the stop (brute-force count)
    flag: np.ndarray         # [P]   image decision-margin flag (slack >= skip_impact)
    flag_grad: np.ndarray    # [P]   any near-threshold decision (skip, stop, clamp): gradient tests
    slack: np.ndarray        # [P]   bound on how far float32 may legitimately differ from float64
                             #       through near-threshold decisions (sum of their impact bounds)


# Unit roundoff of float32 and the safety factor of the per-evaluation error bound below.
U32 = 2.0 ** -24
ERR_COEF = 32.0


def render_pixels(proj: OracleProjection, order: np.ndarray, pixels: np.ndarray, opts,
                  bg=(0.0, 0.0, 0.0), batch: int = 0, err_coef: float = ERR_COEF,
                  skip_impact=2.5e-5, t_min: Optional[float] = None) -> PixelResult:
    """Front-to-back compositing (Eq. 1) at pixel centres (x+0.5, y+0.5), brute force.

    For each pixel and each Gaussian of ``order`` (front to back):
      sigma = 1/2 d^T conic d with d = p - mean2d; a = A exp(-sigma);
      a < alpha_min: skipped; otherwise alpha = min(alpha_clamp, a), C += c alpha T,
      T *= 1 - alpha, and if T < t_min the pixel stops (the Gaussian that crossed the
      threshold is blended).  Output C + T bg.

    Decision margins.  The tiled float32 renderer decides the same skips, stops and clamps
    from float32 values, so a decision may flip where the float64 value lies within the
    float32 evaluation's error of its threshold.  That error is bounded per evaluation
    (pair of Gaussian and pixel): to first order, with u = 2^-24,
      |ln a_32 - ln a_64| <= eps = err_coef u (1 + |ln A| + (|y_0| sqrt(S00) + |y_1| sqrt(S11))^2),
    y = conic d.  The last term is the propagation of a relative perturbation of order u in
    every entry of the float32 screen covariance S (from the chain R, s, W, J, S = G G^T +
    lowpass I) through conic = S^-1: d(d^T S^-1 d) = -y^T dS y with |dS_ij| <= c u
    sqrt(S_ii S_jj); it grows with the ellipse's elongation.  |ln A| covers the table
    lookup and the log2 of A, the 1 the remaining roundings of the exponent (centre offset,
    quadratic form).  err_coef = 32 is twice the largest ratio of the observed float32
    error to (1 + |ln A| + that term) over 675k evaluations near the threshold on the 1k-,
    200k- and 1M-Gaussian workloads, emulating the kernel's op order.
      skip:  |ln(a / alpha_min)| < eps.  A flip moves the pixel by at most
             alpha_min T_before max|c - S| <= alpha_min T_before (1 + eps) (colours and
             background in [0, 1]).
      stop:  the float32 transmittance after k blends carries a relative error of at most
             m_k = sum over the blends j <= k of (u + alpha_j / (1 - alpha_j) (eps_j + 2u))
             (an unclamped alpha inherits a's error, the exp2 rounds once, the update
             T - alpha T rounds once), so |ln(T_k / t_min)| < m_k may flip.  Then one side
             blends the Gaussians the other drops until its T falls below t_min, which
             moves the pixel by at most (m_k + alpha_max_after) T_k (1 + m_k), with
             alpha_max_after the largest alpha after that point.
      clamp: |ln(a / alpha_clamp)| < eps (only the gradient is discontinuous there).
    ``slack`` sums the image bounds per pixel; ``flag`` marks pixels whose slack reaches
    ``skip_impact``; ``flag_grad`` marks every pixel with any near-threshold skip, stop or
    clamp decision (where the gradient is discontinuous).
    """
    aclamp = float(np.float32(opts["alpha_clamp"]))
    amin = float(np.float32(opts["alpha_min"]))
    tmin = float(np.float32(opts["t_min"] if t_min is None else t_min))
    order_t = torch.as_tensor(np.asarray(order, np.int64))
    mu = proj.mean2d[order_t]
    con = proj.conic[order_t]
    rgb = proj.rgb[order_t]
    A = proj.A[order_t]
    M = int(order_t.shape[0])
    P = int(pixels.shape[0])
    bgt = torch.as_tensor(np.asarray(bg, np.float64))
    if batch <= 0:
        batch = max(1, min(P, (1 << 23) // max(M, 1)))
    cols, Ts, lasts, nevs, flags, gflags, slacks = [], [], [], [], [], [], []
    with torch.no_grad():
        cov = proj.cov2d[order_t].detach()
        sq00 = torch.sqrt(cov[:, 0].clamp(min=0.0))
        sq11 = torch.sqrt(cov[:, 2].clamp(min=0.0))
        conD = con.detach()
        muD = mu.detach()
        with np.errstate(divide="ignore"):
            lnA_all = torch.log(A.detach())
        ln_amin, ln_aclamp = math.log(amin), math.log(aclamp)
        ln_tmin = math.log(tmin) if tmin > 0 else -math.inf
    for s in range(0, P, batch):
        pix = torch.as_tensor(np.asarray(pixels[s:s + batch], np.float64))
        Pb = pix.shape[0]
        if M == 0:
            cols.append(bgt.expand(Pb, 3).clone())
            Ts.append(torch.ones(Pb, dtype=torch.float64))
            lasts.append(np.full(Pb, -1))
            nevs.append(np.zeros(Pb, np.int64))
            flags.append(np.zeros(Pb, bool))
            gflags.append(np.zeros(Pb, bool))
            slacks.append(np.zeros(Pb))
            continue
        # Every Gaussian at every pixel.  A Gaussian with a below alpha_min has alpha = 0
        # and multiplies T by exactly 1, so the compositing below runs over each pixel's
        # candidates in depth order: every Gaussian with ln a >= ln alpha_min - 1/2 (a
        # superset of the blended ones and of those within any decision margin), padded
        # with alpha = 0; a is evaluated again, differentiably, for the candidates.
        with torch.no_grad():
            dxD = (pix[:, 0:1] + 0.5) - muD[None, :, 0]
            dyD = (pix[:, 1:2] + 0.5) - muD[None, :, 1]
            lnaD = lnA_all[None, :] - 0.5 * (conD[None, :, 0] * dxD * dxD + 2.0 * conD[None, :, 1] * dxD * dyD +
                                             conD[None, :, 2] * dyD * dyD)
            cand = lnaD >= ln_amin - 0.5
            del dxD, dyD, lnaD
            cnt = cand.sum(1)
            Kp = max(int(cnt.max()), 1)
            rows, colsi = cand.nonzero(as_tuple=True)
            del cand
            pos = torch.arange(rows.shape[0]) - (torch.cumsum(cnt, 0) - cnt)[rows]
            valid = torch.zeros((Pb, Kp), dtype=torch.bool)
            valid[rows, pos] = True
            gidx = torch.full((Pb, Kp), -1, dtype=torch.int64)
            gidx[rows, pos] = colsi
        dxf = (pix[rows, 0] + 0.5) - mu[colsi, 0]
        dyf = (pix[rows, 1] + 0.5) - mu[colsi, 1]
        cf = con[colsi]
        sigf = 0.5 * (cf[:, 0] * dxf * dxf + 2.0 * cf[:, 1] * dxf * dyf + cf[:, 2] * dyf * dyf)
        ac = torch.zeros((Pb, Kp), dtype=torch.float64).index_put((rows, pos), A[colsi] * torch.exp(-sigf))
        rgbc = torch.zeros((Pb, Kp, 3), dtype=torch.float64).index_put((rows, pos), rgb[colsi])
        blend = (ac >= amin) & valid
        alpha = torch.where(blend, torch.where(ac < aclamp, ac, torch.full_like(ac, aclamp)), torch.zeros_like(ac))
        T_incl = torch.cumprod(1.0 - alpha, dim=1)
        with torch.no_grad():
            stop = T_incl < tmin
            has_stop = stop.any(1)
            k = torch.where(has_stop, stop.to(torch.int8).argmax(1), torch.full_like(has_stop, Kp - 1, dtype=torch.int64))
            ar = torch.arange(Kp)[None, :]
            upto = ar <= k[:, None]
        T_excl = torch.cat([torch.ones_like(T_incl[:, :1]), T_incl[:, :-1]], dim=1)
        wgt = alpha * T_excl * upto.to(alpha.dtype)
        C = (wgt[:, :, None] * rgbc).sum(1)
        T_fin = T_incl.gather(1, k[:, None])[:, 0]
        cols.append(C + T_fin[:, None] * bgt[None, :])
        Ts.append(T_fin)
        with torch.no_grad():
            bl = blend & upto
            last_c = torch.where(bl, gidx, torch.full_like(gidx, -1)).max(1).values
            lasts.append(last_c.numpy())
            stop_col = gidx.gather(1, k[:, None])[:, 0]
            nevs.append(torch.where(has_stop, stop_col + 1, torch.full_like(stop_col, M)).numpy())
            ad = ac.detach()
            al = alpha.detach()
            Ti, Te = T_incl.detach(), T_excl.detach()
            g0 = gidx.clamp(min=0)
            dxc = torch.zeros((Pb, Kp), dtype=torch.float64)
            dyc = torch.zeros((Pb, Kp), dtype=torch.float64)
            dxc[rows, pos] = dxf.detach()
            dyc[rows, pos] = dyf.detach()
            # per-evaluation bound on the float32 error of ln a
            y0 = conD[g0, 0] * dxc + conD[g0, 1] * dyc
            y1 = conD[g0, 1] * dxc + conD[g0, 2] * dyc
            lnA = torch.log(A.detach()[g0])
            eps = err_coef * U32 * (1.0 + lnA.abs() + (y0.abs() * sq00[g0] + y1.abs() * sq11[g0]) ** 2)
            ln_a = torch.log(ad.clamp(min=1e-300))
            near_skip = ((ln_a - ln_amin).abs() < eps) & upto & valid
            unclamped = ad < aclamp
            step = torch.where(bl, U32 + torch.where(unclamped, al / (1.0 - al), torch.zeros_like(al)) * (eps + 2 * U32),
                               torch.zeros_like(al))
            m_t = torch.cumsum(step, dim=1)
            near_stop = ((torch.log(Ti) - ln_tmin).abs() < m_t) & bl
            amax_from = torch.flip(torch.cummax(torch.flip(al, [1]), 1).values, [1])
            amax_after = torch.cat([amax_from[:, 1:], torch.zeros_like(amax_from[:, :1])], 1)
            slack = (near_skip.to(al.dtype) * (amin * (1 + eps)) * Te).sum(1) + \
                    (near_stop.to(al.dtype) * (m_t + amax_after) * Ti * (1 + m_t)).sum(1)
            slacks.append(slack.numpy())
            flags.append((slack >= skip_impact).numpy())
            near_clamp = ((ln_a - ln_aclamp).abs() < eps) & bl
            gflags.append((near_skip.any(1) | near_stop.any(1) | near_clamp.any(1)).numpy())
    return PixelResult(color=torch.cat(cols, 0), T=torch.cat(Ts, 0), last=np.concatenate(lasts),
                       n_eval=np.concatenate(nevs), flag=np.concatenate(flags),
                       flag_grad=np.concatenate(gflags), slack=np.concatenate(slacks))


def _shading_arrays(g):
    sh = getattr(g, "shading", None)
    return None if sh is None else (sh.normals, sh.k_ambient, sh.k_diffuse, sh.k_specular, sh.shininess)


def render_image(g, cam, lut, opts, pixels=None, bg=None, t_min=None, **kw):
    """Convenience: O1 depth order + O2 for one frame.  Returns (PixelResult, proj, order, fp)."""
    fp = footprint_f32(g, cam, lut, opts)
    proj = project_f64(g.means, g.log_scales, g.quats, g.scalars, g.weights, cam, lut, opts,
                       shading=_shading_arrays(g))
    order = depth_order(fp, proj.kept)
    if pixels is None:
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        pixels = np.stack([xs.reshape(-1), ys.reshape(-1)], 1)
    bg = opts.get("bg", (0.0, 0.0, 0.0)) if bg is None else bg
    res = render_pixels(proj, order, pixels, opts, bg=bg, t_min=t_min, **kw)
    return res, proj, order, fp


# ---------------------------------------------------------------------------------------
# O3: gradients by autograd through O2
# ---------------------------------------------------------------------------------------

@dataclass
class OracleGrads:
    d_means: np.ndarray
    d_log_scales: np.ndarray
    d_quats: np.ndarray
    d_scalars: np.ndarray
    d_weights: Optional[np.ndarray]
    # per-Gaussian screen-space gradients (the blend adjoint's output)
    d_mean2d: np.ndarray
    d_conic: np.ndarray
    d_rgb: np.ndarray
    d_A: np.ndarray
    loss: float
    # lighting attributes (None for an unshaded model)
    d_normals: Optional[np.ndarray] = None
    d_k_ambient: Optional[np.ndarray] = None
    d_k_diffuse: Optional[np.ndarray] = None
    d_k_specular: Optional[np.ndarray] = None
    d_shininess: Optional[np.ndarray] = None


def gradients(g, cam, lut, opts, d_color, pixels=None, bg=None, batch: int = 0) -> OracleGrads:
    """Gradient of L = sum_p sum_ch d_color[p,ch] * image[p,ch] w.r.t. every Gaussian
    parameter (float64 autograd through ``project_f64`` and ``render_pixels``).

    The screen-space gradients are taken w.r.t. mean2d, the conic (a, b, c) as it enters
    sigma = 1/2 (a dx^2 + 2 b dx dy + c dy^2), rgb and A."""
    fp = footprint_f32(g, cam, lut, opts)
    leaves = [torch.tensor(np.asarray(x, np.float64), requires_grad=True)
              for x in (g.means, g.log_scales, g.quats, g.scalars)]
    w = None if g.weights is None else torch.tensor(np.asarray(g.weights, np.float64), requires_grad=True)
    sh_arr = _shading_arrays(g)
    sh = None if sh_arr is None else [torch.tensor(np.asarray(x, np.float64), requires_grad=True) for x in sh_arr]
    proj = project_f64(*leaves, w, cam, lut, opts, shading=sh)
    # The image depends on the parameters only through the per-Gaussian screen-space
    # quantities, so their gradients are summed over the pixel batches first (leaf copies),
    # then taken through the projection once (chain rule).
    inter = [proj.mean2d, proj.conic, proj.rgb, proj.A]
    cut = [t.detach().requires_grad_(True) for t in inter]
    proj_cut = OracleProjection(mean2d=cut[0], conic=cut[1], cov2d=proj.cov2d.detach(), rgb=cut[2], A=cut[3],
                                depth=proj.depth.detach(), kept=proj.kept)
    order = depth_order(fp, proj.kept)
    if pixels is None:
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        pixels = np.stack([xs.reshape(-1), ys.reshape(-1)], 1)
    bg = opts.get("bg", (0.0, 0.0, 0.0)) if bg is None else bg
    d_color = torch.as_tensor(np.asarray(d_color, np.float64))
    if batch <= 0:
        batch = max(1, min(pixels.shape[0], (1 << 22) // max(len(order), 1)))
    total = 0.0
    for s in range(0, pixels.shape[0], batch):
        res = render_pixels(proj_cut, order, pixels[s:s + batch], opts, bg=bg, batch=batch)
        L = (res.color * d_color[s:s + batch]).sum()
        total += float(L.detach())
        L.backward()
    grads_cut = [torch.zeros_like(c) if c.grad is None else c.grad for c in cut]
    torch.autograd.backward(inter, grads_cut)

    def gnp(t):
        return np.zeros(tuple(t.shape)) if t.grad is None else t.grad.detach().numpy().copy()
    return OracleGrads(d_means=gnp(leaves[0]), d_log_scales=gnp(leaves[1]), d_quats=gnp(leaves[2]),
                       d_scalars=gnp(leaves[3]), d_weights=None if w is None else gnp(w),
                       d_mean2d=gnp(cut[0]), d_conic=gnp(cut[1]), d_rgb=gnp(cut[2]),
                       d_A=gnp(cut[3]), loss=total,
                       **({} if sh is None else dict(d_normals=gnp(sh[0]), d_k_ambient=gnp(sh[1]),
                                                     d_k_diffuse=gnp(sh[2]), d_k_specular=gnp(sh[3]),
                                                     d_shininess=gnp(sh[4]))))


# ---------------------------------------------------------------------------------------
# Training-loop neighbours (section "Training"): SSIM loss, Adam, densification statistics
# ---------------------------------------------------------------------------------------

SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def l1_loss(image, target, scale: Optional[float] = None):
    """The L1 term of the training loss (section "Training"): scale * sum |image - target|
    over every pixel-channel, scale = 1 / (number of pixel-channels) unless given, and its
    gradient scale * sign(image - target) with sign(0) = 0.  float64."""
    x = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    if scale is None:
        scale = 1.0 / max(x.size, 1)
    return float(scale * np.abs(x).sum()), scale * np.sign(x)


def ssim_window_1d(size: int = SSIM_WINDOW, sigma: float = SSIM_SIGMA) -> np.ndarray:
    """Normalised 1D Gaussian taps of the SSIM window (Wang et al.; the 2D window is the
    outer product)."""
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(x * x) / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim_map(img, ref):
    """Per-pixel SSIM of two images [P, H, W] (P independent planes, e.g. frames x
    channels), float64 torch: local means, variances and covariance under the Gaussian
    window, zero outside the image ("same" size),
        S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
    C1 = 0.01^2, C2 = 0.03^2 (data range 1)."""
    x = img if torch.is_tensor(img) else torch.as_tensor(np.asarray(img, np.float64))
    y = ref if torch.is_tensor(ref) else torch.as_tensor(np.asarray(ref, np.float64))
    x = x.to(torch.float64)[:, None]
    y = y.to(torch.float64)[:, None]
    g = torch.as_tensor(ssim_window_1d())
    w2 = (g[:, None] * g[None, :])[None, None]
    pad = SSIM_WINDOW // 2

    def blur(t):
        return torch.nn.functional.conv2d(t, w2, padding=pad)
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    s = ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))
    return s[:, 0]


def ssim_loss(img, ref, weight: float):
    """weight * sum over planes and pixels of (1 - SSIM) and its gradient w.r.t. img
    (float64 autograd).  Returns (loss, d_img as numpy)."""
    x = torch.tensor(np.asarray(img, np.float64), requires_grad=True)
    L = weight * (1.0 - ssim_map(x, ref)).sum()
    L.backward()
    return float(L.detach()), x.grad.numpy().copy()


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """One Adam update (Kingma & Ba) in float64, in place on copies; ``step`` counts from 1:
        m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
        p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
    Returns (p, m, v)."""
    p = np.asarray(p, np.float64).copy()
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    p -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def densify_stats(g2d_frames, kept_frames):
    """Densification statistics over a group of frames (the adaptive density control of the
    3DGS-style training the paper follows): per Gaussian, the sum over the frames in which
    it was kept of the norm of the gradient w.r.t. its projected centre, and the number of
    those frames.  g2d_frames: [F, n, 9] screen-space gradients (d mx, d my first);
    kept_frames: [F, n] bool."""
    g = np.asarray(g2d_frames, np.float64)
    k = np.asarray(kept_frames, bool)
    norm = np.sqrt(g[..., 0] ** 2 + g[..., 1] ** 2)
    return (norm * k).sum(0), k.sum(0).astype(np.int64)


def vq_decode(idx, book, widths):
    """Vector-quantised storage of model attributes (the paper compresses trained models by
    clustering most parameters into a codebook): Gaussian i's attribute vector is row
    idx[i] of ``book`` [k, dim]; the row is split, in order, into fields of the given
    widths (e.g. 3 log-scales then 4 quaternion components).  An index outside the codebook
    gives NaN in every field, which culls the Gaussian.  Returns one float32 array per
    field, [n, width] (a width-1 field as [n])."""
    idx = np.asarray(idx).astype(np.int64)
    book = np.asarray(book, np.float32)
    k, dim = book.shape
    assert sum(widths) == dim
    ok = (idx >= 0) & (idx < k)
    rows = np.full((idx.shape[0], dim), np.nan, np.float32)
    rows[ok] = book[idx[ok]]
    out, c = [], 0
    for w in widths:
        f = rows[:, c:c + w]
        out.append(f[:, 0].copy() if w == 1 else f.copy())
        c += w
    return out


# Adaptive density control (section "Training": Gaussians with large view-space positional
# gradients are cloned or split, low-weight Gaussians are pruned, after Kerbl et al.).
KEEP, CLONE, SPLIT, PRUNE = 0, 1, 2, 3
SPLIT_SHRINK = 1.6      # children's scale = parent's / (0.8 * 2 children)


def densify_plan(grad_accum, vis_count, log_scales, weights, grad_thresh, log_scale_thresh, prune_weight):
    """Per-Gaussian decision, every comparison in float32 (the kernel's precision):
    g = accum / vis (0 where vis = 0);  PRUNE when the weight is not >= prune_weight (no weight
    array: never);  else SPLIT when g >= grad_thresh and the largest log-scale exceeds
    log_scale_thresh (a large Gaussian is divided), CLONE when g >= grad_thresh otherwise (a
    small one is copied);  else KEEP.  Returns (action uint8 [n], counts [4])."""
    f32 = np.float32
    acc = np.asarray(grad_accum, np.float32)
    vis = np.asarray(vis_count, np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.where(vis > 0, acc / np.maximum(vis, 1).astype(np.float32), f32(0)).astype(np.float32)
    big = np.asarray(log_scales, np.float32).max(1) > f32(log_scale_thresh)
    hot = g >= f32(grad_thresh)
    act = np.where(hot, np.where(big, SPLIT, CLONE), KEEP).astype(np.uint8)
    if weights is not None:
        low = ~(np.asarray(weights, np.float32) >= f32(prune_weight))
        act[low] = PRUNE
    return act, np.bincount(act, minlength=4).astype(np.int64)


def densify_apply(action, means, log_scales, quats, z, fields):
    """The model after the decisions, in float64: first the survivors (KEEP and CLONE) in
    index order, then one copy of each CLONE Gaussian in index order, then the two children
    of each SPLIT Gaussian in index order.  Child c of parent i sits at
    mu_i + R(q_i) diag(exp(log_s_i)) z[i, c] (z [n, 2, 3], standard normal draws passed in)
    with log-scales log_s_i - ln 1.6.  ``fields`` is a list of (array [n] or [n, w], role):
    role 0 copies the value to clones and children, 1 means (children as above), 2 log-scales
    (children as above), 3 zero for every new Gaussian (optimizer moments).  Returns the new
    arrays in the same order."""
    act = np.asarray(action)
    surv = np.nonzero((act == KEEP) | (act == CLONE))[0]
    clo = np.nonzero(act == CLONE)[0]
    spl = np.nonzero(act == SPLIT)[0]
    q = torch.as_tensor(np.asarray(quats, np.float64))
    q = q / q.norm(dim=1, keepdim=True)
    R = quat_to_rot_f64(q).numpy()
    s = np.exp(np.asarray(log_scales, np.float64))
    zz = np.asarray(z, np.float64)
    # offsets of the children: R diag(s) z
    off = np.einsum("nij,ncj->nci", R, s[:, None, :] * zz)           # [n, 2, 3]
    out = []
    for arr, role in fields:
        a = np.asarray(arr, np.float64)
        if role == 1:
            child = (a[spl, None, :] + off[spl]).reshape(-1, a.shape[1])
        elif role == 2:
            child = np.repeat(a[spl] - math.log(SPLIT_SHRINK), 2, axis=0)
        elif role == 3:
            child = np.zeros((2 * len(spl),) + a.shape[1:])
        else:
            child = np.repeat(a[spl], 2, axis=0)
        copies = np.zeros((len(clo),) + a.shape[1:]) if role == 3 else a[clo]
        out.append(np.concatenate([a[surv], copies, child], axis=0))
    return out
