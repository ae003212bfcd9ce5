"""Seeded generators for the synthetic workloads.

The paper trains and renders on volume datasets (Vortex, Chameleon, RBL, Mito, a CT head;
section "Setup") that are not available here.  These generators stand in for them with
Gaussian sets shaped like the paper's volumes: uniform filler plus isosurface-like
spherical shells, scalar values in [0,1], small anisotropic scales, random rotations, orbit
cameras around the volume (section "Evaluation of Metrics": spherical orbit, whole bounding
box in view), and 256-entry RGBA transfer-function tables whose opacity has a few peaks,
like the narrow/broad opacity maps of the evaluation.

Every array is produced from ``numpy.random.Generator(PCG64(seed))`` with
``seed = SEED_BASE + config_index`` (plus a per-model / per-request sub-seed), so the
oracle side and the GPU side see bit-identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 0x2504_13339

__all__ = [
    "SEED_BASE", "Gaussians", "Shading", "random_shading", "Camera", "rng_for", "uniform_gaussians", "shell_gaussians",
    "clustered_gaussians", "random_tf", "identity_tf", "constant_tf", "fibonacci_directions",
    "random_direction", "look_at_camera", "perturbed_copy", "sample_pixels", "Workload",
    "workload", "serve_trace", "DEFAULT_OPTS", "tent_opacity", "sequential_rgb", "tent_tfs", "vq_encode",
]

# Renderer options used by every workload (alpha clamp, skip threshold, stop threshold
# from the workload definitions; low-pass, near plane and guard band are this library's
# readings where the paper is silent).
DEFAULT_OPTS = dict(alpha_clamp=0.99, alpha_min=1.0 / 255.0, t_min=1e-4, lowpass=0.3,
                    near_z=0.2, guard=1.3, bg=(0.0, 0.0, 0.0))


def rng_for(config_index: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + int(config_index), int(sub)]))


@dataclass
class Shading:
    """Per-Gaussian lighting attributes (section "The VEG Representation", Blinn-Phong):
    normal, ambient / diffuse / specular coefficients and shininess, already activated."""
    normals: np.ndarray      # [n,3] float32, any length > 0
    k_ambient: np.ndarray    # [n]
    k_diffuse: np.ndarray    # [n]
    k_specular: np.ndarray   # [n]
    shininess: np.ndarray    # [n] > 0

    def subset(self, idx) -> "Shading":
        return Shading(self.normals[idx].copy(), self.k_ambient[idx].copy(), self.k_diffuse[idx].copy(),
                       self.k_specular[idx].copy(), self.shininess[idx].copy())

    def astype(self, dt) -> "Shading":
        return Shading(*(np.asarray(a, dt) for a in (self.normals, self.k_ambient, self.k_diffuse,
                                                      self.k_specular, self.shininess)))


@dataclass
class Gaussians:
    means: np.ndarray        # [n,3] float32
    log_scales: np.ndarray   # [n,3] float32
    quats: np.ndarray        # [n,4] float32, (w,x,y,z)
    scalars: np.ndarray      # [n]   float32 in [0,1]
    weights: Optional[np.ndarray] = None  # [n] float32 or None (== 1)
    shading: Optional[Shading] = None     # lighting attributes or None (TF colour only)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Gaussians":
        return Gaussians(self.means[idx].copy(), self.log_scales[idx].copy(),
                         self.quats[idx].copy(), self.scalars[idx].copy(),
                         None if self.weights is None else self.weights[idx].copy(),
                         None if self.shading is None else self.shading.subset(idx))


def random_shading(rng, n, k_ambient=(0.1, 0.4), k_diffuse=(0.4, 0.9), k_specular=(0.0, 0.5),
                   shininess=(2.0, 64.0)) -> Shading:
    """Random lighting attributes: normals from an isotropic normal distribution (unit
    after normalisation), coefficients uniform in the given ranges, shininess log-uniform."""
    nrm = rng.standard_normal((n, 3)).astype(np.float32)
    ka = rng.uniform(*k_ambient, n).astype(np.float32)
    kd = rng.uniform(*k_diffuse, n).astype(np.float32)
    ks = rng.uniform(*k_specular, n).astype(np.float32)
    beta = np.exp(rng.uniform(math.log(shininess[0]), math.log(shininess[1]), n)).astype(np.float32)
    return Shading(nrm, ka, kd, ks, beta)


@dataclass
class Camera:
    view: np.ndarray   # [12] float32, world->camera 3x4 row-major (x right, y down, z forward)
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _log_uniform_scales(rng, n, lo, hi):
    return rng.uniform(math.log(lo), math.log(hi), size=(n, 3)).astype(np.float32)


def uniform_gaussians(rng, n, scale_lo=0.01, scale_hi=0.08, box=1.0) -> Gaussians:
    means = rng.uniform(-box, box, size=(n, 3)).astype(np.float32)
    ls = _log_uniform_scales(rng, n, scale_lo, scale_hi)
    q = _unit_quats(rng, n)
    v = rng.uniform(0.0, 1.0, size=n).astype(np.float32)
    return Gaussians(means, ls, q, v)


def shell_gaussians(rng, n, scale_lo=0.01, scale_hi=0.08, n_shells=5, jitter=0.02,
                    radius_lo=0.15, radius_hi=0.5) -> Gaussians:
    """Points on ``n_shells`` random spherical shells; one fixed scalar per shell."""
    centres = rng.uniform(-0.6, 0.6, size=(n_shells, 3))
    radii = rng.uniform(radius_lo, radius_hi, size=n_shells)
    shell_v = rng.uniform(0.0, 1.0, size=n_shells)
    which = rng.integers(0, n_shells, size=n)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radii[which] + rng.normal(0.0, jitter, size=n)
    means = (centres[which] + d * r[:, None]).astype(np.float32)
    ls = _log_uniform_scales(rng, n, scale_lo, scale_hi)
    q = _unit_quats(rng, n)
    v = shell_v[which].astype(np.float32)
    return Gaussians(means, ls, q, v)


def clustered_gaussians(rng, n, frac_shell=0.7, scale_lo=0.01, scale_hi=0.08,
                        **shell_kw) -> Gaussians:
    n_shell = int(round(n * frac_shell))
    a = shell_gaussians(rng, n_shell, scale_lo, scale_hi, **shell_kw)
    b = uniform_gaussians(rng, n - n_shell, scale_lo, scale_hi)
    perm = rng.permutation(n)
    cat = lambda x, y: np.concatenate([x, y], axis=0)[perm].copy()
    return Gaussians(cat(a.means, b.means), cat(a.log_scales, b.log_scales),
                     cat(a.quats, b.quats), cat(a.scalars, b.scalars))


def random_tf(rng, k=256, n_peaks=3) -> np.ndarray:
    """[k,4] float32 RGBA table: opacity = clipped sum of ``n_peaks`` Gaussian bumps at
    random scalars; colour = piecewise-linear through 6 random colours at sorted knots
    (0, four random interior knots, 1).  Straight (not premultiplied) colour."""
    x = np.arange(k, dtype=np.float64) / (k - 1)
    m = rng.uniform(0.0, 1.0, n_peaks)
    s = rng.uniform(0.02, 0.08, n_peaks)
    h = rng.uniform(0.5, 1.0, n_peaks)
    op = np.clip((h[None] * np.exp(-((x[:, None] - m[None]) ** 2) / (2 * s[None] ** 2))).sum(1), 0, 1)
    knots = np.concatenate([[0.0], np.sort(rng.uniform(0.0, 1.0, 4)), [1.0]])
    cols = rng.uniform(0.0, 1.0, (6, 3))
    rgb = np.stack([np.interp(x, knots, cols[:, c]) for c in range(3)], axis=1)
    return np.concatenate([rgb, op[:, None]], axis=1).astype(np.float32)


def tent_opacity(x, n_steps: int, step: int) -> np.ndarray:
    """Opacity map ``step`` of the opacity-guided training family (section "Training"): the
    scalar range [0,1] is cut into ``n_steps`` equal steps; map j is a tent centred in step
    j, c = (j + 1/2) / n_steps, falling off linearly with slope n_steps:
    O_j(x) = max(0, 1 - n_steps |x - c|).  Peak 1 (the paper does not state the height).
    Neighbouring tents overlap by half, so the maps sum to 1 on [c_0, c_{n-1}]."""
    x = np.asarray(x, np.float64)
    c = (step + 0.5) / n_steps
    return np.maximum(0.0, 1.0 - n_steps * np.abs(x - c))


def sequential_rgb(x) -> np.ndarray:
    """A sequential (non-diverging) colour map, dark blue through teal and green to yellow,
    piecewise linear in RGB through five knots.  The paper trains with one sequential
    colour map and reports that the colour mapping matters little as long as it is not
    diverging; this one is this project's own."""
    x = np.asarray(x, np.float64)
    knots = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    cols = np.array([[0.10, 0.05, 0.35], [0.15, 0.30, 0.55], [0.10, 0.55, 0.55], [0.40, 0.75, 0.30],
                     [0.98, 0.90, 0.15]])
    return np.stack([np.interp(x, knots, cols[:, ch]) for ch in range(3)], axis=-1)


def tent_tfs(n_steps: int, k: int = 256) -> List[np.ndarray]:
    """The ``n_steps`` [k,4] float32 tables of the opacity-guided family: colour from
    ``sequential_rgb``, opacity from ``tent_opacity``, both sampled at x_j = j / (k-1)."""
    x = np.arange(k, dtype=np.float64) / (k - 1)
    rgb = sequential_rgb(x)
    return [np.concatenate([rgb, tent_opacity(x, n_steps, j)[:, None]], axis=1).astype(np.float32)
            for j in range(n_steps)]


def vq_encode(rng, x, k: int, iters: int = 4, chunk: int = 65536):
    """Codebook of ``k`` rows for the vectors ``x`` [n, dim] and the index of each vector's
    nearest row (Euclidean), by a few Lloyd (k-means) iterations from k distinct rows of x
    (distinct values where x has at least k) drawn with ``rng``.  Stands in for the compression step that produces a stored model;
    returns (idx uint16 [n], book float32 [k, dim])."""
    x = np.asarray(x, np.float32)
    n = x.shape[0]
    assert 1 <= k <= 65536 and k <= n
    u = np.unique(x, axis=0)                     # start from distinct rows where there are enough
    src = u if u.shape[0] >= k else x
    book = src[rng.choice(src.shape[0], k, replace=False)].astype(np.float64)

    def nearest(b):
        idx = np.empty(n, np.int64)
        bb = (b * b).sum(1)
        for s in range(0, n, chunk):
            xs = x[s:s + chunk].astype(np.float64)
            d = bb[None, :] - 2.0 * xs @ b.T
            idx[s:s + chunk] = np.argmin(d, axis=1)
        return idx
    for _ in range(iters):
        idx = nearest(book)
        cnt = np.bincount(idx, minlength=k)
        acc = np.zeros_like(book)
        np.add.at(acc, idx, x.astype(np.float64))
        filled = cnt > 0
        book[filled] = acc[filled] / cnt[filled, None]
    idx = nearest(book)
    return idx.astype(np.uint16), book.astype(np.float32)


def identity_tf(k=256) -> np.ndarray:
    x = (np.arange(k, dtype=np.float64) / (k - 1)).astype(np.float32)
    return np.stack([x, x, x, x], axis=1).copy()


def constant_tf(k=256, rgba=(0.3, 0.6, 0.9, 0.5)) -> np.ndarray:
    return np.tile(np.asarray(rgba, np.float32)[None], (k, 1)).copy()


def fibonacci_directions(n) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - 2.0 * (k + 0.5) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def random_direction(rng) -> np.ndarray:
    d = rng.standard_normal(3)
    return d / np.linalg.norm(d)


def look_at_camera(direction, radius, width, height, fovy_deg=50.0, target=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at ``target + radius*direction`` looking at ``target``.

    Axes follow the OpenCV convention (x right, y down, z forward).  World up is +z, or +y
    when the view direction is within 0.999 of +-z.  The field of view is vertical:
    fx = fy = (H/2)/tan(fovy/2); the principal point is the image centre.
    """
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    tgt = np.asarray(target, np.float64)
    eye = tgt + radius * d
    fwd = tgt - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 0.0, 1.0])
    if abs(fwd @ up) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd], axis=0)
    trans = -rot @ eye
    view = np.concatenate([rot, trans[:, None]], axis=1).reshape(12).astype(np.float32)
    f = (0.5 * height) / math.tan(math.radians(fovy_deg) * 0.5)
    return Camera(view=view, fx=float(np.float32(f)), fy=float(np.float32(f)),
                  cx=float(0.5 * width), cy=float(0.5 * height), width=int(width), height=int(height))


def perturbed_copy(rng, g: Gaussians, mean_sigma=0.01, scalar_sigma=0.05) -> Gaussians:
    """Copy with means + N(0, mean_sigma) and scalars + N(0, scalar_sigma) clipped to [0,1]."""
    means = (g.means + rng.normal(0.0, mean_sigma, g.means.shape)).astype(np.float32)
    v = np.clip(g.scalars + rng.normal(0.0, scalar_sigma, g.scalars.shape), 0.0, 1.0).astype(np.float32)
    return Gaussians(means, g.log_scales.copy(), g.quats.copy(), v,
                     None if g.weights is None else g.weights.copy(),
                     None if g.shading is None else g.shading.subset(slice(None)))


def sample_pixels(rng, width, height, n, centre_frac=0.5) -> np.ndarray:
    """[n,2] int32 (x,y) pixel coordinates: ``centre_frac`` of them inside the central
    quarter of the image (where the synthetic volumes are densest), the rest uniform."""
    nc = int(n * centre_frac)
    cx = rng.integers(width // 4, max(width // 4 + 1, 3 * width // 4), size=nc)
    cy = rng.integers(height // 4, max(height // 4 + 1, 3 * height // 4), size=nc)
    ux = rng.integers(0, width, size=n - nc)
    uy = rng.integers(0, height, size=n - nc)
    return np.stack([np.concatenate([cx, ux]), np.concatenate([cy, uy])], axis=1).astype(np.int32)


@dataclass
class Workload:
    name: str
    gaussians: Gaussians
    cameras: List[Camera]
    tfs: List[np.ndarray]
    frames: List[tuple]                  # (camera index, tf index) per frame
    opts: dict = field(default_factory=lambda: dict(DEFAULT_OPTS))
    target_gaussians: Optional[Gaussians] = None  # perturbed copy for training targets
    description: str = ""

    @property
    def width(self):
        return self.cameras[0].width

    @property
    def height(self):
        return self.cameras[0].height


def _frames(n_views, n_tfs):
    return [(v, t) for v in range(n_views) for t in range(n_tfs)]


def workload(index: int, n_override: Optional[int] = None, views_override: Optional[int] = None,
             tfs_override: Optional[int] = None, res_override: Optional[int] = None) -> Workload:
    """The synthetic workloads: 0..4 (3 is the serving trace) and 5, the opacity-guided
    training family.  Overrides shrink a workload for tests while keeping its structure
    (same generator, same seed)."""
    rng = rng_for(index)
    if index == 0:
        n = n_override or 1000
        g = uniform_gaussians(rng, n, 0.01, 0.08)
        res = res_override or 64
        cams = [look_at_camera(random_direction(rng), 3.0, res, res)]
        tfs = [random_tf(rng)]
        return Workload("render-1k-64px", g, cams, tfs, _frames(1, 1),
                        description="1,000 uniform Gaussians, one TF, 64x64, forward")
    if index == 1:
        n = n_override or 200_000
        g = clustered_gaussians(rng, n, 0.7, 0.01, 0.08)
        nv, nt, res = views_override or 8, tfs_override or 4, res_override or 800
        cams = [look_at_camera(d, 3.0, res, res) for d in fibonacci_directions(nv)]
        tfs = [random_tf(rng) for _ in range(nt)]
        tgt = perturbed_copy(rng_for(index, 1), g)
        return Workload("train-200k-800px-8x4", g, cams, tfs, _frames(nv, nt), target_gaussians=tgt,
                        description="200k shell-clustered Gaussians, 8 views x 4 TFs, 800x800, fwd+bwd")
    if index == 2:
        n = n_override or 1_000_000
        g = clustered_gaussians(rng, n, 0.7, 0.002, 0.03)
        nv, nt, res = views_override or 16, tfs_override or 3, res_override or 1024
        cams = [look_at_camera(d, 3.0, res, res) for d in fibonacci_directions(nv)]
        tfs = [random_tf(rng) for _ in range(nt)]
        tgt = perturbed_copy(rng_for(index, 1), g)
        return Workload("train-1M-1024px-16x3", g, cams, tfs, _frames(nv, nt), target_gaussians=tgt,
                        description="1M shell-clustered Gaussians, 16 views x 3 TFs, 1024x1024, fwd+bwd with recompute")
    if index == 4:
        n = n_override or 4_000_000
        g = clustered_gaussians(rng, n, 0.5, 0.002, 0.03)
        nv, nt, res = views_override or 32, tfs_override or 4, res_override or 2048
        cams = [look_at_camera(d, 3.0, res, res) for d in fibonacci_directions(nv)]
        tfs = [random_tf(rng) for _ in range(nt)]
        tgt = perturbed_copy(rng_for(index, 1), g)
        return Workload("stress-4M-2048px-32x4", g, cams, tfs, _frames(nv, nt), target_gaussians=tgt,
                        description="4M Gaussians (50% uniform, 50% shells), 32 views x 4 TFs, 2048x2048")
    if index == 5:
        # opacity-guided training: every view rendered with the whole tent family (10 steps,
        # the paper's default), 500k Gaussians (the paper's initial count), 800x800
        n = n_override or 500_000
        g = clustered_gaussians(rng, n, 0.7, 0.002, 0.03)
        nv, nt, res = views_override or 8, tfs_override or 10, res_override or 800
        cams = [look_at_camera(d, 3.0, res, res) for d in fibonacci_directions(nv)]
        tfs = tent_tfs(nt)
        tgt = perturbed_copy(rng_for(index, 1), g)
        return Workload("opacity-guided-500k-800px-8x10", g, cams, tfs, _frames(nv, nt), target_gaussians=tgt,
                        description="500k shell-clustered Gaussians, 8 views x 10 tent opacity maps, 800x800, fwd+bwd")
    raise ValueError("workload index must be 0, 1, 2, 4 or 5 (3 is the serving trace: serve_trace())")


@dataclass
class ServeRequest:
    arrival_s: float
    model: int
    camera: Camera
    tf: np.ndarray


def serve_trace(rate_hz: float, n_requests: int, model_sizes=(100_000, 500_000, 1_000_000, 3_000_000),
                resolutions=((512, 512), (1024, 1024), (1920, 1080)), seed_sub: int = 0,
                build_models: bool = True):
    """Models and a Poisson request trace for the serving workload.

    Models: shell-clustered; the 100k/500k ones with log-U[0.01,0.08] scales, the 1M/3M
    ones with log-U[0.002,0.03].  Requests: exponential inter-arrival times at ``rate_hz``,
    uniform model, camera uniform on the sphere at radius U[2.5,4], fresh random TF,
    resolution uniform over ``resolutions``.
    """
    models = []
    if build_models:
        for mi, n in enumerate(model_sizes):
            mrng = rng_for(3, 1000 + mi)
            lo, hi = (0.01, 0.08) if n <= 500_000 else (0.002, 0.03)
            models.append(clustered_gaussians(mrng, n, 0.7, lo, hi))
    rng = rng_for(3, 1 + seed_sub)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    reqs = []
    for i in range(n_requests):
        m = int(rng.integers(0, len(model_sizes)))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        cam = look_at_camera(random_direction(rng), float(rng.uniform(2.5, 4.0)), w, h)
        reqs.append(ServeRequest(float(t[i]), m, cam, random_tf(rng)))
    return models, reqs
