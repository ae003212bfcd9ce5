"""Thin Python binding of libveg: the C entry points under the same names.

Each function marshals torch tensors and Python objects into the C structs of
include/veg.h and calls the library; every step of the rasterizer runs in the HIP kernels.
Device memory is owned by torch tensors held in the small container classes below.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import check, load

__all__ = [
    "Gaussians", "Proj", "Bins", "default_opts", "make_opts", "veg_project", "veg_bin_count", "veg_bin_sort",
    "veg_bin_overflow", "veg_bin_status", "veg_render_fwd", "veg_render_bwd", "veg_project_bwd", "veg_l1_loss", "veg_fill_u32",
    "veg_debug_math", "veg_bin_hit_words", "alloc_proj", "alloc_bins", "alloc_bin_workspace", "stream_handle",
    "veg_ssim_workspace_bytes", "veg_ssim_loss", "veg_image_loss", "veg_project_bwd_fused", "veg_adam_step", "veg_densify_stats", "veg_project_views",
    "veg_vq_decode", "decode_vq_model", "veg_densify_plan", "veg_densify_apply", "veg_densify_workspace_bytes",
    "KEEP", "CLONE", "SPLIT", "PRUNE", "FIELD_COPY", "FIELD_MEANS", "FIELD_LOG_SCALES", "FIELD_ZERO_NEW",
]

KEEP, CLONE, SPLIT, PRUNE = 0, 1, 2, 3
FIELD_COPY, FIELD_MEANS, FIELD_LOG_SCALES, FIELD_ZERO_NEW = 0, 1, 2, 3


def stream_handle(stream: Optional[torch.cuda.Stream] = None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


LIGHTING = ("normals", "k_ambient", "k_diffuse", "k_specular", "shininess")


@dataclass
class Gaussians:
    """Device SoA model: means [n,3], log_scales [n,3], quats [n,4], scalars [n], weights [n]
    or None, and optionally the lighting attributes normals [n,3], k_ambient, k_diffuse,
    k_specular, shininess [n] (all or none)."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    scalars: torch.Tensor
    weights: Optional[torch.Tensor] = None
    normals: Optional[torch.Tensor] = None
    k_ambient: Optional[torch.Tensor] = None
    k_diffuse: Optional[torch.Tensor] = None
    k_specular: Optional[torch.Tensor] = None
    shininess: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def lit(self) -> bool:
        return self.normals is not None

    def struct(self) -> _lib.veg_gaussians:
        for name in ("means", "log_scales", "quats", "scalars", "weights") + LIGHTING:
            t = getattr(self, name)
            if t is not None and t.dtype != torch.float32:
                raise ValueError(f"{name} must be float32")
        return _lib.veg_gaussians(self.n, _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats),
                                  _ptr(self.scalars), _ptr(self.weights), *(_ptr(getattr(self, k)) for k in LIGHTING))

    @staticmethod
    def from_numpy(g, device="cuda") -> "Gaussians":
        def t(a):
            return None if a is None else torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        sh = getattr(g, "shading", None)
        lit = {} if sh is None else {k: t(getattr(sh, k)) for k in LIGHTING}
        return Gaussians(t(g.means), t(g.log_scales), t(g.quats), t(g.scalars), t(getattr(g, "weights", None)), **lit)


def default_opts() -> _lib.veg_opts:
    o = _lib.veg_opts()
    load().veg_opts_default(ctypes.byref(o))
    return o


def make_opts(d: Optional[dict] = None) -> _lib.veg_opts:
    o = default_opts()
    if d:
        for k, v in d.items():
            if k == "bg":
                o.bg[0], o.bg[1], o.bg[2] = (float(x) for x in v)
            else:
                setattr(o, k, float(v))
    return o


def camera_struct(c) -> _lib.veg_camera:
    cs = _lib.veg_camera()
    view = list(map(float, c.view))
    for k in range(12):
        cs.view[k] = view[k]
    cs.fx, cs.fy, cs.cx, cs.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
    cs.width, cs.height = int(c.width), int(c.height)
    return cs


@dataclass
class Proj:
    struct: _lib.veg_proj
    frames: torch.Tensor
    rec: torch.Tensor
    count: torch.Tensor
    depth: torch.Tensor
    keep: list = field(default_factory=list)   # keeps TF tables alive while the stream uses them

    @property
    def n_pairs(self) -> int:
        return int(self.struct.n) * int(self.struct.n_frames)


def alloc_proj(n: int, n_frames: int, device="cuda") -> Proj:
    pairs = max(1, n * n_frames)
    frames = torch.empty(load().veg_frames_bytes(n_frames), dtype=torch.uint8, device=device)
    rec = torch.empty(pairs * _lib.VEG_REC_FLOATS, dtype=torch.float32, device=device)
    count = torch.empty(pairs, dtype=torch.int32, device=device)
    depth = torch.empty(pairs, dtype=torch.int32, device=device)
    st = _lib.veg_proj(n, n_frames, 0, 0, 0, 0, 0, _ptr(frames), _ptr(rec), _ptr(count), _ptr(depth))
    return Proj(st, frames, rec, count, depth)


def veg_project(g: Gaussians, cams: Sequence, tfs: Sequence[torch.Tensor], opts=None, proj: Optional[Proj] = None,
                stream=None) -> Proj:
    """Projection of len(cams) frames over one model; tfs[f] is a device [k,4] float32 table."""
    nf = len(cams)
    if len(tfs) != nf:
        raise ValueError("one TF per camera")
    if proj is None:
        proj = alloc_proj(g.n, nf, device=g.means.device)
    cam_arr = (_lib.veg_camera * nf)(*[camera_struct(c) for c in cams])
    tf_arr = (_lib.veg_tf * nf)(*[_lib.veg_tf(_ptr(t), int(t.shape[0])) for t in tfs])
    proj.keep = list(tfs)
    o = opts if isinstance(opts, _lib.veg_opts) else make_opts(opts)
    gs = g.struct()
    check(load().veg_project(ctypes.byref(gs), nf, cam_arr, tf_arr, ctypes.byref(o), ctypes.byref(proj.struct),
                             stream_handle(stream)), "veg_project")
    return proj


def veg_project_views(g: Gaussians, cams: Sequence, tfs: Sequence[torch.Tensor], opts=None,
                      proj: Optional[Proj] = None, stream=None) -> Proj:
    """Projection of len(cams) views x len(tfs) // len(cams) tables; frame v * K + k uses
    cams[v] and tfs[v * K + k], and the frames of a view share one key list."""
    nv = len(cams)
    if nv < 1 or len(tfs) % nv != 0:
        raise ValueError("need the same number of tables for every view")
    K = len(tfs) // nv
    if proj is None:
        proj = alloc_proj(g.n, nv * K, device=g.means.device)
    cam_arr = (_lib.veg_camera * nv)(*[camera_struct(c) for c in cams])
    tf_arr = (_lib.veg_tf * len(tfs))(*[_lib.veg_tf(_ptr(t), int(t.shape[0])) for t in tfs])
    proj.keep = list(tfs)
    o = opts if isinstance(opts, _lib.veg_opts) else make_opts(opts)
    gs = g.struct()
    check(load().veg_project_views(ctypes.byref(gs), nv, K, cam_arr, tf_arr, ctypes.byref(o),
                                   ctypes.byref(proj.struct), stream_handle(stream)), "veg_project_views")
    return proj


def alloc_bin_workspace(proj: Proj, device="cuda") -> torch.Tensor:
    nbytes = load().veg_bin_workspace_bytes(proj.n_pairs, 0)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def veg_bin_count(proj: Proj, ws: torch.Tensor, sync: bool = True, stream=None) -> Optional[int]:
    e = ctypes.c_int64(-1)
    check(load().veg_bin_count(ctypes.byref(proj.struct), _ptr(ws), ws.numel(), ctypes.byref(e) if sync else None,
                               stream_handle(stream)), "veg_bin_count")
    return int(e.value) if sync else None


@dataclass
class Bins:
    struct: _lib.veg_bins
    keys: torch.Tensor
    vals: torch.Tensor
    keys_alt: torch.Tensor
    vals_alt: torch.Tensor
    ranges: torch.Tensor
    hits: Optional[torch.Tensor] = None

    @property
    def capacity(self) -> int:
        return int(self.struct.capacity)


def veg_bin_hit_words(capacity: int, total_tiles: int) -> int:
    return int(load().veg_bin_hit_words(int(capacity), int(total_tiles)))


def alloc_bins(proj: Proj, capacity: int, device="cuda", hits: bool = True) -> Bins:
    """Key-list buffers for ``capacity`` entries; with ``hits`` also the per-entry hit bits
    that let the backward pass skip entries the forward pass blended nowhere."""
    cap = max(1, int(capacity))
    k = torch.empty(cap, dtype=torch.int32, device=device)
    v = torch.empty(cap, dtype=torch.int32, device=device)
    ka = torch.empty(cap, dtype=torch.int32, device=device)
    va = torch.empty(cap, dtype=torch.int32, device=device)
    r = torch.empty(max(1, 2 * int(proj.struct.total_tiles)), dtype=torch.int32, device=device)
    h = None
    if hits:
        nw = max(1, int(proj.struct.tfs_per_view)) * veg_bin_hit_words(capacity, proj.struct.total_tiles)
        h = torch.empty(max(1, nw), dtype=torch.int64, device=device)
    st = _lib.veg_bins(_ptr(k), _ptr(v), _ptr(ka), _ptr(va), _ptr(r), int(capacity),
                       _ptr(h) if h is not None else None, int(h.numel()) if h is not None else 0)
    return Bins(st, k, v, ka, va, r, h)


def veg_bin_sort(proj: Proj, ws: torch.Tensor, bins: Bins, stream=None) -> Bins:
    check(load().veg_bin_sort(ctypes.byref(proj.struct), _ptr(ws), ws.numel(), ctypes.byref(bins.struct),
                              stream_handle(stream)), "veg_bin_sort")
    return bins


def veg_bin_status(ws: torch.Tensor, dst: torch.Tensor, stream=None) -> torch.Tensor:
    """dst (device int64 [2]) <- (entries E, overflow flag) of the last veg_bin_sort on ``ws``,
    without synchronising."""
    if dst.dtype != torch.int64 or dst.numel() < 2 or not dst.is_contiguous():
        raise ValueError("dst must be a contiguous int64 tensor of at least 2 elements")
    check(load().veg_bin_status(_ptr(ws), ws.numel(), _ptr(dst), stream_handle(stream)), "veg_bin_status")
    return dst


def veg_bin_static(proj: Proj, bins: Bins, status: torch.Tensor, stream=None) -> Bins:
    """veg_bin_count + veg_bin_sort + veg_bin_status in one call with the library's own
    scratch (nothing allocated, no workspace); status (device int64 [2]) <- (E, overflow)."""
    if status.dtype != torch.int64 or status.numel() < 2 or not status.is_contiguous():
        raise ValueError("status must be a contiguous int64 tensor of at least 2 elements")
    check(load().veg_bin_static(ctypes.byref(proj.struct), ctypes.byref(bins.struct), _ptr(status),
                                stream_handle(stream)), "veg_bin_static")
    return bins


def veg_bin_overflow(ws: torch.Tensor, stream=None):
    e = ctypes.c_int64(0)
    ov = ctypes.c_int32(0)
    check(load().veg_bin_overflow(_ptr(ws), ws.numel(), ctypes.byref(e), ctypes.byref(ov), stream_handle(stream)),
          "veg_bin_overflow")
    return int(e.value), bool(ov.value)


def veg_render_fwd(proj: Proj, bins: Bins, opts, image: torch.Tensor, t_final: Optional[torch.Tensor],
                   n_last: Optional[torch.Tensor], n_contrib: Optional[torch.Tensor] = None, stream=None):
    o = opts if isinstance(opts, _lib.veg_opts) else make_opts(opts)
    check(load().veg_render_fwd(ctypes.byref(proj.struct), ctypes.byref(bins.struct), ctypes.byref(o), _ptr(image),
                                _ptr(t_final), _ptr(n_last), _ptr(n_contrib), stream_handle(stream)),
          "veg_render_fwd")


def veg_render_fwd_l1(proj: Proj, bins: Bins, opts, target: torch.Tensor, scale: float, loss_slots: torch.Tensor,
                      d_image: torch.Tensor, t_final: Optional[torch.Tensor], n_last: Optional[torch.Tensor],
                      stream=None):
    """Forward pass with the L1 term fused: d_image <- scale * sign(colour - target), loss_slots
    (device float64 [VEG_L1_SLOTS]) += scale * sum |colour - target| spread over the slots."""
    if loss_slots.dtype != torch.float64 or loss_slots.numel() < _lib.VEG_L1_SLOTS:
        raise ValueError("loss_slots must be a float64 tensor of VEG_L1_SLOTS elements")
    o = opts if isinstance(opts, _lib.veg_opts) else make_opts(opts)
    check(load().veg_render_fwd_l1(ctypes.byref(proj.struct), ctypes.byref(bins.struct), ctypes.byref(o),
                                   _ptr(target), float(scale), _ptr(loss_slots), _ptr(d_image), _ptr(t_final),
                                   _ptr(n_last), stream_handle(stream)), "veg_render_fwd_l1")


def veg_render_bwd(proj: Proj, bins: Bins, opts, t_final: torch.Tensor, n_last: torch.Tensor, d_image: torch.Tensor,
                   g2d: torch.Tensor, stream=None):
    o = opts if isinstance(opts, _lib.veg_opts) else make_opts(opts)
    check(load().veg_render_bwd(ctypes.byref(proj.struct), ctypes.byref(bins.struct), ctypes.byref(o), _ptr(t_final),
                                _ptr(n_last), _ptr(d_image), _ptr(g2d), stream_handle(stream)), "veg_render_bwd")


def veg_project_bwd(g: Gaussians, proj: Proj, opts, g2d: torch.Tensor, d_means, d_log_scales, d_quats, d_scalars,
                    d_weights=None, stream=None, d_lighting=None):
    """``d_lighting``: None or (d_normals, d_k_ambient, d_k_diffuse, d_k_specular, d_shininess)."""
    o = opts if isinstance(opts, _lib.veg_opts) else make_opts(opts)
    gs = g.struct()
    lg = (None,) * 5 if d_lighting is None else tuple(d_lighting)
    gr = _lib.veg_grads(_ptr(d_means), _ptr(d_log_scales), _ptr(d_quats), _ptr(d_scalars), _ptr(d_weights),
                        *(_ptr(t) for t in lg))
    check(load().veg_project_bwd(ctypes.byref(gs), ctypes.byref(proj.struct), ctypes.byref(o), _ptr(g2d),
                                 ctypes.byref(gr), stream_handle(stream)), "veg_project_bwd")


def veg_project_bwd_fused(g: Gaussians, proj: Proj, opts, g2d: torch.Tensor, d_means, d_log_scales, d_quats,
                          d_scalars, d_weights=None, stream=None, d_lighting=None, grad_accum=None, vis_count=None,
                          consume_g2d: bool = False):
    """veg_project_bwd plus, from the same g2d reads, the densification statistics (when
    ``grad_accum`` and ``vis_count`` are given) and, with ``consume_g2d``, g2d left zero."""
    o = opts if isinstance(opts, _lib.veg_opts) else make_opts(opts)
    gs = g.struct()
    lg = (None,) * 5 if d_lighting is None else tuple(d_lighting)
    gr = _lib.veg_grads(_ptr(d_means), _ptr(d_log_scales), _ptr(d_quats), _ptr(d_scalars), _ptr(d_weights),
                        *(_ptr(t) for t in lg))
    check(load().veg_project_bwd_fused(ctypes.byref(gs), ctypes.byref(proj.struct), ctypes.byref(o), _ptr(g2d),
                                       ctypes.byref(gr), _ptr(grad_accum), _ptr(vis_count), int(bool(consume_g2d)),
                                       stream_handle(stream)), "veg_project_bwd_fused")


def veg_l1_loss(image: torch.Tensor, target: torch.Tensor, scale: float, loss: torch.Tensor, d_image: torch.Tensor,
                stream=None):
    if loss.dtype != torch.float64:
        raise ValueError("loss accumulator must be float64")
    check(load().veg_l1_loss(_ptr(image), _ptr(target), image.numel(), float(scale), _ptr(loss), _ptr(d_image),
                             stream_handle(stream)), "veg_l1_loss")


def veg_ssim_workspace_bytes(n_planes: int, width: int, height: int) -> int:
    return int(load().veg_ssim_workspace_bytes(n_planes, width, height))


def veg_ssim_loss(image: torch.Tensor, target: torch.Tensor, weight: float, loss: torch.Tensor,
                  d_image: torch.Tensor, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Adds weight * sum(1 - SSIM) over the planes of ``image`` (any leading shape, the last
    two dimensions H, W) to ``loss`` and its gradient to ``d_image``.  Returns the workspace
    (allocated here when ``ws`` is None or too small)."""
    if loss.dtype != torch.float64:
        raise ValueError("loss accumulator must be float64")
    if image.shape != target.shape or image.shape != d_image.shape or image.dim() < 2:
        raise ValueError("image, target and d_image must share one shape [..., H, W]")
    H, W = int(image.shape[-2]), int(image.shape[-1])
    planes = image.numel() // max(1, H * W)
    need = veg_ssim_workspace_bytes(planes, W, H)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(max(need, 4), dtype=torch.uint8, device=image.device)
    check(load().veg_ssim_loss(_ptr(image), _ptr(target), planes, W, H, float(weight), _ptr(loss), _ptr(d_image),
                               _ptr(ws), ws.numel() * ws.element_size(), stream_handle(stream)), "veg_ssim_loss")
    return ws


def veg_image_loss(image: torch.Tensor, target: torch.Tensor, l1_scale: float, ssim_weight: float, loss: torch.Tensor,
                   d_image: torch.Tensor, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The whole image loss in one pass: adds l1_scale * sum|image - target| + ssim_weight *
    sum(1 - SSIM) to ``loss`` and writes (overwrites) its gradient into ``d_image``.  Shapes
    and workspace as for veg_ssim_loss; returns the workspace."""
    if loss.dtype != torch.float64:
        raise ValueError("loss accumulator must be float64")
    if image.shape != target.shape or image.shape != d_image.shape or image.dim() < 2:
        raise ValueError("image, target and d_image must share one shape [..., H, W]")
    H, W = int(image.shape[-2]), int(image.shape[-1])
    planes = image.numel() // max(1, H * W)
    need = veg_ssim_workspace_bytes(planes, W, H)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(max(need, 4), dtype=torch.uint8, device=image.device)
    check(load().veg_image_loss(_ptr(image), _ptr(target), planes, W, H, float(l1_scale), float(ssim_weight),
                                _ptr(loss), _ptr(d_image), _ptr(ws), ws.numel() * ws.element_size(),
                                stream_handle(stream)), "veg_image_loss")
    return ws


def veg_adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float, step: int,
                  beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, stream=None):
    for t in (param, grad, m, v):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != param.numel():
            raise ValueError("adam: param, grad, m, v must be contiguous float32 of one size")
    check(load().veg_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), float(lr), float(beta1),
                               float(beta2), float(eps), int(step), stream_handle(stream)), "veg_adam_step")


def veg_densify_stats(proj: "Proj", g2d: torch.Tensor, grad_accum: torch.Tensor, vis_count: torch.Tensor,
                      stream=None):
    if grad_accum.dtype != torch.float32 or vis_count.dtype != torch.int32:
        raise ValueError("grad_accum must be float32 and vis_count int32")
    if grad_accum.numel() < int(proj.struct.n) or vis_count.numel() < int(proj.struct.n):
        raise ValueError("grad_accum / vis_count smaller than the number of Gaussians")
    check(load().veg_densify_stats(ctypes.byref(proj.struct), _ptr(g2d), _ptr(grad_accum), _ptr(vis_count),
                                   stream_handle(stream)), "veg_densify_stats")


def veg_vq_decode(idx: torch.Tensor, book: torch.Tensor, outs: Sequence[torch.Tensor], stream=None):
    """Expands codebook indices (device uint16 [n]) into ``outs`` (device float32 [n, w] or
    [n] for w = 1); the codebook rows [k, dim] are split across them in order."""
    if idx.dtype != torch.uint16 or book.dtype != torch.float32 or book.dim() != 2:
        raise ValueError("idx must be uint16 and book float32 [k, dim]")
    n = idx.numel()
    fields = []
    for o in outs:
        w = 1 if o.dim() == 1 else int(o.shape[1])
        if o.dtype != torch.float32 or not o.is_contiguous() or o.numel() != n * w:
            raise ValueError("each output must be a contiguous float32 [n] or [n, w] tensor")
        fields.append(_lib.veg_vq_field(_ptr(o), w))
    arr = (_lib.veg_vq_field * len(fields))(*fields)
    check(load().veg_vq_decode(_ptr(idx), n, _ptr(book.contiguous()), int(book.shape[0]), int(book.shape[1]), arr,
                               len(fields), stream_handle(stream)), "veg_vq_decode")


def decode_vq_model(means: torch.Tensor, scalars: torch.Tensor, shape_idx: torch.Tensor, shape_book: torch.Tensor,
                    weights: Optional[torch.Tensor] = None, stream=None) -> "Gaussians":
    """A model stored with its shape (log-scales and quaternion, 7 values) in a codebook,
    decoded into a Gaussians set (positions, scalars and weights stay per Gaussian)."""
    n = means.shape[0]
    ls = torch.empty((n, 3), dtype=torch.float32, device=means.device)
    q = torch.empty((n, 4), dtype=torch.float32, device=means.device)
    veg_vq_decode(shape_idx, shape_book, [ls, q], stream=stream)
    return Gaussians(means, ls, q, scalars, weights)


def veg_densify_workspace_bytes(n: int) -> int:
    return int(load().veg_densify_workspace_bytes(int(n)))


def veg_densify_plan(grad_accum: torch.Tensor, vis_count: torch.Tensor, log_scales: torch.Tensor,
                     weights: Optional[torch.Tensor], grad_thresh: float, log_scale_thresh: float,
                     prune_weight: float, read_counts: bool = True, stream=None):
    """Clone / split / prune decisions; returns (action uint8 [n], counts [KEEP, CLONE, SPLIT,
    PRUNE] or None, workspace for veg_densify_apply)."""
    n = int(log_scales.shape[0])
    if grad_accum.dtype != torch.float32 or vis_count.dtype != torch.int32 or grad_accum.numel() < n \
            or vis_count.numel() < n:
        raise ValueError("grad_accum float32 [n] and vis_count int32 [n] expected")
    action = torch.empty(max(1, n), dtype=torch.uint8, device=log_scales.device)
    ws = torch.empty(max(4, veg_densify_workspace_bytes(n)), dtype=torch.uint8, device=log_scales.device)
    counts = (ctypes.c_int64 * 4)() if read_counts else None
    check(load().veg_densify_plan(n, _ptr(grad_accum), _ptr(vis_count), _ptr(log_scales.contiguous()), _ptr(weights),
                                  float(grad_thresh), float(log_scale_thresh), float(prune_weight), _ptr(action),
                                  ctypes.cast(counts, ctypes.c_void_p) if counts is not None else None, _ptr(ws),
                                  ws.numel(), stream_handle(stream)), "veg_densify_plan")
    return action, (list(counts) if counts is not None else None), ws


def veg_densify_apply(action: torch.Tensor, quats: torch.Tensor, log_scales: torch.Tensor, z: torch.Tensor,
                      fields: Sequence[tuple], ws: torch.Tensor, stream=None):
    """Writes the new model: fields are (src [n] or [n, w], dst [n_new] or [n_new, w], role)."""
    n = int(log_scales.shape[0])
    if z.dtype != torch.float32 or z.numel() < 6 * n:
        raise ValueError("z must be float32 [n, 2, 3]")
    fs = []
    for src, dst, role in fields:
        w = 1 if src.dim() == 1 else int(src.shape[1])
        if src.dtype != torch.float32 or dst.dtype != torch.float32 or not src.is_contiguous() \
                or not dst.is_contiguous() or (dst.numel() // max(1, w)) * w != dst.numel():
            raise ValueError("fields must be contiguous float32 tensors of one width")
        fs.append(_lib.veg_densify_field(_ptr(src), _ptr(dst), w, int(role)))
    arr = (_lib.veg_densify_field * len(fs))(*fs)
    check(load().veg_densify_apply(n, _ptr(action), _ptr(quats.contiguous()), _ptr(log_scales.contiguous()),
                                   _ptr(z.contiguous()), arr, len(fs), _ptr(ws), ws.numel(), stream_handle(stream)),
          "veg_densify_apply")


def veg_fill_u32(t: torch.Tensor, value: int = 0, stream=None):
    nwords = t.numel() * t.element_size() // 4
    check(load().veg_fill_u32(_ptr(t), nwords, ctypes.c_uint32(value & 0xFFFFFFFF), stream_handle(stream)),
          "veg_fill_u32")


def veg_debug_math(op: int, x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    out = torch.empty_like(x)
    check(load().veg_debug_math(op, _ptr(x), _ptr(y), _ptr(out), x.numel(), stream_handle(stream)), "veg_debug_math")
    return out
