"""Rendering, backward and the multi-view x multi-TF training step on top of the C ABI.

All arithmetic runs in libveg's kernels; this module only sequences the calls and owns
the device buffers (torch tensors).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import veg as V


@dataclass
class FwdState:
    proj: V.Proj
    bins: V.Bins
    ws: torch.Tensor
    image: torch.Tensor
    t_final: torch.Tensor
    n_last: torch.Tensor
    n_entries: int
    opts: object
    n_contrib: Optional[torch.Tensor] = None


class _NoTimer:
    def __call__(self, name):
        return self

    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


NO_TIMER = _NoTimer()


class EventTimer:
    """Records HIP events on the current stream around named library calls; no host sync."""

    def __init__(self):
        self.pairs = {}
        self._name = None

    def __call__(self, name):
        self._name = name
        return self

    def __enter__(self):
        self._s = torch.cuda.Event(enable_timing=True)
        self._e = torch.cuda.Event(enable_timing=True)
        self._s.record()
        return self

    def __exit__(self, *a):
        self._e.record()
        self.pairs.setdefault(self._name, []).append((self._s, self._e))
        return False

    def totals_ms(self):
        torch.cuda.synchronize()
        return {k: [s.elapsed_time(e) for s, e in v] for k, v in self.pairs.items()}


def render(g: V.Gaussians, cams: Sequence, tfs: Sequence[torch.Tensor], opts=None, stream=None,
           capacity: Optional[int] = None, timer=NO_TIMER, want_contrib: bool = False,
           hits: bool = True, shared: bool = False, status: Optional[torch.Tensor] = None,
           l1: Optional[tuple] = None) -> FwdState:
    """Forward render of len(tfs) frames (one model, one image size).

    Frame f uses cams[f] and tfs[f]; with ``shared`` there are len(tfs) // len(cams) tables
    per camera instead, frame v * K + k uses cams[v] and tfs[v * K + k], and a view's frames
    share one projection and key list.  With ``capacity`` None the key-list length is read
    back (one stream synchronisation) and the buffers are sized exactly; otherwise
    ``capacity`` entries are allocated, no synchronisation happens, and an overflow must be
    checked with ``veg_bin_overflow``, or later from ``status`` (device int64 [2], written
    with the entry count and the overflow flag).  ``hits`` records which entries were
    blended anywhere, for a following backward pass (set it False for forward-only
    rendering).  With ``l1`` = (target, scale, loss_slots) the L1 term of the loss is fused
    into the forward pass: ``image`` then holds scale * sign(image - target) (the loss's
    gradient w.r.t. the image) and scale * sum |image - target| is added to loss_slots."""
    o = V.make_opts(opts) if not hasattr(opts, "alpha_clamp") else opts
    dev = g.means.device
    proj = V.alloc_proj(g.n, len(tfs), device=dev)
    ws = V.alloc_bin_workspace(proj, device=dev)
    with timer("project"):
        if shared:
            V.veg_project_views(g, cams, tfs, o, proj=proj, stream=stream)
        else:
            V.veg_project(g, cams, tfs, o, proj=proj, stream=stream)
    with timer("bin_count"):
        V.veg_bin_count(proj, ws, sync=False, stream=stream)
    if capacity is None:
        E, _ = V.veg_bin_overflow(ws, stream=stream)
        cap = E
    else:
        E, cap = -1, int(capacity)
    bins = V.alloc_bins(proj, cap, device=dev, hits=hits)
    with timer("bin_sort"):
        V.veg_bin_sort(proj, ws, bins, stream=stream)
    if status is not None:
        V.veg_bin_status(ws, status, stream=stream)
    F, H, W = len(tfs), int(proj.struct.height), int(proj.struct.width)
    image = torch.empty((F, 3, H, W), dtype=torch.float32, device=dev)
    t_final = torch.empty((F, H, W), dtype=torch.float32, device=dev)
    n_last = torch.empty((F, H, W), dtype=torch.int32, device=dev)
    n_contrib = torch.empty((F, H, W), dtype=torch.int32, device=dev) if want_contrib else None
    with timer("blend_fwd"):
        if l1 is not None and not want_contrib:
            V.veg_render_fwd_l1(proj, bins, o, l1[0], l1[1], l1[2], image, t_final, n_last, stream=stream)
        else:
            V.veg_render_fwd(proj, bins, o, image, t_final, n_last, n_contrib, stream=stream)
            if l1 is not None:
                V.veg_l1_loss(image, l1[0], l1[1], l1[2][:1], image, stream=stream)
    return FwdState(proj, bins, ws, image, t_final, n_last, E, o, n_contrib)


@dataclass
class Grads:
    d_means: torch.Tensor
    d_log_scales: torch.Tensor
    d_quats: torch.Tensor
    d_scalars: torch.Tensor
    d_weights: Optional[torch.Tensor] = None
    d_normals: Optional[torch.Tensor] = None
    d_k_ambient: Optional[torch.Tensor] = None
    d_k_diffuse: Optional[torch.Tensor] = None
    d_k_specular: Optional[torch.Tensor] = None
    d_shininess: Optional[torch.Tensor] = None

    @staticmethod
    def zeros(g: V.Gaussians, stream=None) -> "Grads":
        def z(shape):
            t = torch.empty(shape, dtype=torch.float32, device=g.means.device)
            V.veg_fill_u32(t, 0, stream=stream)
            return t
        n = g.n
        lit = {} if not g.lit else dict(d_normals=z((n, 3)), d_k_ambient=z((n,)), d_k_diffuse=z((n,)),
                                        d_k_specular=z((n,)), d_shininess=z((n,)))
        return Grads(z((n, 3)), z((n, 3)), z((n, 4)), z((n,)), z((n,)) if g.weights is not None else None, **lit)

    @property
    def lighting(self):
        if self.d_normals is None:
            return None
        return (self.d_normals, self.d_k_ambient, self.d_k_diffuse, self.d_k_specular, self.d_shininess)

    def zero_(self, stream=None):
        for t in (self.d_means, self.d_log_scales, self.d_quats, self.d_scalars, self.d_weights) + \
                (self.lighting or ()):
            if t is not None:
                V.veg_fill_u32(t, 0, stream=stream)


def alloc_g2d(proj: V.Proj, stream=None) -> torch.Tensor:
    g2d = torch.empty(max(1, 9 * proj.n_pairs), dtype=torch.float32, device=proj.rec.device)
    V.veg_fill_u32(g2d, 0, stream=stream)
    return g2d


def render_backward(g: V.Gaussians, st: FwdState, d_image: torch.Tensor, grads: Grads, stream=None,
                    g2d: Optional[torch.Tensor] = None, timer=NO_TIMER, densify=None,
                    consume_g2d: bool = False) -> torch.Tensor:
    """Accumulates dL/dparams into ``grads`` given dL/dimage; returns the screen-space g2d.
    ``g2d`` (optional) must hold zeros; with ``consume_g2d`` the projection backward leaves
    it zero again, ready for the next call.  ``densify`` (with grad_accum, vis_count) adds
    the densification statistics from the same pass."""
    if g2d is None:
        with timer("zero_g2d"):
            g2d = alloc_g2d(st.proj, stream=stream)
    elif g2d.numel() < 9 * st.proj.n_pairs:
        raise ValueError("g2d holds fewer than 9 floats per pair")
    with timer("blend_bwd"):
        V.veg_render_bwd(st.proj, st.bins, st.opts, st.t_final, st.n_last, d_image.contiguous(), g2d, stream=stream)
    with timer("project_bwd"):
        if densify is None and not consume_g2d:
            V.veg_project_bwd(g, st.proj, st.opts, g2d, grads.d_means, grads.d_log_scales, grads.d_quats,
                              grads.d_scalars, grads.d_weights, stream=stream, d_lighting=grads.lighting)
        else:
            V.veg_project_bwd_fused(g, st.proj, st.opts, g2d, grads.d_means, grads.d_log_scales, grads.d_quats,
                                    grads.d_scalars, grads.d_weights, stream=stream, d_lighting=grads.lighting,
                                    grad_accum=None if densify is None else densify.grad_accum,
                                    vis_count=None if densify is None else densify.vis_count,
                                    consume_g2d=consume_g2d)
    return g2d


class VEGRender(torch.autograd.Function):
    """image[F,3,H,W] = render(means, log_scales, quats, scalars, weights[, lighting]; cams, tfs).

    ``scalars``, ``weights`` and the lighting coefficients are the activated values (apply
    the sigmoid or other activation before).  ``lighting`` is None or the tuple (normals,
    k_ambient, k_diffuse, k_specular, shininess)."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, scalars, weights, cams, tfs, opts, *lighting):
        def c(t):
            return None if t is None else t.detach().contiguous()
        lit = dict(zip(V.LIGHTING, (c(t) for t in lighting))) if lighting else {}
        g = V.Gaussians(c(means), c(log_scales), c(quats), c(scalars), c(weights), **lit)
        st = render(g, cams, tfs, opts)
        ctx.g = g
        ctx.st = st
        ctx.has_w = weights is not None
        ctx.n_lit = len(lighting)
        return st.image

    @staticmethod
    def backward(ctx, d_image):
        grads = Grads.zeros(ctx.g)
        render_backward(ctx.g, ctx.st, d_image.contiguous(), grads)
        lit = grads.lighting if ctx.n_lit else ()
        return (grads.d_means, grads.d_log_scales, grads.d_quats, grads.d_scalars,
                grads.d_weights if ctx.has_w else None, None, None, None) + tuple(lit)


def render_autograd(means, log_scales, quats, scalars, weights, cams, tfs, opts=None, lighting=None):
    return VEGRender.apply(means, log_scales, quats, scalars, weights, cams, tfs, opts, *(lighting or ()))


@dataclass
class StepResult:
    loss: float
    n_entries: List[int]
    status: Optional[torch.Tensor] = None   # device [groups, 2] (entries, overflow) with a capacity


class KeyListOverflow(RuntimeError):
    """A key list needed more entries than the capacity given for it."""


def check_status(status: torch.Tensor, capacity: int) -> List[int]:
    """Entries per group from a training step's ``status`` (one synchronisation); raises
    KeyListOverflow if a group's key list did not fit ``capacity``."""
    st = status.cpu().tolist()
    bad = [e for e, ov in st if ov]
    if bad:
        raise KeyListOverflow(f"key list of {max(bad)} entries exceeds the capacity {capacity}")
    return [int(e) for e, _ in st]


@dataclass
class DensifyStats:
    """Per-Gaussian accumulators for densification and pruning: the summed norm of
    dL/d(projected centre) over the frames where the Gaussian was kept, and that count."""
    grad_accum: torch.Tensor
    vis_count: torch.Tensor

    @staticmethod
    def zeros(n: int, device="cuda", stream=None) -> "DensifyStats":
        a = torch.empty(max(1, n), dtype=torch.float32, device=device)
        c = torch.empty(max(1, n), dtype=torch.int32, device=device)
        V.veg_fill_u32(a, 0, stream=stream)
        V.veg_fill_u32(c, 0, stream=stream)
        return DensifyStats(a, c)


def views_of(frames: Sequence[tuple]) -> int:
    """Tables per view when ``frames`` is a view-major product (every camera with the same
    tables, in the same order), else 0."""
    if not frames:
        return 0
    K = 1
    while K < len(frames) and frames[K][0] == frames[0][0]:
        K += 1
    if len(frames) % K != 0:
        return 0
    tabs = [t for _, t in frames[:K]]
    for v in range(len(frames) // K):
        blk = frames[v * K:(v + 1) * K]
        if any(c != blk[0][0] for c, _ in blk) or [t for _, t in blk] != tabs:
            return 0
    return K


def train_step(g: V.Gaussians, cams: Sequence, tfs: Sequence[torch.Tensor], frames: Sequence[tuple],
               targets: torch.Tensor, grads: Grads, group: int, opts=None, ssim_lambda: float = 0.0, stream=None,
               loss_acc: Optional[torch.Tensor] = None, read_loss: bool = True, timer=NO_TIMER, on_group=None,
               want_contrib: bool = False, densify: Optional[DensifyStats] = None,
               shared=False, capacity: Optional[int] = None, g2d: Optional[torch.Tensor] = None) -> StepResult:
    """One multi-view x multi-TF training step with the image loss
    (1 - lambda) mean|image - target| + lambda mean(1 - SSIM), means over all frames,
    channels and pixels.

    Frames are processed in groups of ``group``: each group is projected, binned, blended,
    differentiated and its key lists are released before the next group starts, so only
    one group's per-pixel state is alive (forward recomputation per group instead of
    storing all frames' lists).  Both loss terms are separable over frames (SSIM's window
    stays inside one image plane), so the accumulated gradient equals the full-step
    gradient.  With ``densify`` the densification statistics of every group are added.

    With ``shared`` the frames share projections and key lists in runs of K consecutive
    frames that have one camera: ``shared=True`` takes K = all the tables of a view (the
    frames must be a view-major product of cameras and tables), an integer ``shared=K``
    takes runs of K (e.g. neighbouring maps of a tent family, whose footprints overlap).  A
    group is then a whole number of runs (``group`` rounded down to a multiple of K, at
    least one run).

    With ``capacity`` every group's key list gets that many entries and the step runs
    without a host synchronisation until the loss is read (``read_loss``), when the entry
    counts and overflow flags are read with it; a list that did not fit raises
    KeyListOverflow (the gradients of that step are then incomplete).  With ``read_loss``
    False the flags are in ``StepResult.status``, for ``check_status`` later.

    ``g2d`` (optional): a float32 buffer of at least 9 x (pairs of the largest group)
    zeros that the caller keeps between steps; every group's backward uses it and leaves it
    zero, so no clear is needed per group (``alloc_g2d`` sizes one for a projection)."""
    o = V.make_opts(opts) if not hasattr(opts, "alpha_clamp") else opts
    if not 0.0 <= ssim_lambda <= 1.0:
        raise ValueError("ssim_lambda must lie in [0, 1]")
    K = 1
    if shared is True:
        K = views_of(frames)
        if K == 0:
            raise ValueError("shared views need frames ordered as views x the same tables")
    elif shared:
        K = int(shared)
        if K < 1 or len(frames) % K or any(frames[i][0] != frames[i - i % K][0] for i in range(len(frames))):
            raise ValueError("shared runs need K consecutive frames with one camera")
    shared = K > 1 or shared is True
    if shared:
        group = max(K, group // K * K)
    F = len(frames)
    H, W = int(targets.shape[-2]), int(targets.shape[-1])
    M = float(F * 3 * H * W)
    if loss_acc is None:
        loss_acc = torch.empty(1, dtype=torch.float64, device=g.means.device)
    V.veg_fill_u32(loss_acc, 0, stream=stream)
    # With the L1 term alone it is fused into the forward pass (its gradient is written in
    # place of the image, the loss into 64 slots summed at the end of the step).
    fuse_l1 = ssim_lambda == 0.0
    slots = torch.empty(V._lib.VEG_L1_SLOTS, dtype=torch.float64, device=g.means.device) if fuse_l1 else None
    if fuse_l1:
        V.veg_fill_u32(slots, 0, stream=stream)
    entries = []
    ssim_ws = None
    status = None
    if capacity is not None:
        status = torch.empty(((F + group - 1) // group, 2), dtype=torch.int64, device=g.means.device)
    for f0 in range(0, F, group):
        fr = frames[f0:f0 + group]
        view_cams = [cams[c] for c, _ in fr[::K]] if shared else [cams[c] for c, _ in fr]
        tgt = targets[f0:f0 + len(fr)].contiguous()
        st = render(g, view_cams, [tfs[t] for _, t in fr], o, stream=stream, timer=timer,
                    want_contrib=want_contrib, shared=shared, capacity=capacity,
                    status=status[f0 // group] if status is not None else None,
                    l1=(tgt, 1.0 / M, slots) if fuse_l1 else None)
        entries.append(st.n_entries)
        if fuse_l1:
            d_image = st.image
        else:   # L1 and SSIM terms in one pass, d_image written
            d_image = torch.empty_like(st.image)
            with timer("image_loss"):
                ssim_ws = V.veg_image_loss(st.image, tgt, (1.0 - ssim_lambda) / M, ssim_lambda / M, loss_acc,
                                           d_image, ws=ssim_ws, stream=stream)
        # the densification statistics come from the projection backward's g2d reads; a
        # caller-kept g2d buffer is consumed (left zero) instead of cleared for every group
        gbuf = g2d[:max(1, 9 * st.proj.n_pairs)] if g2d is not None else None
        g2d_g = render_backward(g, st, d_image, grads, stream=stream, timer=timer, g2d=gbuf, densify=densify,
                                consume_g2d=g2d is not None)
        if on_group is not None:
            on_group(f0, st)
        del st, d_image, g2d_g
    if fuse_l1:
        torch.sum(slots, 0, keepdim=True, out=loss_acc)
    loss = float(loss_acc.item()) if read_loss else float("nan")
    if status is not None and read_loss:
        entries = check_status(status, capacity)
    return StepResult(loss, entries, status)


def train_step_l1(*args, **kw) -> StepResult:
    """The training step with the L1 term alone (lambda = 0)."""
    kw["ssim_lambda"] = 0.0
    return train_step(*args, **kw)


class Adam:
    """Adam over float32 parameter tensors, each with its own learning rate; one
    veg_adam_step launch per tensor (moments held here, zero-initialised)."""

    def __init__(self, params: Sequence[tuple], betas=(0.9, 0.999), eps: float = 1e-15, stream=None):
        self.params = [(p, float(lr)) for p, lr in params]
        self.betas, self.eps, self.t = betas, float(eps), 0
        self.m = [torch.empty_like(p) for p, _ in self.params]
        self.v = [torch.empty_like(p) for p, _ in self.params]
        for t in self.m + self.v:
            V.veg_fill_u32(t, 0, stream=stream)

    def step(self, grads: Sequence[torch.Tensor], stream=None):
        if len(grads) != len(self.params):
            raise ValueError("one gradient per parameter tensor")
        self.t += 1
        for (p, lr), gr, m, v in zip(self.params, grads, self.m, self.v):
            V.veg_adam_step(p, gr, m, v, lr, self.t, self.betas[0], self.betas[1], self.eps, stream=stream)


def densify_model(g: V.Gaussians, stats: DensifyStats, grad_thresh: float, log_scale_thresh: float,
                  prune_weight: float, z: torch.Tensor, adam: Optional[Adam] = None, stream=None):
    """One densification step: clone, split and prune decisions from ``stats`` (see
    veg_densify_plan), then the new model (see veg_densify_apply); ``z`` [n, 2, 3] holds the
    standard normal draws for split children.  With ``adam`` its parameters are rebound to
    the new tensors and its moments carried over (zero for new Gaussians).  Returns
    (new Gaussians, counts [KEEP, CLONE, SPLIT, PRUNE])."""
    n = g.n
    action, counts, ws = V.veg_densify_plan(stats.grad_accum, stats.vis_count, g.log_scales, g.weights, grad_thresh,
                                            log_scale_thresh, prune_weight, stream=stream)
    n_new = n + counts[V.CLONE] + counts[V.SPLIT] - counts[V.PRUNE]

    def like(t):
        return torch.empty((n_new,) + tuple(t.shape[1:]), dtype=t.dtype, device=t.device)
    names = ("means", "log_scales", "quats", "scalars", "weights") + V.LIGHTING
    out, fields = {}, []
    for name in names:
        t = getattr(g, name)
        if t is None:
            continue
        out[name] = like(t)
        role = V.FIELD_MEANS if name == "means" else V.FIELD_LOG_SCALES if name == "log_scales" else V.FIELD_COPY
        fields.append((t, out[name], role))
    V.veg_densify_apply(action, g.quats, g.log_scales, z, fields, ws, stream=stream)
    if adam is not None:
        params, moms = [], []
        for (p, lr), m, v in zip(adam.params, adam.m, adam.v):
            name = next(k for k in out if getattr(g, k) is p)
            nm, nv = like(m), like(v)
            moms += [(m, nm, V.FIELD_ZERO_NEW), (v, nv, V.FIELD_ZERO_NEW)]
            params.append((out[name], lr, nm, nv))
        for k in range(0, len(moms), 16):
            V.veg_densify_apply(action, g.quats, g.log_scales, z, moms[k:k + 16], ws, stream=stream)
        adam.params = [(p, lr) for p, lr, _, _ in params]
        adam.m = [m for _, _, m, _ in params]
        adam.v = [v for _, _, _, v in params]
    return V.Gaussians(**out), counts
