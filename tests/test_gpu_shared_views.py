"""Views rendered with several transfer functions that share one projection and key list
(veg_project_views): the list and records bit-exact against the oracle's shared-footprint
mirror, every frame's image and gradients against the per-frame oracle, and the training
step against the same step without sharing."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import compare_image, hip, image_pixels, luts_to_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

OPTS = dict(synth.DEFAULT_OPTS)


def _case(n=3000, views=2, K=3, res=80, tents=False):
    w = synth.workload(1, n_override=n, views_override=views, tfs_override=K, res_override=res)
    if tents:
        w.tfs = synth.tent_tfs(K)
    return w


def _render_shared(w, contrib=False):
    V, R = hip()
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    st = R.render(g, w.cameras, [luts[t] for _, t in w.frames], OPTS, shared=True, want_contrib=contrib)
    torch.cuda.synchronize()
    return g, luts, st


def _rects(r):
    r01, r23 = r[:, 9].view(np.uint32), r[:, 10].view(np.uint32)
    return np.stack([r01 & 0xFFFF, r01 >> 16, r23 & 0xFFFF, r23 >> 16], 1).astype(np.int64)


@pytest.mark.parametrize("K,tents", [(3, False), (10, True), (1, False)])
def test_shared_key_list_and_records_bit_exact(K, tents):
    w = _case(K=K, tents=tents)
    g, luts, st = _render_shared(w)
    assert int(st.proj.struct.tfs_per_view) == K
    n, F = w.gaussians.n, len(w.frames)
    count = st.proj.count.cpu().numpy().view(np.uint32)[: n * F].astype(np.int64).reshape(F, n)
    depth = st.proj.depth.cpu().numpy().view(np.uint32)[: n * F].reshape(F, n)
    rec = st.proj.rec.cpu().numpy()[: n * F * 12].reshape(F, n, 12)
    fps = []
    geo = [0, 1, 2, 3, 4, 9, 10]
    for v, cam in enumerate(w.cameras):
        un = oracle.footprint_shared_f32(w.gaussians, cam, w.tfs, OPTS)
        kept = un.count > 0
        o = v * K
        assert np.array_equal(count[o], un.count), f"view {v}: shared tile counts differ"
        assert np.array_equal(depth[o][kept], un.depth_bits[kept])
        assert np.array_equal(_rects(rec[o][kept]), un.rect[kept])
        if K > 1:   # keep bits of the view's frames, in the depth slots of its second frame
            bits = np.zeros(n, np.int64)
            for k in range(K):
                own_k = oracle.footprint_f32(w.gaussians, cam, w.tfs[k], OPTS)
                bits |= own_k.keep.astype(np.int64) << min(k, 31)
            assert np.array_equal(depth[o + 1][kept].astype(np.int64), bits[kept])
        for k in range(K):
            f = o + k
            if k > 0:
                assert not count[f].any(), f"frame {f}: only the list owner is counted"
            fps.append(un if k == 0 else dataclasses.replace(un, count=np.zeros_like(un.count),
                                                               keep=np.zeros_like(un.keep)))
            r = rec[f][kept]
            assert np.array_equal(np.ascontiguousarray(r[:, geo]).view(np.uint32),
                                  np.ascontiguousarray(rec[o][kept][:, geo]).view(np.uint32))
            # the frame's own A where its own footprint keeps the Gaussian, else 0
            own = oracle.footprint_f32(w.gaussians, cam, w.tfs[k], OPTS)
            a_ref = np.where(own.keep[kept], own.A[kept], np.float32(0)).astype(np.float32)
            assert np.array_equal(r[:, 5], a_ref), f"frame {f}: per-frame A"
            assert np.all(own.keep <= kept)
            word = r[:, 11].view(np.uint32)
            assert np.array_equal(word & 0xFFF, np.full(kept.sum(), f, np.uint32))
            # the frame's own tile rectangle as insets from the shared one (0 where culled or
            # when the view has one table), each clamped to [0, 31]
            ur, orr = un.rect[kept].astype(np.int64), own.rect[kept].astype(np.int64)
            ins = np.stack([orr[:, 0] - ur[:, 0], orr[:, 1] - ur[:, 1], ur[:, 2] - orr[:, 2],
                            ur[:, 3] - orr[:, 3]], 1).clip(0, 31)
            ins[~own.keep[kept] | (K == 1)] = 0
            ref = (ins[:, 0] | (ins[:, 1] << 5) | (ins[:, 2] << 10) | (ins[:, 3] << 15)).astype(np.uint32)
            assert np.array_equal(word >> 12, ref), f"frame {f}: own-rectangle insets"
    # tiles are numbered per view; the oracle's list over the owners (one per view) gives
    # pair ids v * n + i, the library's owner pairs are (v K) * n + i
    tiles, depths, pairs, ranges, _ = oracle.key_list(fps[::K], list(w.cameras))
    pairs = pairs // n * (K * n) + pairs % n
    E = tiles.shape[0]
    assert st.n_entries == E
    assert np.array_equal(st.bins.keys.cpu().numpy().view(np.uint32)[:E].astype(np.int64), tiles)
    assert np.array_equal(st.bins.vals.cpu().numpy().view(np.uint32)[:E].astype(np.int64), pairs)
    rg = st.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    assert np.array_equal(rg, ranges)


@pytest.mark.parametrize("K,tents,views", [(3, False, 2), (10, True, 1), (5, True, 2)])
def test_shared_images_match_oracle(K, tents, views):
    w = _case(n=2000, K=K, tents=tents, res=64, views=views)
    g, luts, st = _render_shared(w)
    for f, (ci, ti) in enumerate(w.frames):
        res, *_ = oracle.render_image(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS)
        compare_image(image_pixels(st.image[f]), res)


def test_shared_blend_counts_equal_unshared():
    """Blended-entry counts per pixel: a frame on a shared list blends what it blends on its
    own list; only the centre's rounding differs, so almost every pixel matches the
    unshared render exactly."""
    V, R = hip()
    w = _case(n=3000, K=4, res=96)
    g, luts, st = _render_shared(w, contrib=True)
    ref = R.render(g, [w.cameras[c] for c, _ in w.frames], [luts[t] for _, t in w.frames], OPTS, want_contrib=True)
    torch.cuda.synchronize()
    same = (st.n_contrib == ref.n_contrib).float().mean().item()
    assert same >= 0.999
    assert (st.image - ref.image).abs().max().item() <= 1e-3
    assert ((st.image - ref.image).abs() > 1e-5).float().mean().item() <= 1e-3


def test_shared_gradients_match_oracle():
    V, R = hip()
    w = _case(n=2000, K=3, res=64)
    g, luts, st = _render_shared(w)
    _check_backward(w, g, st)


def _check_backward(w, g, st):
    V, R = hip()
    F, H, W = len(w.frames), w.width, w.height
    rng = np.random.default_rng(91)
    d_all = np.zeros((F, 3, H, W), np.float32)
    acc = None
    for f, (ci, ti) in enumerate(w.frames):
        res, *_ = oracle.render_image(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS)
        d = rng.standard_normal((H * W, 3)).astype(np.float32).astype(np.float64)
        d[res.flag | res.flag_grad] = 0.0
        d_all[f] = d.T.reshape(3, H, W)
        gr = oracle.gradients(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS, d)
        cur = {k: getattr(gr, k) for k in ("d_means", "d_log_scales", "d_quats", "d_scalars")}
        acc = cur if acc is None else {k: acc[k] + cur[k] for k in acc}
    grads = R.Grads.zeros(g)
    R.render_backward(g, st, torch.as_tensor(d_all).cuda(), grads)
    torch.cuda.synchronize()
    for k, ref in acc.items():
        assert rel_err(getattr(grads, k).cpu().numpy(), ref) <= 1e-3, k


def test_shared_backward_without_hit_bits_matches_oracle():
    """Without hit bits the backward pass walks the whole shared list and must drop the
    same entries the forward pass dropped for the frame."""
    V, R = hip()
    w = _case(n=2000, K=4, res=64, tents=True)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    st = R.render(g, w.cameras, [luts[t] for _, t in w.frames], OPTS, shared=True, hits=False)
    torch.cuda.synchronize()
    assert st.bins.hits is None
    _check_backward(w, g, st)


def test_shared_train_step_matches_unshared():
    """Loss (1 - 0.2) L1 + 0.2 (1 - SSIM) over 3 views x 2 tables in groups of two views;
    a frame of a shared view keeps exactly the Gaussians its own footprint keeps, so the
    visibility counts are equal."""
    V, R = hip()
    w = _case(n=4000, views=3, K=2, res=80)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    rng = np.random.default_rng(92)
    tgt = torch.as_tensor(rng.uniform(0, 1, (len(w.frames), 3, 80, 80)).astype(np.float32)).cuda()
    out = {}
    for shared in (False, True):
        grads = R.Grads.zeros(g)
        dens = R.DensifyStats.zeros(w.gaussians.n)
        res = R.train_step(g, w.cameras, luts, w.frames, tgt, grads, 4, OPTS, ssim_lambda=0.2, densify=dens,
                           shared=shared)
        torch.cuda.synchronize()
        out[shared] = (res.loss, {k: getattr(grads, k).cpu().numpy() for k in
                                  ("d_means", "d_log_scales", "d_quats", "d_scalars")},
                       dens.vis_count.cpu().numpy())
    assert abs(out[True][0] - out[False][0]) <= 1e-5 * abs(out[False][0])
    for k, v in out[True][1].items():
        assert rel_err(v, out[False][1][k]) <= 1e-3, k
    assert np.array_equal(out[True][2], out[False][2])



def test_shared_view_with_a_table_that_culls_everything():
    """A zero-opacity table in the middle of a view: its frame is background everywhere and
    adds nothing to any gradient; the other frames match the oracle."""
    V, R = hip()
    w = _case(n=2000, K=3, res=64, views=1)
    w.tfs[1] = synth.constant_tf(rgba=(0.3, 0.6, 0.9, 0.0))
    g, luts, st = _render_shared(w)
    bg = np.array(OPTS["bg"], np.float32)
    assert np.array_equal(st.image[1].cpu().numpy(), np.broadcast_to(bg[:, None, None], (3, 64, 64)))
    assert bool((st.t_final[1] == 1.0).all()) and bool((st.n_last[1] == -1).all())
    for f in (0, 2):
        res, *_ = oracle.render_image(w.gaussians, w.cameras[0], w.tfs[f], OPTS)
        compare_image(image_pixels(st.image[f]), res)
    d = torch.zeros_like(st.image)
    d[1] = 1.0                                     # only the culled frame has a loss gradient
    grads = R.Grads.zeros(g)
    R.render_backward(g, st, d, grads)
    torch.cuda.synchronize()
    assert float(grads.d_means.abs().max()) == 0.0 and float(grads.d_scalars.abs().max()) == 0.0


def test_one_table_per_view_is_the_plain_projection_bit_for_bit():
    """veg_project_views with one table per view takes exactly veg_project's path."""
    V, R = hip()
    w = _case(n=3000, K=1, res=80, views=3)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    a = R.render(g, w.cameras, [luts[t] for _, t in w.frames], OPTS, shared=True)
    b = R.render(g, [w.cameras[c] for c, _ in w.frames], [luts[t] for _, t in w.frames], OPTS)
    torch.cuda.synchronize()
    assert torch.equal(a.image, b.image) and torch.equal(a.n_last, b.n_last)
    assert torch.equal(a.proj.count, b.proj.count)
    kept = a.proj.count[: a.proj.n_pairs] > 0          # records exist for counted pairs only
    ra, rb = a.proj.rec.view(-1, 12)[: a.proj.n_pairs], b.proj.rec.view(-1, 12)[: b.proj.n_pairs]
    assert torch.equal(ra[kept], rb[kept])
    assert a.n_entries == b.n_entries and torch.equal(a.bins.keys[:a.n_entries], b.bins.keys[:b.n_entries])
    assert torch.equal(a.bins.vals[:a.n_entries], b.bins.vals[:b.n_entries])


def test_shared_views_with_lighting_match_oracle():
    """Blinn-Phong shading on a shared list: each frame shades its own table's colour under
    the view's headlight."""
    V, R = hip()
    w = _case(n=2000, K=3, res=64, views=1)
    w.gaussians.shading = synth.random_shading(synth.rng_for(0, 93), w.gaussians.n)
    g, luts, st = _render_shared(w)
    assert g.lit
    for f, (ci, ti) in enumerate(w.frames):
        res, *_ = oracle.render_image(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS)
        compare_image(image_pixels(st.image[f]), res)


def test_train_step_sharing_in_runs_of_two_matches_own_lists():
    """Tent maps shared by neighbouring pairs (shared=2) against every frame on its own list:
    same loss and gradients up to the centre's rounding, same visibility counts."""
    V, R = hip()
    w = _case(n=4000, views=2, K=4, res=80, tents=True)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    rng = np.random.default_rng(94)
    tgt = torch.as_tensor(rng.uniform(0, 1, (len(w.frames), 3, 80, 80)).astype(np.float32)).cuda()
    out = {}
    for shared in (False, 2):
        grads = R.Grads.zeros(g)
        dens = R.DensifyStats.zeros(w.gaussians.n)
        res = R.train_step(g, w.cameras, luts, w.frames, tgt, grads, 8, OPTS, densify=dens, shared=shared)
        torch.cuda.synchronize()
        out[shared] = (res.loss, {k: getattr(grads, k).cpu().numpy() for k in ("d_means", "d_scalars")},
                       dens.vis_count.cpu().numpy())
    assert abs(out[2][0] - out[False][0]) <= 1e-5 * abs(out[False][0])
    for k, v in out[2][1].items():
        assert rel_err(v, out[False][1][k]) <= 1e-3, k
    assert np.array_equal(out[2][2], out[False][2])


def test_views_of_more_than_32_tables_keep_every_frame_from_slot_31():
    """The keep bits hold 32 frames; from slot 31 on every frame reads bit 31, which a view of
    more than 32 frames sets for every Gaussian, so those frames are never filtered by it."""
    V, R = hip()
    w = _case(n=800, views=1, K=34, res=48, tents=True)
    g, luts, st = _render_shared(w)
    for f in (0, 30, 31, 32, 33):
        ci, ti = w.frames[f]
        res, *_ = oracle.render_image(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS)
        compare_image(image_pixels(st.image[f]), res)


def test_densify_visibility_on_a_view_of_34_tables_equals_own_lists():
    """Densification visibility on a shared list reads the view's keep bits for slots 0-30
    and the frame's record from slot 31 on: counts equal the own-list run's exactly."""
    V, R = hip()
    w = _case(n=800, views=1, K=34, res=48, tents=True)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    rng = np.random.default_rng(95)
    tgt = torch.as_tensor(rng.uniform(0, 1, (len(w.frames), 3, 48, 48)).astype(np.float32)).cuda()
    vis = {}
    for shared in (False, True):
        grads = R.Grads.zeros(g)
        dens = R.DensifyStats.zeros(w.gaussians.n)
        R.train_step(g, w.cameras, luts, w.frames, tgt, grads, 34, OPTS, densify=dens, shared=shared)
        torch.cuda.synchronize()
        vis[shared] = dens.vis_count.cpu().numpy()
    assert vis[False].sum() > 0
    assert np.array_equal(vis[True], vis[False])


@pytest.mark.parametrize("K,tents,views", [(1, False, 2), (3, False, 2), (34, True, 1)])
def test_fused_projection_backward_equals_the_separate_passes(K, tents, views):
    """veg_project_bwd_fused: parameter gradients and densification statistics bit for bit
    those of veg_project_bwd followed by veg_densify_stats (own lists, a view of three
    tables, a view of 34 tent maps whose slots from 31 on test the record), and the consumed
    g2d left all zero."""
    V, R = hip()
    w = _case(n=1500, views=views, K=K, res=64, tents=tents)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    cams = w.cameras if K > 1 else [w.cameras[c] for c, _ in w.frames]
    st = R.render(g, cams, [luts[t] for _, t in w.frames], OPTS, shared=K > 1)
    rng = np.random.default_rng(41)
    d_img = torch.as_tensor(rng.standard_normal(tuple(st.image.shape)).astype(np.float32)).cuda()
    g2d = R.alloc_g2d(st.proj)
    V.veg_render_bwd(st.proj, st.bins, st.opts, st.t_final, st.n_last, d_img, g2d)
    g2d_b = g2d.clone()
    n = w.gaussians.n
    ga, da = R.Grads.zeros(g), R.DensifyStats.zeros(n)
    V.veg_project_bwd(g, st.proj, st.opts, g2d, ga.d_means, ga.d_log_scales, ga.d_quats, ga.d_scalars, ga.d_weights)
    V.veg_densify_stats(st.proj, g2d, da.grad_accum, da.vis_count)
    gb, db = R.Grads.zeros(g), R.DensifyStats.zeros(n)
    V.veg_project_bwd_fused(g, st.proj, st.opts, g2d_b, gb.d_means, gb.d_log_scales, gb.d_quats, gb.d_scalars,
                            gb.d_weights, grad_accum=db.grad_accum, vis_count=db.vis_count, consume_g2d=True)
    torch.cuda.synchronize()
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars", "d_weights"):
        a, b = getattr(ga, name), getattr(gb, name)
        if a is not None:
            assert torch.equal(a, b), name
    assert torch.equal(da.grad_accum, db.grad_accum)
    assert torch.equal(da.vis_count, db.vis_count) and int(da.vis_count.sum()) > 0
    assert float(g2d.abs().sum()) > 0 and not bool(g2d_b.any())
