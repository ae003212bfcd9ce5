"""Parity of the HIP path (called through the C ABI) with the CPU oracle.

Bars: integer outputs (cull, tile counts, depth keys, tile rectangles, sorted key list,
per-tile ranges) bit-exact against the oracle's float32 footprint mirror; images within
1e-4 max-abs per channel of the float64 brute-force oracle on pixels without a
decision-margin flag; gradients within 1e-3 relative (max-abs error over max-abs value,
per parameter tensor) of the oracle's float64 autograd adjoint.
"""
import types

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import all_pixels, compare_image, hip, image_pixels, luts_to_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu
OPTS = dict(synth.DEFAULT_OPTS)


def _run(g_np, cams, tfs, opts=OPTS):
    V, R = hip()
    g = to_dev(g_np)
    st = R.render(g, cams, luts_to_dev(tfs), opts)
    torch.cuda.synchronize()
    return g, st


# ----------------------------------------------------------------------------- device helpers

def test_device_float32_helpers_are_bitwise_equal_to_the_mirror():
    V, _ = hip()
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(-87, 88, 300000), rng.uniform(-6, -2, 100000), np.linspace(-87, 87.99, 100001),
                        [0.0, -0.0, 1.0, -1.0, 88.0, 87.999, -87.0, -87.0001, 1e-30, -1e-30]]).astype(np.float32)
    got = V.veg_debug_math(0, torch.as_tensor(x).cuda()).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), oracle.exp32(x).view(np.uint32))
    y = np.concatenate([np.exp(rng.uniform(-80, 80, 300000)), rng.uniform(1, 255, 200000),
                        [1.0, 2.0, 255.0, 1.0000001, 1.4142135, 1.4142136, 1e-37]]).astype(np.float32)
    got = V.veg_debug_math(1, torch.as_tensor(y).cuda()).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), oracle.log32(y).view(np.uint32))
    a = rng.standard_normal(200000).astype(np.float32) * np.float32(1e3)
    b = (rng.standard_normal(200000).astype(np.float32) + np.float32(0.01))
    got = V.veg_debug_math(2, torch.as_tensor(a).cuda(), torch.as_tensor(b).cuda()).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), (a / b).view(np.uint32))
    s = np.abs(a) + np.float32(1e-20)
    got = V.veg_debug_math(3, torch.as_tensor(s).cuda()).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), np.sqrt(s).view(np.uint32))


def test_wave_prefix_sum_and_reduction():
    V, _ = hip()
    rng = np.random.default_rng(12)
    n = 64 * 37
    u = rng.integers(0, 1000, n).astype(np.uint32)
    got = V.veg_debug_math(4, torch.as_tensor(u.view(np.float32)).cuda()).cpu().numpy().view(np.uint32)
    ref = np.cumsum(u.reshape(-1, 64).astype(np.uint64), axis=1).astype(np.uint32).reshape(-1)
    assert np.array_equal(got, ref)
    f = rng.standard_normal(n).astype(np.float32)
    got = V.veg_debug_math(5, torch.as_tensor(f).cuda()).cpu().numpy().reshape(-1, 64)[:, 63]
    assert np.allclose(got, f.reshape(-1, 64).astype(np.float64).sum(1), atol=1e-4)


# ----------------------------------------------------------------------------- projection and keys

def _proj_arrays(st, n, n_frames):
    count = st.proj.count.cpu().numpy().view(np.uint32)[: n * n_frames].astype(np.int64)
    depth = st.proj.depth.cpu().numpy().view(np.uint32)[: n * n_frames]
    rec = st.proj.rec.cpu().numpy()[: n * n_frames * 12].reshape(-1, 12)
    return count, depth, rec


def _check_footprint(w, st, frames):
    n = w.gaussians.n
    count, depth, rec = _proj_arrays(st, n, len(frames))
    for f, (ci, ti) in enumerate(frames):
        fp = oracle.footprint_f32(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS)
        c = count[f * n:(f + 1) * n]
        assert np.array_equal(c, fp.count), f"frame {f}: tile counts differ at {np.nonzero(c != fp.count)[0][:10]}"
        k = fp.count > 0
        assert np.array_equal(depth[f * n:(f + 1) * n][k], fp.depth_bits[k])
        r = rec[f * n:(f + 1) * n][k]
        rect01 = r[:, 9].view(np.uint32)
        rect23 = r[:, 10].view(np.uint32)
        rect = np.stack([rect01 & 0xFFFF, rect01 >> 16, rect23 & 0xFFFF, rect23 >> 16], 1).astype(np.int64)
        assert np.array_equal(rect, fp.rect[k])
        assert np.array_equal(r[:, 11].view(np.uint32), np.full(k.sum(), f, np.uint32))
        # float fields against the float64 projection
        proj = oracle.project_f64(w.gaussians.means, w.gaussians.log_scales, w.gaussians.quats, w.gaussians.scalars,
                                  w.gaussians.weights, w.cameras[ci], w.tfs[ti], OPTS)
        mx = r[:, 0].astype(np.float64) + 16.0 * rect[:, 0]
        my = r[:, 1].astype(np.float64) + 16.0 * rect[:, 1]
        m2 = proj.mean2d.detach().numpy()[k]
        assert np.abs(mx - m2[:, 0]).max() < 2e-5 and np.abs(my - m2[:, 1]).max() < 2e-5
        con = proj.conic.detach().numpy()[k]
        got = r[:, 2:5].astype(np.float64)
        assert (np.abs(got - con) / np.abs(con).max(1, keepdims=True)).max() < 2e-5
        assert np.abs(r[:, 5] - proj.A.detach().numpy()[k]).max() < 1e-6
        assert np.abs(r[:, 6:9] - proj.rgb.detach().numpy()[k]).max() < 1e-6


def _check_keys(w, st, frames):
    n = w.gaussians.n
    fps = [oracle.footprint_f32(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS) for ci, ti in frames]
    tiles, depths, pairs, ranges, _ = oracle.key_list(fps, [w.cameras[ci] for ci, _ in frames])
    E = tiles.shape[0]
    assert st.n_entries == E
    keys = st.bins.keys.cpu().numpy().view(np.uint32)[:E].astype(np.int64)
    vals = st.bins.vals.cpu().numpy().view(np.uint32)[:E].astype(np.int64)
    assert np.array_equal(keys, tiles)
    assert np.array_equal(vals, pairs)
    rg = st.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    assert np.array_equal(rg, ranges)


@pytest.mark.parametrize("case", ["c0", "c1_small", "odd_size", "large_2048x2000", "large_2064x2000", "wide_depth"])
def test_projection_and_key_list_bit_exact(case):
    """Small frames, a ragged one, two frames of 16,000 and 16,125 tiles (14-bit tile ids,
    two tile-id passes), and cameras inside the scene's extent, whose kept depth keys span
    more than 2^24 (every depth-key pass runs; the other scenes span less, and their key
    lists come from the passes below bit 24 alone)."""
    if case == "c0":
        w = synth.workload(0)
    elif case == "c1_small":
        w = synth.workload(1, n_override=20000, views_override=3, tfs_override=2, res_override=200)
    elif case in ("large_2048x2000", "large_2064x2000"):
        w = synth.workload(1, n_override=20000, views_override=2, tfs_override=1, res_override=200)
        width = 2048 if case == "large_2048x2000" else 2064
        w.cameras = [synth.look_at_camera(d, 3.0, width, 2000) for d in synth.fibonacci_directions(2)]
    elif case == "wide_depth":
        w = synth.workload(0, n_override=3000)
        w.cameras = [synth.look_at_camera(d, 1.0, 160, 120) for d in synth.fibonacci_directions(2)]
        bits = [oracle.footprint_f32(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS) for ci, ti in w.frames]
        span = max(int(fp.depth_bits[fp.count > 0].max()) - int(fp.depth_bits[fp.count > 0].min()) for fp in bits)
        assert span >= 1 << 24, span
    else:
        w = synth.workload(0, n_override=3000)
        w.cameras = [synth.look_at_camera(synth.random_direction(synth.rng_for(0, 7)), 2.5, 97, 61)]
    frames = w.frames
    g, st = _run(w.gaussians, [w.cameras[c] for c, _ in frames], [w.tfs[t] for _, t in frames])
    _check_footprint(w, st, frames)
    _check_keys(w, st, frames)


# ----------------------------------------------------------------------------- forward image

def _frame_result(w, ci, ti, pixels=None):
    return oracle.render_image(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS, pixels=pixels)


def test_forward_image_c0_full_frame():
    w = synth.workload(0)
    g, st = _run(w.gaussians, w.cameras, w.tfs)
    res, proj, order, fp = _frame_result(w, 0, 0)
    gpu = image_pixels(st.image[0])
    emax, frac = compare_image(gpu, res)
    # transmittance and the last blended Gaussian agree on unflagged pixels
    T = st.t_final[0].reshape(-1).cpu().numpy()
    ok = ~res.flag
    assert np.abs(T - res.T.detach().numpy())[ok].max() <= 1e-5
    nl = st.n_last[0].reshape(-1).cpu().numpy()
    vals = st.bins.vals.cpu().numpy().view(np.uint32)
    gpu_last = np.where(nl >= 0, vals[np.maximum(nl, 0)].astype(np.int64) % w.gaussians.n, -1)
    ref_last = np.where(res.last >= 0, order[np.maximum(res.last, 0)], -1)
    assert np.array_equal(gpu_last[ok], ref_last[ok])


def test_forward_is_deterministic():
    w = synth.workload(1, n_override=20000, views_override=2, tfs_override=2, res_override=160)
    frames = w.frames
    _, a = _run(w.gaussians, [w.cameras[c] for c, _ in frames], [w.tfs[t] for _, t in frames])
    _, b = _run(w.gaussians, [w.cameras[c] for c, _ in frames], [w.tfs[t] for _, t in frames])
    assert torch.equal(a.image, b.image) and torch.equal(a.n_last, b.n_last)


def test_forward_dense_scene_with_early_stop():
    """Dense opacity so many pixels stop early; still <= 1e-4 off unflagged pixels."""
    w = synth.workload(0, n_override=6000)
    lut = w.tfs[0].copy()
    lut[:, 3] = np.maximum(lut[:, 3], 0.6)
    w.tfs = [lut]
    g, st = _run(w.gaussians, w.cameras, w.tfs)
    res, *_ = _frame_result(w, 0, 0)
    assert (res.T.detach().numpy() < 1e-4).mean() > 0.05
    compare_image(image_pixels(st.image[0]), res)


def test_forward_with_weights_and_background():
    w = synth.workload(0, n_override=2000)
    w.gaussians.weights = synth.rng_for(0, 3).uniform(0.2, 1.0, w.gaussians.n).astype(np.float32)
    opts = dict(OPTS, bg=(0.2, 0.5, 1.0))
    V, R = hip()
    g = to_dev(w.gaussians)
    st = R.render(g, w.cameras, luts_to_dev(w.tfs), opts)
    res, *_ = oracle.render_image(w.gaussians, w.cameras[0], w.tfs[0], opts, bg=opts["bg"])
    compare_image(image_pixels(st.image[0]), res)


def test_forward_c1_frames_sampled_pixels():
    """Two frames of the 200k-Gaussian, 800x800 workload at its real size; 512 sampled pixels each."""
    w = synth.workload(1)
    frames = [(0, 0), (5, 3)]
    g, st = _run(w.gaussians, [w.cameras[c] for c, _ in frames], [w.tfs[t] for _, t in frames])
    rng = synth.rng_for(1, 50)
    for f, (ci, ti) in enumerate(frames):
        px = synth.sample_pixels(rng, 800, 800, 512)
        res, *_ = _frame_result(w, ci, ti, pixels=px)
        gpu_all = image_pixels(st.image[f])
        gpu = gpu_all[px[:, 1] * 800 + px[:, 0]]
        compare_image(gpu, res)


# ----------------------------------------------------------------------------- edge cases

def _tiny(means, scales, v, W=40, H=24, lut=None, w=None):
    g = synth.Gaussians(np.asarray(means, np.float32), np.log(np.asarray(scales, np.float64)).astype(np.float32),
                        np.tile(np.array([[1, 0, 0, 0]], np.float32), (len(means), 1)), np.asarray(v, np.float32),
                        None if w is None else np.asarray(w, np.float32))
    cam = synth.Camera(view=np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3.0], np.float32), fx=30.0, fy=30.0,
                       cx=W / 2, cy=H / 2, width=W, height=H)
    return g, cam, (synth.identity_tf() if lut is None else lut)


def test_empty_model_gives_background():
    V, R = hip()
    g = synth.Gaussians(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32),
                        np.zeros(0, np.float32))
    cam = synth.Camera(view=np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3.0], np.float32), fx=30.0, fy=30.0, cx=20,
                       cy=12, width=40, height=24)
    opts = dict(OPTS, bg=(0.1, 0.2, 0.3))
    st = R.render(to_dev(g), [cam], luts_to_dev([synth.identity_tf()]), opts)
    img = st.image.cpu().numpy()
    assert st.n_entries == 0
    assert np.allclose(img[0, 0], 0.1) and np.allclose(img[0, 2], 0.3)
    assert (st.t_final.cpu().numpy() == 1.0).all() and (st.n_last.cpu().numpy() == -1).all()


def test_all_culled_and_non_finite_inputs():
    V, R = hip()
    g, cam, lut = _tiny([[0, 0, 0], [0.1, 0, 0], [0, 0.1, -2.9], [np.nan, 0, 0]], [[0.1] * 3] * 4, [0.5] * 4)
    lut = lut.copy()
    lut[:, 3] = 0.001   # every A < 1/255
    st = R.render(to_dev(g), [cam], luts_to_dev([lut]), OPTS)
    assert st.n_entries == 0
    assert (st.image.cpu().numpy() == 0).all()
    # non-finite Gaussian next to a visible one: the visible one renders, the NaN one is culled
    g2, cam2, lut2 = _tiny([[0, 0, 0], [np.nan, 0, 0], [0, np.inf, 0]], [[0.1] * 3] * 3, [0.7] * 3)
    st2 = R.render(to_dev(g2), [cam2], luts_to_dev([lut2]), OPTS)
    cnt = st2.proj.count.cpu().numpy()[:3]
    assert cnt[0] > 0 and cnt[1] == 0 and cnt[2] == 0
    res, *_ = oracle.render_image(g2.subset([0]), cam2, lut2, OPTS)
    compare_image(image_pixels(st2.image[0]), res)


@pytest.mark.parametrize("n_list", [1, 63, 64, 65, 255, 256, 257, 700])
def test_tile_list_lengths_around_batch_boundaries(n_list):
    """n_list Gaussians stacked on the axis at distinct depths, all covering the centre
    tiles: exercises partial, exact and multiple LDS batches."""
    V, R = hip()
    rng = np.random.default_rng(n_list)
    z = np.linspace(-1.0, 1.0, n_list)
    means = np.stack([rng.uniform(-0.01, 0.01, n_list), rng.uniform(-0.01, 0.01, n_list), z], 1)
    lut = synth.identity_tf().copy()
    lut[:, 3] = 0.02   # faint, so the lists are walked to the end
    g, cam, _ = _tiny(means, [[0.05] * 3] * n_list, rng.uniform(0, 1, n_list), lut=lut)
    st = R.render(to_dev(g), [cam], luts_to_dev([lut]), OPTS)
    res, *_ = oracle.render_image(g, cam, lut, OPTS)
    compare_image(image_pixels(st.image[0]), res)
    rg = st.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert (rg[:, 1] - rg[:, 0]).max() == n_list


def test_gaussian_larger_than_the_image():
    V, R = hip()
    g, cam, lut = _tiny([[0, 0, 0]], [[3.0, 2.0, 1.0]], [0.6], W=70, H=45)
    st = R.render(to_dev(g), [cam], luts_to_dev([lut]), OPTS)
    assert st.proj.count.cpu().numpy()[0] == 5 * 3
    res, *_ = oracle.render_image(g, cam, lut, OPTS)
    compare_image(image_pixels(st.image[0]), res)


def test_key_list_with_tile_rows_wider_than_a_digit():
    """A 4160-pixel-wide frame (260 tile columns, 780 tiles, so the first tile-id pass takes 8
    bits) with a Gaussian whose footprint covers every column: its tile rows hold more tiles
    than a digit has values, which the emission's digit histogram counts as whole turns of
    the 256 bins.  Key list and ranges bit for bit against the oracle."""
    g, cam, lut = _tiny([[0, 0, 0], [0.5, 0, 0], [-1.0, 0.1, 0]], [[150.0, 0.3, 1.0], [0.05] * 3, [0.2, 0.1, 0.1]],
                        [0.9, 0.6, 0.7], W=4160, H=40)
    fp = oracle.footprint_f32(g, cam, lut, OPTS)
    assert fp.rect[0, 2] - fp.rect[0, 0] + 1 >= 256
    w = types.SimpleNamespace(gaussians=g, cameras=[cam], tfs=[lut])
    _, st = _run(g, [cam], [lut])
    _check_footprint(w, st, [(0, 0)])
    _check_keys(w, st, [(0, 0)])


@pytest.mark.parametrize("W,H", [(1, 1), (300, 1), (1, 200)])
def test_degenerate_frame_shapes(W, H):
    """Frames of one pixel, one row and one column (a single tile, or one row or column of
    mostly empty tiles): footprints, key list and ranges bit for bit, every pixel of the image
    and the gradients of the screen-space quantities and of the parameters against the
    oracle.  The single pixel reaches the transmittance stop."""
    w = synth.workload(0, n_override=3000)
    w.cameras = [synth.look_at_camera(synth.fibonacci_directions(2)[0], 2.5, W, H)]
    w.tfs = w.tfs[:1]
    _, st = _run(w.gaussians, w.cameras, w.tfs)
    _check_footprint(w, st, [(0, 0)])
    _check_keys(w, st, [(0, 0)])
    d = np.random.default_rng(23).standard_normal((W * H, 3))
    st, grads, g2d, ref = _grads_case(w, d)
    res, *_ = _frame_result(w, 0, 0)
    compare_image(image_pixels(st.image[0]), res)
    n = w.gaussians.n
    g2 = g2d.cpu().numpy().reshape(-1, 9)[:n].T
    assert np.abs(ref.d_rgb).max() > 0.0
    assert rel_err(g2[0:2].T, ref.d_mean2d) <= 1e-3
    assert rel_err(g2[2:5].T, ref.d_conic) <= 1e-3
    assert rel_err(g2[5:8].T, ref.d_rgb) <= 1e-3
    assert rel_err(g2[8], ref.d_A) <= 1e-3
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars"):
        assert rel_err(getattr(grads, name).cpu().numpy(), getattr(ref, name)) <= 1e-3, name


# ----------------------------------------------------------------------------- backward

def _grads_case(w, d, ci=0, ti=0):
    V, R = hip()
    g = to_dev(w.gaussians)
    cam = w.cameras[ci]
    st = R.render(g, [cam], luts_to_dev([w.tfs[ti]]), OPTS)
    res, *_ = oracle.render_image(w.gaussians, cam, w.tfs[ti], OPTS)
    flag = res.flag | res.flag_grad
    d = d.copy()
    d[flag] = 0.0   # both sides see zero dL/dC on flagged pixels
    H, W = cam.height, cam.width
    d_img = torch.as_tensor(d.T.reshape(1, 3, H, W).copy(), dtype=torch.float32).cuda()
    grads = R.Grads.zeros(g)
    g2d = R.render_backward(g, st, d_img, grads)
    torch.cuda.synchronize()
    ref = oracle.gradients(w.gaussians, cam, w.tfs[ti], OPTS, d)
    return st, grads, g2d, ref


def test_backward_c0_matches_oracle_adjoint():
    w = synth.workload(0)
    d = np.random.default_rng(21).standard_normal((64 * 64, 3))
    st, grads, g2d, ref = _grads_case(w, d)
    n = w.gaussians.n
    g2 = g2d.cpu().numpy().reshape(-1, 9)[:n].T
    assert rel_err(g2[0:2].T, ref.d_mean2d) <= 1e-3
    assert rel_err(g2[2:5].T, ref.d_conic) <= 1e-3
    assert rel_err(g2[5:8].T, ref.d_rgb) <= 1e-3
    assert rel_err(g2[8], ref.d_A) <= 1e-3
    assert rel_err(grads.d_means.cpu().numpy(), ref.d_means) <= 1e-3
    assert rel_err(grads.d_log_scales.cpu().numpy(), ref.d_log_scales) <= 1e-3
    assert rel_err(grads.d_quats.cpu().numpy(), ref.d_quats) <= 1e-3
    assert rel_err(grads.d_scalars.cpu().numpy(), ref.d_scalars) <= 1e-3


def test_backward_skipping_unblended_entries_changes_nothing():
    """The forward pass's per-entry hit bits only let the backward pass skip entries that
    blend into no pixel of their tile: gradients with and without them agree (up to the
    order of float atomics across tiles), and entries are in fact skipped."""
    V, R = hip()
    w = synth.workload(1, n_override=60000, res_override=256)
    g = to_dev(w.gaussians)
    cams = [w.cameras[c] for c, _ in w.frames[:3]]
    luts = luts_to_dev(w.tfs)
    tfs = [luts[t] for _, t in w.frames[:3]]
    d_img = torch.randn((3, 3, 256, 256), generator=torch.Generator().manual_seed(5)).cuda()
    out = []
    for hits in (True, False):
        st = R.render(g, cams, tfs, OPTS, hits=hits)
        grads = R.Grads.zeros(g)
        g2d = R.render_backward(g, st, d_img, grads)
        torch.cuda.synchronize()
        out.append((st, grads, g2d))
    (sa, ga, g2a), (sb, gb, g2b) = out
    assert torch.equal(sa.image, sb.image) and torch.equal(sa.n_last, sb.n_last)
    assert rel_err(g2a.cpu().numpy(), g2b.cpu().numpy()) <= 1e-5
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars"):
        assert rel_err(getattr(ga, name).cpu().numpy(), getattr(gb, name).cpu().numpy()) <= 1e-5, name
    # bits of the entries up to each tile's last blended one (the batches the forward pass
    # processed): some set, some clear
    rg = sa.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    words = sa.bins.hits.cpu().numpy().view(np.uint64)
    jm = sa.n_last.cpu().numpy().reshape(3, 16, 16, 16, 16).max(axis=(2, 4)).reshape(-1).astype(np.int64)
    n_set = n_all = 0
    for t in np.nonzero((rg[:, 1] > rg[:, 0]) & (jm >= rg[:, 0]))[0].tolist():
        s0 = int(rg[t, 0])
        for j in range(s0, min(int(jm[t]), int(rg[t, 1]) - 1) + 1):
            n_all += 1
            n_set += (int(words[(s0 >> 6) + t + (j - s0) // 64]) >> ((j - s0) % 64)) & 1
    assert 0 < n_set < n_all


def test_backward_with_weights_dense_scene():
    w = synth.workload(0, n_override=3000)
    w.gaussians.weights = synth.rng_for(0, 4).uniform(0.3, 1.0, w.gaussians.n).astype(np.float32)
    lut = w.tfs[0].copy()
    lut[:, 3] = np.maximum(lut[:, 3], 0.5)
    w.tfs = [lut]
    d = np.random.default_rng(22).standard_normal((64 * 64, 3))
    st, grads, g2d, ref = _grads_case(w, d)
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars", "d_weights"):
        assert rel_err(getattr(grads, name).cpu().numpy(), getattr(ref, name)) <= 1e-3, name


def test_backward_matches_finite_differences_tiny():
    """Tiny scene: the GPU gradient against float64 central differences of the oracle."""
    rng = np.random.default_rng(23)
    n = 10
    g = synth.uniform_gaussians(rng, n, 0.08, 0.25, box=0.5)
    cam = synth.look_at_camera(synth.random_direction(rng), 3.0, 32, 32)
    lut = synth.random_tf(rng)
    lut[:, 3] = np.clip(lut[:, 3] + 0.3, 0, 0.8)
    d = rng.standard_normal((32 * 32, 3))
    V, R = hip()
    gd = to_dev(g)
    st = R.render(gd, [cam], luts_to_dev([lut]), OPTS)
    grads = R.Grads.zeros(gd)
    d_img = torch.as_tensor(d.T.reshape(1, 3, 32, 32).copy(), dtype=torch.float32).cuda()
    R.render_backward(gd, st, d_img, grads)
    gm = grads.d_means.cpu().numpy()

    def loss(means):
        gg = synth.Gaussians(means, g.log_scales.astype(np.float64), g.quats.astype(np.float64),
                             g.scalars.astype(np.float64))
        fp = oracle.footprint_f32(g, cam, lut, OPTS)
        proj = oracle.project_f64(gg.means, gg.log_scales, gg.quats, gg.scalars, None, cam, lut, OPTS)
        order = oracle.depth_order(fp, proj.kept)
        r = oracle.render_pixels(proj, order, all_pixels(32, 32), OPTS)
        return float((r.color.detach().numpy() * d).sum())
    fd = np.zeros_like(gm, dtype=np.float64)
    for i in range(n):
        for k in range(3):
            m = g.means.astype(np.float64)
            h = 1e-6
            m[i, k] += h
            lp = loss(m)
            m[i, k] -= 2 * h
            lm = loss(m)
            fd[i, k] = (lp - lm) / (2 * h)
    assert rel_err(gm, fd) <= 1e-3


# ----------------------------------------------------------------------------- loss

@pytest.mark.parametrize("n,offset", [(100003, 0), (100004, 0), (100004, 1)])
def test_l1_loss_kernel(n, offset):
    """Sizes and alignments that take the scalar path (odd size; views one element past an
    aligned start) and the 16-byte path (size a multiple of 4, aligned)."""
    V, R = hip()
    rng = np.random.default_rng(24)
    a = rng.uniform(0, 1, n).astype(np.float32)
    b = a.copy()
    b[::3] += rng.uniform(-0.5, 0.5, b[::3].shape).astype(np.float32)
    b[5::7] = a[5::7]   # some exact zeros of the difference
    loss = torch.zeros(1, dtype=torch.float64).cuda()
    da = torch.zeros(n + offset, dtype=torch.float32).cuda()
    db = torch.zeros(n + offset, dtype=torch.float32).cuda()
    dd = torch.zeros(n + offset, dtype=torch.float32).cuda()
    da[offset:] = torch.as_tensor(a).cuda()
    db[offset:] = torch.as_tensor(b).cuda()
    d = dd[offset:]
    V.veg_l1_loss(da[offset:], db[offset:], 1.0 / a.size, loss, d)
    ref, gref = oracle.l1_loss(a, b, scale=float(np.float32(1.0 / a.size)))
    assert abs(loss.item() - ref) <= 1e-6 * ref
    assert np.array_equal(d.cpu().numpy(), gref.astype(np.float32))


def test_needles_at_45_degrees_image_and_gradients():
    """Strongly elongated Gaussians turned 45 degrees in the image plane (long axis 10-30 px,
    short axis at the low-pass width; (S00 S11) / det from about 100 to 900): the forward pass
    skips quadrants by the ellipse's box, whose rounding allowance must grow with the
    elongation, and the backward pass must recover the same blended sets.  Image and
    gradients against the oracle.  (Along a needle's long axis the float32 quadratic form
    loses about log2((S00 S11) / det) bits to cancellation, so much longer needles leave
    the 1e-4 / 1e-3 bars.)"""
    rng = np.random.default_rng(45)
    n = 24
    W = H = 128
    f = (0.5 * H) / np.tan(np.radians(25.0))
    cam = synth.Camera(view=np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 2.0], np.float32), fx=float(np.float32(f)),
                       fy=float(np.float32(f)), cx=0.5 * W, cy=0.5 * H, width=W, height=H)
    means = np.zeros((n, 3), np.float32)
    means[:, :2] = rng.uniform(-0.5, 0.5, (n, 2))
    means[:, 2] = rng.uniform(-0.3, 0.3, n)
    long = np.exp(rng.uniform(np.log(0.15), np.log(0.45), n))
    scales = np.stack([long, np.full(n, 1e-3), np.full(n, 1e-3)], 1)
    ang = np.where(rng.uniform(size=n) < 0.5, np.pi / 4, -np.pi / 4) + rng.uniform(-0.05, 0.05, n)
    quats = np.stack([np.cos(ang / 2), np.zeros(n), np.zeros(n), np.sin(ang / 2)], 1).astype(np.float32)
    g = synth.Gaussians(means, np.log(scales).astype(np.float32), quats, rng.uniform(0.2, 0.9, n).astype(np.float32))
    lut = synth.random_tf(rng)
    lut[:, 3] = np.clip(lut[:, 3] + 0.4, 0.0, 1.0)
    w = synth.Workload("needles-45deg", g, [cam], [lut], [(0, 0)])
    V, R = hip()
    gd = to_dev(g)
    st = R.render(gd, [cam], luts_to_dev([lut]), OPTS)
    torch.cuda.synchronize()
    res, *_ = oracle.render_image(g, cam, lut, OPTS)
    compare_image(image_pixels(st.image[0]), res)
    d = rng.standard_normal((W * H, 3))
    st2, grads, g2d, ref = _grads_case(w, d)
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars"):
        assert rel_err(getattr(grads, name).cpu().numpy(), getattr(ref, name)) <= 1e-3, name


@pytest.mark.parametrize("shared", [False, True])
def test_forward_with_fused_l1_equals_forward_then_l1(shared):
    """veg_render_fwd_l1 writes exactly what veg_render_fwd followed by veg_l1_loss gives:
    the image gradient bit for bit (sign times scale of the same float32 colour), the same
    transmittance, last indices and hit bits, and the loss up to summation order (both
    calls on one projection and key list; hit words cleared before each)."""
    V, R = hip()
    w = synth.workload(1, n_override=6000, views_override=2, tfs_override=2, res_override=96)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    cams = w.cameras if shared else [w.cameras[c] for c, _ in w.frames]
    tfs = [luts[t] for _, t in w.frames]
    F = len(w.frames)
    st = R.render(g, cams, tfs, OPTS, shared=shared)
    o = V.make_opts(OPTS)
    rng = np.random.default_rng(61)
    tgt = torch.as_tensor(rng.uniform(0, 1, (F, 3, 96, 96)).astype(np.float32)).cuda()
    scale = 1.0 / tgt.numel()
    img = torch.empty_like(st.image)
    t1, n1 = torch.empty_like(st.t_final), torch.empty_like(st.n_last)
    st.bins.hits.zero_()
    V.veg_render_fwd(st.proj, st.bins, o, img, t1, n1)
    h1 = st.bins.hits.clone()
    tgt[:, :, 40:56, 40:56] = img[:, :, 40:56, 40:56]   # colour == target there: sign 0
    loss_ref = torch.zeros(1, dtype=torch.float64).cuda()
    d_ref = torch.empty_like(img)
    V.veg_l1_loss(img, tgt, scale, loss_ref, d_ref)
    slots = torch.zeros(64, dtype=torch.float64).cuda()
    d_img = torch.empty_like(img)
    t2, n2 = torch.empty_like(t1), torch.empty_like(n1)
    st.bins.hits.zero_()
    V.veg_render_fwd_l1(st.proj, st.bins, o, tgt, scale, slots, d_img, t2, n2)
    torch.cuda.synchronize()
    assert torch.equal(d_img, d_ref)
    assert torch.equal(t2, t1) and torch.equal(n2, n1)
    assert torch.equal(st.bins.hits, h1)
    assert (d_ref == 0).any() and (d_ref > 0).any() and (d_ref < 0).any()
    assert abs(slots.sum().item() - loss_ref.item()) <= 1e-12 * loss_ref.item()
    l_or, _ = oracle.l1_loss(img.cpu().numpy(), tgt.cpu().numpy(), scale=scale)
    assert abs(slots.sum().item() - l_or) <= 1e-6 * l_or
