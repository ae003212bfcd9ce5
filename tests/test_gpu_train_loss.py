"""Training-loop neighbours of the renderer against the oracle: the SSIM loss term and its
image gradient, the Adam update, the densification statistics, and the training step with
the mixed loss (1 - lambda) L1 + lambda (1 - SSIM), lambda = 0.2."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import hip, luts_to_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _ssim_case(seed, planes, H, W, near):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (planes, H, W)).astype(np.float32)
    if near:   # a target close to the image, as late in training
        y = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1).astype(np.float32)
    else:
        y = rng.uniform(0, 1, x.shape).astype(np.float32)
    return x, y


def _gpu_ssim(x, y, weight, d_init=None):
    V, R = hip()
    loss = torch.zeros(1, dtype=torch.float64).cuda()
    d = torch.zeros(x.shape, dtype=torch.float32).cuda() if d_init is None else torch.as_tensor(d_init).cuda()
    V.veg_ssim_loss(torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda(), weight, loss, d)
    torch.cuda.synchronize()
    return loss.item(), d.cpu().numpy()


@pytest.mark.parametrize("planes,H,W,near", [(6, 37, 75, False), (3, 64, 64, True), (2, 16, 32, False),
                                             (1, 5, 3, False), (1, 1, 1, True), (9, 100, 33, True)])
def test_ssim_loss_and_gradient_match_oracle(planes, H, W, near):
    """Shapes span several 32x16 output tiles with ragged right and bottom tails, images
    smaller than the 11-tap window, and a single pixel."""
    x, y = _ssim_case(planes * 1000 + H * 7 + W, planes, H, W, near)
    weight = 0.2 / x.size
    got_l, got_d = _gpu_ssim(x, y, weight)
    ref_l, ref_d = oracle.ssim_loss(x, y, weight)
    assert abs(got_l - ref_l) <= 1e-4 * abs(ref_l) + 1e-12
    assert rel_err(got_d, ref_d) <= 1e-3


def test_ssim_gradient_is_added_to_d_image_and_loss_accumulates():
    V, R = hip()
    x, y = _ssim_case(5, 4, 48, 40, True)
    base = np.random.default_rng(6).standard_normal(x.shape).astype(np.float32)
    weight = 1.0 / x.size
    loss = torch.full((1,), 0.5, dtype=torch.float64).cuda()
    d = torch.as_tensor(base).cuda()
    V.veg_ssim_loss(torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda(), weight, loss, d)
    torch.cuda.synchronize()
    ref_l, ref_d = oracle.ssim_loss(x, y, weight)
    assert abs(loss.item() - (0.5 + ref_l)) <= 1e-4 * (0.5 + ref_l)
    assert rel_err(d.cpu().numpy() - base, ref_d) <= 1e-3


@pytest.mark.parametrize("planes,H,W,lam", [(6, 37, 75, 0.2), (3, 64, 64, 0.2), (1, 5, 3, 0.5), (2, 40, 48, 1.0)])
def test_image_loss_equals_l1_then_ssim(planes, H, W, lam):
    """The fused loss writes d_image bit for bit as veg_l1_loss followed by veg_ssim_loss,
    the loss within summation-order rounding; both against the oracle's two terms."""
    V, R = hip()
    x, y = _ssim_case(planes * 31 + H + W, planes, H, W, True)
    x[0, 0, :2] = y[0, 0, :2]   # zero differences: sign(0) = 0 on both paths
    M = x.size
    xd, yd = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    loss_a = torch.zeros(1, dtype=torch.float64).cuda()
    d_a = torch.full(x.shape, float("nan")).cuda()   # overwritten, never read
    V.veg_image_loss(xd, yd, (1 - lam) / M, lam / M, loss_a, d_a)
    loss_b = torch.zeros(1, dtype=torch.float64).cuda()
    d_b = torch.empty(x.shape).cuda()
    V.veg_l1_loss(xd, yd, (1 - lam) / M, loss_b, d_b)
    V.veg_ssim_loss(xd, yd, lam / M, loss_b, d_b)
    torch.cuda.synchronize()
    assert torch.equal(d_a, d_b)
    assert abs(loss_a.item() - loss_b.item()) <= 1e-12 * abs(loss_b.item())
    ref_l1 = oracle.l1_loss(x, y, (1 - lam) / M)
    ref_s, ref_d = oracle.ssim_loss(x, y, lam / M)
    assert abs(loss_a.item() - (ref_l1[0] + ref_s)) <= 1e-4 * (ref_l1[0] + ref_s)
    assert rel_err(d_a.cpu().numpy(), ref_l1[1] + ref_d) <= 1e-3


def test_ssim_of_identical_images_is_zero_loss_and_zero_gradient():
    x, _ = _ssim_case(7, 2, 40, 50, False)
    got_l, got_d = _gpu_ssim(x, x.copy(), 1.0)
    assert abs(got_l) <= 1e-6
    assert np.abs(got_d).max() <= 1e-6


def test_ssim_rejects_bad_arguments():
    import ctypes
    from paper_2504_13339_amd import _lib
    V, R = hip()
    lib = _lib.load()
    x = torch.zeros((2, 8, 8), device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert lib.veg_ssim_workspace_bytes(2, 8, 8) == 3 * 4 * 2 * 64
    rc = lib.veg_ssim_loss(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 2, 8, 8,
                           ctypes.c_float(1.0), ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                           ctypes.c_void_p(small.data_ptr()), 16, None)
    assert rc == 1 and b"workspace" in lib.veg_last_error()
    rc = lib.veg_ssim_loss(None, None, 70000, 8, 8, ctypes.c_float(1.0), None, None, None, 0, None)
    assert rc == 1


def f32(x):
    return float(np.float32(x))


@pytest.mark.parametrize("n", [1, 1000, 1_000_003])
def test_adam_steps_match_oracle(n):
    """Three consecutive steps (bias correction changes with the step), with some zero
    gradients; parameters of mixed scale."""
    V, R = hip()
    rng = np.random.default_rng(n)
    p = (rng.standard_normal(n) * rng.choice([1e-3, 1.0, 10.0], n)).astype(np.float32)
    lr = 2.5e-2
    pd, md, vd = torch.as_tensor(p).cuda(), torch.zeros(n).cuda(), torch.zeros(n).cuda()
    pr, mr, vr = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        g = (rng.standard_normal(n) * 1e-3).astype(np.float32)
        g[::7] = 0.0
        before = pd.cpu().numpy().astype(np.float64)
        V.veg_adam_step(pd, torch.as_tensor(g).cuda(), md, vd, lr, step)
        torch.cuda.synchronize()
        # the ABI takes the hyperparameters as float32: the oracle gets the same rounded values
        # (1 - float32(0.999) differs from 1 - 0.999 by 1.3e-5 relative)
        pr, mr, vr = oracle.adam_step(before, g, mr, vr, step, f32(lr), f32(0.9), f32(0.999), f32(1e-15))
        got = pd.cpu().numpy().astype(np.float64)
        # the kernel rounds the new value once to float32: within one ulp of the float64 result
        ulp = np.spacing(np.abs(pr).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got - pr) <= ulp + 1e-5 * lr)
        assert rel_err(md.cpu().numpy(), mr) <= 1e-6 and rel_err(vd.cpu().numpy(), vr) <= 1e-6
        if step == 1:    # zero moments and a zero gradient: no update at all
            assert np.array_equal(got[::7], before[::7])


def test_adam_first_step_zero_gradient_leaves_parameters_and_rejects_bad_arguments():
    import ctypes
    from paper_2504_13339_amd import _lib
    V, R = hip()
    p = torch.linspace(-1, 1, 513).cuda()
    p0 = p.clone()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    V.veg_adam_step(p, torch.zeros_like(p), m, v, 0.1, 1)
    torch.cuda.synchronize()
    assert torch.equal(p, p0)
    lib = _lib.load()
    assert lib.veg_adam_step(None, None, None, None, 4, ctypes.c_float(0.1), ctypes.c_float(0.9),
                             ctypes.c_float(0.999), ctypes.c_float(1e-15), 0, None) == 1
    assert lib.veg_adam_step(None, None, None, None, 4, ctypes.c_float(0.1), ctypes.c_float(1.0),
                             ctypes.c_float(0.999), ctypes.c_float(1e-15), 1, None) == 1


def test_densify_stats_match_oracle_on_seeded_screen_gradients():
    """The kept mask comes from the oracle's float32 footprint (bit-exact with the kernel's
    projection, tested elsewhere); the screen-space gradients are seeded random values, so
    no oracle input is taken from the HIP path.  Two calls accumulate."""
    V, R = hip()
    w = synth.workload(1, n_override=3000, views_override=3, tfs_override=2, res_override=64)
    frames = w.frames[:4]
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    proj = V.veg_project(g, [w.cameras[c] for c, _ in frames], [luts[t] for _, t in frames], w.opts)
    n, F = w.gaussians.n, len(frames)
    rng = np.random.default_rng(90)
    g2d = rng.standard_normal((F, n, 9)).astype(np.float32)
    kept = np.stack([oracle.footprint_f32(w.gaussians, w.cameras[c], w.tfs[t], w.opts).count > 0
                     for c, t in frames])
    assert kept.any() and not kept.all()
    acc = torch.zeros(n, dtype=torch.float32).cuda()
    vis = torch.zeros(n, dtype=torch.int32).cuda()
    gd = torch.as_tensor(g2d.reshape(-1)).cuda()
    V.veg_densify_stats(proj, gd, acc, vis)
    V.veg_densify_stats(proj, gd, acc, vis)
    torch.cuda.synchronize()
    ref_a, ref_c = oracle.densify_stats(g2d, kept)
    assert np.array_equal(vis.cpu().numpy(), 2 * ref_c)
    assert rel_err(acc.cpu().numpy(), 2 * ref_a) <= 1e-5


def _small():
    return synth.workload(1, n_override=4000, views_override=3, tfs_override=2, res_override=80)


def test_train_step_with_ssim_matches_oracle_and_grouping_does_not_matter():
    """Loss (1 - 0.2) mean L1 + 0.2 mean(1 - SSIM) over 6 frames; its value and the parameter
    gradients against the oracle (its own images, its own loss gradient per frame)."""
    V, R = hip()
    w = _small()
    lam = 0.2
    rng = synth.rng_for(1, 61)
    H = W = w.width
    refs, tg = [], []
    for ci, ti in w.frames:
        res, *_ = oracle.render_image(w.gaussians, w.cameras[ci], w.tfs[ti], w.opts)
        c = res.color.detach().numpy()                       # [H*W, 3]
        t = c + 0.05 * np.sign(rng.standard_normal(c.shape))
        refs.append(c)
        tg.append(t.T.reshape(3, H, W))
    tgt_np = np.stack(tg).astype(np.float32)
    F = len(w.frames)
    M = F * 3 * H * W
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    tgt = torch.as_tensor(tgt_np).cuda()
    out = {}
    for group in (1, F):
        grads = R.Grads.zeros(g)
        dens = R.DensifyStats.zeros(w.gaussians.n)
        res = R.train_step(g, w.cameras, luts, w.frames, tgt, grads, group, w.opts, ssim_lambda=lam, densify=dens)
        torch.cuda.synchronize()
        out[group] = (res.loss, {k: getattr(grads, k).cpu().numpy() for k in
                                 ("d_means", "d_log_scales", "d_quats", "d_scalars")},
                      dens.vis_count.cpu().numpy())
    assert abs(out[F][0] - out[1][0]) <= 1e-9
    assert np.array_equal(out[F][2], out[1][2])
    for k, v in out[F][1].items():
        assert rel_err(v, out[1][1][k]) <= 1e-5, k
    loss_ref, acc = 0.0, None
    vis_ref = np.zeros(w.gaussians.n, np.int64)
    for f, (ci, ti) in enumerate(w.frames):
        c = refs[f]
        img = c.T.reshape(3, H, W)
        t64 = tgt_np[f].astype(np.float64)
        sl, sd = oracle.ssim_loss(img, t64, lam / M)
        l1, d_l1 = oracle.l1_loss(img, t64, scale=(1 - lam) / M)
        loss_ref += l1 + sl
        d_img = d_l1 + sd      # [3, H, W]
        gr = oracle.gradients(w.gaussians, w.cameras[ci], w.tfs[ti], w.opts, d_img.reshape(3, -1).T)
        cur = {"d_means": gr.d_means, "d_log_scales": gr.d_log_scales, "d_quats": gr.d_quats,
               "d_scalars": gr.d_scalars}
        acc = cur if acc is None else {k: acc[k] + cur[k] for k in acc}
        vis_ref += oracle.footprint_f32(w.gaussians, w.cameras[ci], w.tfs[ti], w.opts).count > 0
    assert abs(out[1][0] - loss_ref) <= 1e-5 * loss_ref
    for k in acc:
        assert rel_err(out[1][1][k], acc[k]) <= 1e-3, k
    assert np.array_equal(out[1][2], vis_ref)
