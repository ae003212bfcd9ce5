"""The multi-view x multi-TF training step (grouped forward recomputation) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import image_pixels, luts_to_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _small():
    w = synth.workload(1, n_override=4000, views_override=3, tfs_override=2, res_override=80)
    return w


def _targets(w):
    """Targets = oracle images offset by +-0.05 (random sign per pixel-channel), so the L1
    sign is far from ambiguous on both sides."""
    rng = synth.rng_for(1, 60)
    H = W = w.width
    out, refs = [], []
    for ci, ti in w.frames:
        res, *_ = oracle.render_image(w.gaussians, w.cameras[ci], w.tfs[ti], w.opts)
        c = res.color.detach().numpy()
        t = c + 0.05 * np.sign(rng.standard_normal(c.shape))
        refs.append((c, res))
        out.append(t.T.reshape(3, H, W))
    return np.stack(out).astype(np.float32), refs


def test_train_step_matches_oracle_and_grouping_does_not_matter():
    from paper_2504_13339_amd import render as R
    w = _small()
    tgt_np, refs = _targets(w)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    tgt = torch.as_tensor(tgt_np).cuda()
    F = len(w.frames)
    H = W = w.width
    M = F * 3 * H * W
    results = {}
    for group in (1, 4, F):
        grads = R.Grads.zeros(g)
        res = R.train_step_l1(g, w.cameras, luts, w.frames, tgt, grads, group, w.opts)
        torch.cuda.synchronize()
        results[group] = (res.loss, {k: getattr(grads, k).cpu().numpy() for k in
                                     ("d_means", "d_log_scales", "d_quats", "d_scalars")})
    # grouping changes nothing but float-atomic summation order
    for group in (4, F):
        assert abs(results[group][0] - results[1][0]) <= 1e-9
        for k, v in results[group][1].items():
            assert rel_err(v, results[1][1][k]) <= 1e-5, (group, k)
    # oracle: L1 mean and its gradient, frame by frame
    loss_ref = 0.0
    acc = None
    for f, (ci, ti) in enumerate(w.frames):
        c, res = refs[f]
        t = tgt_np[f].reshape(3, -1).T.astype(np.float64)
        lf, d = oracle.l1_loss(c, t, scale=1.0 / M)
        loss_ref += lf
        gr = oracle.gradients(w.gaussians, w.cameras[ci], w.tfs[ti], w.opts, d)
        cur = {"d_means": gr.d_means, "d_log_scales": gr.d_log_scales, "d_quats": gr.d_quats,
               "d_scalars": gr.d_scalars}
        acc = cur if acc is None else {k: acc[k] + cur[k] for k in acc}
    assert abs(results[1][0] - loss_ref) <= 1e-6 * loss_ref
    for k in acc:
        assert rel_err(results[1][1][k], acc[k]) <= 1e-3, k


def test_autograd_function_matches_render_backward():
    from paper_2504_13339_amd import render as R
    w = synth.workload(0, n_override=1500)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    params = [t.clone().requires_grad_(True) for t in (g.means, g.log_scales, g.quats, g.scalars)]
    img = R.render_autograd(*params, None, w.cameras, luts, w.opts)
    d = torch.randn_like(img)
    (img * d).sum().backward()
    st = R.render(g, w.cameras, luts, w.opts)
    grads = R.Grads.zeros(g)
    R.render_backward(g, st, d, grads)
    torch.cuda.synchronize()
    assert torch.equal(img.detach(), st.image)
    for p, ref in zip(params, (grads.d_means, grads.d_log_scales, grads.d_quats, grads.d_scalars)):
        assert rel_err(p.grad.cpu().numpy(), ref.cpu().numpy()) <= 1e-5
