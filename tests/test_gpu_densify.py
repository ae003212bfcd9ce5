"""Adaptive density control against the oracle: the clone / split / prune decisions bit
for bit, and the new model (survivors, clone copies, split children) with copies bit-exact
and the children's centres and scales to float32 rounding."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import hip

pytestmark = pytest.mark.gpu

TH = dict(grad_thresh=0.02, log_scale_thresh=-4.0, prune_weight=0.005)


def _case(n, seed):
    rng = np.random.default_rng(seed)
    g = synth.workload(1, n_override=n).gaussians
    vis = rng.integers(0, 6, n).astype(np.int32)
    acc = (rng.exponential(0.02, n) * vis).astype(np.float32)
    w = rng.uniform(0, 0.05, n).astype(np.float32)
    w[::97] = np.nan
    z = rng.standard_normal((n, 2, 3)).astype(np.float32)
    return g, acc, vis, w, z


@pytest.mark.parametrize("n", [1, 300, 100003])
def test_plan_matches_oracle_bit_for_bit(n):
    V, R = hip()
    g, acc, vis, w, z = _case(n, n)
    act, counts, ws = V.veg_densify_plan(torch.as_tensor(acc).cuda(), torch.as_tensor(vis).cuda(),
                                         torch.as_tensor(g.log_scales).cuda(), torch.as_tensor(w).cuda(), **TH)
    torch.cuda.synchronize()
    ref, rc = oracle.densify_plan(acc, vis, g.log_scales, w, **TH)
    assert np.array_equal(act.cpu().numpy()[:n], ref)
    assert counts == list(rc)
    if n > 1000:
        assert (rc > 100).all()   # every branch is exercised


def test_apply_matches_oracle():
    V, R = hip()
    n = 20011
    g, acc, vis, w, z = _case(n, 5)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda()
    act, counts, ws = V.veg_densify_plan(dev(acc), torch.as_tensor(vis).cuda(), dev(g.log_scales), dev(w), **TH)
    n_new = n + counts[1] + counts[2] - counts[3]
    mom = np.random.default_rng(6).standard_normal((n, 4)).astype(np.float32)
    srcs = [(g.means, 1), (g.log_scales, 2), (g.quats, 0), (g.scalars, 0), (w, 0), (mom, 3)]
    fields, outs = [], []
    for a, role in srcs:
        d = torch.empty((n_new,) + a.shape[1:], dtype=torch.float32, device="cuda")
        fields.append((dev(a), d, role))
        outs.append(d)
    V.veg_densify_apply(act, dev(g.quats), dev(g.log_scales), dev(z), fields, ws)
    torch.cuda.synchronize()
    ref_act, _ = oracle.densify_plan(acc, vis, g.log_scales, w, **TH)
    ref = oracle.densify_apply(ref_act, g.means, g.log_scales, g.quats, z, srcs)
    n_copy = n + counts[1] - counts[2] - counts[3]          # survivors and clone copies
    for (a, role), got, r in zip(srcs, outs, ref):
        got = got.cpu().numpy()
        assert got.shape == r.shape
        # survivors and clone copies are copies (or zeros) bit for bit
        assert np.array_equal(got[:n_copy], r[:n_copy].astype(np.float32), equal_nan=True), role
        if role == 1:
            assert np.abs(got[n_copy:] - r[n_copy:]).max() <= 1e-5 * (1 + np.abs(r[n_copy:]).max())
        elif role == 2:
            assert np.abs(got[n_copy:] - r[n_copy:]).max() <= 1e-6 * (1 + np.abs(r[n_copy:]).max())
        else:
            assert np.array_equal(got[n_copy:], r[n_copy:].astype(np.float32), equal_nan=True), role


def test_densify_model_rebinds_adam_and_renders():
    V, R = hip()
    w0 = synth.workload(1, n_override=5000, views_override=1, tfs_override=1, res_override=64)
    g = V.Gaussians.from_numpy(w0.gaussians)
    g.weights = torch.full((g.n,), 0.5, device="cuda")
    g.weights[::10] = 0.001
    stats = R.DensifyStats.zeros(g.n)
    rng = np.random.default_rng(7)
    stats.grad_accum.copy_(torch.as_tensor(rng.exponential(0.05, g.n).astype(np.float32)))
    stats.vis_count.fill_(1)
    adam = R.Adam([(g.means, 1e-3), (g.weights, 1e-2)])
    adam.m[0].fill_(1.0)
    z = torch.as_tensor(rng.standard_normal((g.n, 2, 3)).astype(np.float32)).cuda()
    g2, counts = R.densify_model(g, stats, 0.05, -4.0, 0.005, z, adam=adam)
    torch.cuda.synchronize()
    assert counts[3] == 500 and g2.n == g.n + counts[1] + counts[2] - counts[3]
    assert adam.params[0][0] is g2.means and adam.params[1][0] is g2.weights
    n_copy = g.n + counts[1] - counts[2] - counts[3]
    m0 = adam.m[0].cpu().numpy()
    assert np.all(m0[:g.n - counts[2] - counts[3]] == 1.0) and np.all(m0[g.n - counts[2] - counts[3]:] == 0.0)
    assert bool((g2.weights >= 0.005).all())
    st = R.render(g2, [w0.cameras[0]], [torch.as_tensor(w0.tfs[0]).cuda()], w0.opts)
    torch.cuda.synchronize()
    assert torch.isfinite(st.image).all() and n_copy > 0
