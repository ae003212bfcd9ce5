"""The blend kernels dispatch their (frame, tile) blocks longest list first when the
sort's spare buffer can hold the order, and in natural order otherwise.  The schedule must
not change any result: images, final transmittance, last-entry indices and hit bits are
bit-identical, gradients agree up to the order of float atomics across tiles."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import hip, luts_to_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu
OPTS = dict(synth.DEFAULT_OPTS)
ORDER_HEADER = 128   # scratch words ahead of the order


def _case(n, res, frames, seed):
    V, R = hip()
    w = synth.workload(1, n_override=n, res_override=res)
    g = to_dev(w.gaussians)
    cams = [w.cameras[c] for c, _ in w.frames[:frames]]
    luts = luts_to_dev(w.tfs)
    tfs = [luts[t] for _, t in w.frames[:frames]]
    d_img = torch.randn((frames, 3, res, res), generator=torch.Generator().manual_seed(seed)).cuda()
    tiles = frames * ((res + 15) // 16) ** 2
    return R, g, cams, tfs, d_img, tiles


def _run(R, g, cams, tfs, d_img, capacity):
    st = R.render(g, cams, tfs, OPTS, capacity=capacity)
    grads = R.Grads.zeros(g)
    g2d = R.render_backward(g, st, d_img, grads)
    torch.cuda.synchronize()
    return st, grads, g2d


@pytest.mark.parametrize("n,res,frames", [(120, 512, 6), (60, 500, 4)])
def test_dispatch_order_changes_no_result(n, res, frames):
    R, g, cams, tfs, d_img, tiles = _case(n, res, frames, seed=11)
    sa, ga, g2a = _run(R, g, cams, tfs, d_img, None)   # capacity = entries
    E = int(sa.bins.struct.capacity)
    # sized so that the first run's spare buffer is too small for the order (natural order)
    assert 0 < E < tiles + ORDER_HEADER
    sb, gb, g2b = _run(R, g, cams, tfs, d_img, E + tiles + ORDER_HEADER)   # ordered
    assert torch.equal(sa.image, sb.image)
    assert torch.equal(sa.t_final, sb.t_final) and torch.equal(sa.n_last, sb.n_last)
    # hit bits of the batches up to each tile's last blended entry (batches after it may
    # not be visited): the word layout depends only on the ranges
    ra = sa.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    rb = sb.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    assert np.array_equal(ra, rb)
    wa = sa.bins.hits.cpu().numpy().view(np.uint64)
    wb = sb.bins.hits.cpu().numpy().view(np.uint64)
    tx = (res + 15) // 16
    nl = np.full((frames, tx * 16, tx * 16), -1, dtype=np.int64)
    nl[:, :res, :res] = sa.n_last.cpu().numpy()
    jm = nl.reshape(frames, tx, 16, tx, 16).max(axis=(2, 4)).reshape(-1)
    n_cmp = 0
    for t in np.nonzero((ra[:, 1] > ra[:, 0]) & (jm >= ra[:, 0]))[0].tolist():
        s0, e0 = int(ra[t, 0]), int(ra[t, 1])
        for b in range((int(jm[t]) - s0) // 64 + 1):
            k = (s0 >> 6) + t + b
            m = (1 << min(64, e0 - s0 - 64 * b)) - 1
            assert (int(wa[k]) & m) == (int(wb[k]) & m), (t, b)
            n_cmp += 1
    assert n_cmp > 0
    assert rel_err(g2a.cpu().numpy(), g2b.cpu().numpy()) <= 1e-5
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars"):
        assert rel_err(getattr(ga, name).cpu().numpy(), getattr(gb, name).cpu().numpy()) <= 1e-5, name


@pytest.mark.parametrize("n,res", [(100, 512), (60, 400)])
def test_dispatch_order_changes_no_result_on_shared_lists(n, res):
    """Three tables per view on one key list: every frame's image, transmittance and last
    indices, and each table slot's hit bits, are the same in natural and sorted order."""
    V, R = hip()
    K, views = 3, 2
    w = synth.workload(1, n_override=n, res_override=res, views_override=views, tfs_override=K)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    cams = [w.cameras[c] for c, _ in w.frames[::K]]
    tfs = [luts[t] for _, t in w.frames]
    F = len(w.frames)
    d_img = torch.randn((F, 3, res, res), generator=torch.Generator().manual_seed(13)).cuda()
    tpv = ((res + 15) // 16) ** 2

    def run(capacity):
        st = R.render(g, cams, tfs, OPTS, capacity=capacity, shared=True)
        grads = R.Grads.zeros(g)
        g2d = R.render_backward(g, st, d_img, grads)
        torch.cuda.synchronize()
        return st, grads, g2d

    sa, ga, g2a = run(None)
    E = int(sa.bins.struct.capacity)
    assert 0 < E < F * tpv + ORDER_HEADER   # natural order in the first run
    sb, gb, g2b = run(E + F * tpv + ORDER_HEADER)
    assert torch.equal(sa.image, sb.image)
    assert torch.equal(sa.t_final, sb.t_final) and torch.equal(sa.n_last, sb.n_last)
    ra = sa.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    assert np.array_equal(ra, sb.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64))
    wa = sa.bins.hits.cpu().numpy().view(np.uint64)
    wb = sb.bins.hits.cpu().numpy().view(np.uint64)
    stride_a = V.veg_bin_hit_words(E, views * tpv)
    stride_b = V.veg_bin_hit_words(E + F * tpv + ORDER_HEADER, views * tpv)
    tx = (res + 15) // 16
    nl = np.full((F, tx * 16, tx * 16), -1, dtype=np.int64)
    nl[:, :res, :res] = sa.n_last.cpu().numpy()
    jm = nl.reshape(F, tx, 16, tx, 16).max(axis=(2, 4)).reshape(F, -1)
    n_cmp = 0
    for f in range(F):
        v, k = divmod(f, K)
        for lt in range(tpv):
            t = v * tpv + lt
            s0, e0 = int(ra[t, 0]), int(ra[t, 1])
            if e0 <= s0 or jm[f, lt] < s0:
                continue
            for b in range((int(jm[f, lt]) - s0) // 64 + 1):
                idx = (s0 >> 6) + t + b
                m = (1 << min(64, e0 - s0 - 64 * b)) - 1
                assert (int(wa[k * stride_a + idx]) & m) == (int(wb[k * stride_b + idx]) & m), (f, lt, b)
                n_cmp += 1
    assert n_cmp > 0
    assert rel_err(g2a.cpu().numpy(), g2b.cpu().numpy()) <= 1e-5
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars"):
        assert rel_err(getattr(ga, name).cpu().numpy(), getattr(gb, name).cpu().numpy()) <= 1e-5, name
