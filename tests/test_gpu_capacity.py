"""A training step with the key lists sized ahead (no host synchronisation until the loss is
read) against the same step with exactly sized lists: same loss, gradients, visibility
counts and entry counts, with and without shared views, in one group and in several.  A
capacity that is too small is reported (KeyListOverflow) instead of giving a silent wrong
step, and the device status read later says the same."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import hip, luts_to_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu
NAMES = ("d_means", "d_log_scales", "d_quats", "d_scalars")


def _setup():
    V, R = hip()
    w = synth.workload(1, n_override=6000, views_override=3, tfs_override=2, res_override=96)
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    F = len(w.frames)
    tgt = torch.rand((F, 3, w.width, w.width), generator=torch.Generator().manual_seed(7)).cuda()
    return R, w, g, luts, tgt


def _step(R, w, g, luts, tgt, group, shared, capacity, read_loss=True):
    grads = R.Grads.zeros(g)
    dens = R.DensifyStats.zeros(w.gaussians.n)
    res = R.train_step(g, w.cameras, luts, w.frames, tgt, grads, group, w.opts, ssim_lambda=0.2, densify=dens,
                       shared=shared, capacity=capacity, read_loss=read_loss)
    torch.cuda.synchronize()
    return res, {k: getattr(grads, k).cpu().numpy() for k in NAMES}, dens.vis_count.cpu().numpy()


@pytest.mark.parametrize("group,shared", [(6, False), (2, False), (6, True), (4, True)])
def test_sized_ahead_step_matches_exact_step(group, shared):
    R, w, g, luts, tgt = _setup()
    ra, ga, va = _step(R, w, g, luts, tgt, group, shared, None)
    cap = max(ra.n_entries) + 100
    rb, gb, vb = _step(R, w, g, luts, tgt, group, shared, cap)
    assert rb.n_entries == ra.n_entries
    assert abs(rb.loss - ra.loss) <= 1e-9 * max(1.0, abs(ra.loss))
    assert np.array_equal(va, vb)
    for k in NAMES:
        assert rel_err(gb[k], ga[k]) <= 1e-5, k
    # the same flags read later from the device status
    rc, _, _ = _step(R, w, g, luts, tgt, group, shared, cap, read_loss=False)
    assert R.check_status(rc.status, cap) == ra.n_entries


def test_too_small_capacity_is_reported():
    R, w, g, luts, tgt = _setup()
    ra, _, _ = _step(R, w, g, luts, tgt, 6, True, None)
    cap = max(ra.n_entries) // 2
    with pytest.raises(R.KeyListOverflow):
        _step(R, w, g, luts, tgt, 6, True, cap)
    rc, _, _ = _step(R, w, g, luts, tgt, 6, True, cap, read_loss=False)
    st = rc.status.cpu().numpy()
    assert st[0, 0] == max(ra.n_entries) and st[0, 1] == 1
    with pytest.raises(R.KeyListOverflow):
        R.check_status(rc.status, cap)
