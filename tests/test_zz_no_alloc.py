"""veg_bin_static, the allocation-free binning call (the library's own scratch array), against
veg_bin_count + veg_bin_sort + veg_bin_status with a caller workspace, through the C ABI:
sorted keys, values, per-tile ranges and the (entries, overflow) status bit for bit, on two
calls in a row on one stream (the second smaller, so it runs on the first one's leftover
scratch), then a call whose list overflows its capacity."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import luts_to_dev, to_dev

pytestmark = pytest.mark.gpu


def _project(w, frames):
    from paper_2504_13339_amd import veg as V
    g = to_dev(w.gaussians)
    luts = luts_to_dev(w.tfs)
    proj = V.veg_project(g, [w.cameras[c] for c, _ in frames], [luts[t] for _, t in frames], w.opts)
    return g, luts, proj


def _poisoned_bins(proj, cap):
    from paper_2504_13339_amd import veg as V
    b = V.alloc_bins(proj, cap, hits=False)
    for t in (b.keys, b.vals, b.keys_alt, b.vals_alt, b.ranges):
        t.fill_(-1)
    return b


def _compare(proj, cap=None):
    from paper_2504_13339_amd import veg as V
    ws = V.alloc_bin_workspace(proj)
    E = V.veg_bin_count(proj, ws, sync=True)
    cap = E + 64 if cap is None else cap
    ref = _poisoned_bins(proj, cap)
    V.veg_bin_sort(proj, ws, ref)
    st_ref = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    V.veg_bin_status(ws, st_ref)
    got = _poisoned_bins(proj, cap)
    st = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    V.veg_bin_static(proj, got, st)
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy(), st_ref.cpu().numpy())
    n = min(E, cap)
    assert np.array_equal(got.keys[:n].cpu().numpy(), ref.keys[:n].cpu().numpy())
    assert np.array_equal(got.vals[:n].cpu().numpy(), ref.vals[:n].cpu().numpy())
    if E <= cap:
        nt = 2 * int(proj.struct.total_tiles)
        assert np.array_equal(got.ranges[:nt].cpu().numpy(), ref.ranges[:nt].cpu().numpy())
    return E, st.cpu().numpy()


def test_bin_static_equals_the_workspace_calls_twice_in_a_row():
    # first call: 2 frames of a 100k-Gaussian shell-clustered model, 200k pairs
    w1 = synth.workload(1, n_override=100_000, views_override=2, tfs_override=1, res_override=256)
    g1, l1, p1 = _project(w1, w1.frames)
    assert p1.n_pairs == 200_000
    E1, st1 = _compare(p1)
    assert E1 > 100_000 and st1[0] == E1 and st1[1] == 0
    # second call, smaller: 1 frame of 20k Gaussians at 160x96
    w2 = synth.workload(1, n_override=20_000, views_override=1, tfs_override=1, res_override=160)
    w2.cameras = [synth.look_at_camera(synth.fibonacci_directions(1)[0], 3.0, 160, 96)]
    g2, l2, p2 = _project(w2, w2.frames)
    E2, st2 = _compare(p2)
    assert 0 < E2 < E1 and st2[0] == E2 and st2[1] == 0


def test_bin_static_reports_an_overflow_like_the_workspace_calls():
    w = synth.workload(1, n_override=30_000, views_override=1, tfs_override=1, res_override=200)
    g, l, p = _project(w, w.frames)
    E, st = _compare(p, cap=1000)
    assert E > 1000 and st[0] == E and st[1] == 1


def test_bin_static_at_its_pair_limit():
    w = synth.workload(1, n_override=262_144, views_override=1, tfs_override=1, res_override=128)
    g, l, p = _project(w, w.frames)
    assert p.n_pairs == 262_144
    E, st = _compare(p)
    assert st[1] == 0
