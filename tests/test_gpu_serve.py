"""The continuous-batching server: results identical alone and in a mixed batch, identical
to the stateless path, within the oracle's tolerance; overflow retry, budget rejection and
invalid requests."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import compare_image, image_pixels, luts_to_dev, to_dev

pytestmark = pytest.mark.gpu


def _models():
    rng = synth.rng_for(3, 500)
    a = synth.clustered_gaussians(rng, 20000, 0.7, 0.01, 0.08)
    b = synth.clustered_gaussians(rng, 60000, 0.7, 0.002, 0.03)
    return [a, b]


def _requests(n, seed=0):
    rng = synth.rng_for(3, 600 + seed)
    res = [(96, 64), (128, 128), (200, 120)]
    out = []
    for i in range(n):
        cam = synth.look_at_camera(synth.random_direction(rng), float(rng.uniform(2.5, 4.0)),
                                   *res[int(rng.integers(0, 3))])
        out.append((int(rng.integers(0, 2)), cam, synth.random_tf(rng)))
    return out


def _server(**kw):
    from paper_2504_13339_amd.serve import Server
    args = dict(max_gaussians=60000, max_entries=3_000_000, max_batch=6, n_streams=2, use_graphs=True,
                max_width=256, max_height=256)
    args.update(kw)
    return Server(**args)


@pytest.mark.parametrize("use_graphs", [True, False])
def test_served_images_are_identical_alone_in_the_mix_and_stateless(use_graphs):
    from paper_2504_13339_amd import render as R
    models = _models()
    reqs = _requests(14)
    with _server(use_graphs=use_graphs) as srv:
        mids = [srv.add_model(to_dev(m)) for m in models]
        outs_mix = [torch.full((3, c.height, c.width), -1.0, device="cuda") for _, c, _ in reqs]
        ids = [srv.submit(mids[m], c, tf, outs_mix[i]) for i, (m, c, tf) in enumerate(reqs)]
        for rid in ids:
            srv.wait(rid)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["batches"] < len(reqs)   # batching happened
        outs_alone = []
        for i, (m, c, tf) in enumerate(reqs):   # one at a time, several graph replays
            o = torch.full((3, c.height, c.width), -1.0, device="cuda")
            srv.wait(srv.submit(mids[m], c, tf, o))
            outs_alone.append(o)
            torch.cuda.synchronize()
            # eager work between replays
            _ = torch.randn(1000, device="cuda").sum().item()
    dev_models = [to_dev(m) for m in models]
    for i, (m, c, tf) in enumerate(reqs):
        assert torch.equal(outs_mix[i], outs_alone[i]), i
        st = R.render(dev_models[m], [c], luts_to_dev([tf]), synth.DEFAULT_OPTS)
        assert torch.equal(st.image[0], outs_mix[i]), i


def test_served_request_matches_oracle():
    models = _models()
    m, c, tf = _requests(1, seed=3)[0]
    with _server() as srv:
        mid = srv.add_model(to_dev(models[1]))
        out = torch.empty((3, c.height, c.width), device="cuda")
        srv.wait(srv.submit(mid, c, tf, out))
    res, *_ = oracle.render_image(models[1], c, tf, synth.DEFAULT_OPTS)
    compare_image(image_pixels(out), res)


def test_overflow_is_retried_alone():
    """Huge Gaussians cover most tiles.  The first request views them from far away (a short
    key list, so the server learns a small entry estimate); the following close-up
    requests are then packed into one batch whose key list overflows the slot, and they are
    re-run one by one, correctly."""
    from paper_2504_13339_amd import render as R
    rng = synth.rng_for(3, 700)
    big = synth.uniform_gaussians(rng, 2000, 0.4, 0.9, box=0.8)
    tf = synth.constant_tf(256, (0.4, 0.7, 0.2, 0.3))
    cams = [synth.look_at_camera(synth.random_direction(rng), 40.0 if i == 0 else 3.5, 200, 120) for i in range(6)]
    with _server(max_entries=400_000, max_batch=6, n_streams=1) as srv:
        mid = srv.add_model(to_dev(big))
        outs = [torch.empty((3, 120, 200), device="cuda") for _ in cams]
        ids = [srv.submit(mid, c, tf, outs[i]) for i, c in enumerate(cams)]
        for rid in ids:
            srv.wait(rid)
        st = srv.stats()
    assert st["retries"] > 0 and st["completed"] == len(cams)
    g = to_dev(big)
    for i, c in enumerate(cams):
        ref = R.render(g, [c], luts_to_dev([tf]), synth.DEFAULT_OPTS)
        assert i == 0 or ref.n_entries > 60_000
        assert torch.equal(ref.image[0], outs[i])


def test_budget_rejection_and_invalid_requests():
    from paper_2504_13339_amd._lib import VegError
    models = _models()
    m, c, tf = _requests(1, seed=7)[0]
    with _server(budget_bytes=1 << 16) as srv:
        mid = srv.add_model(to_dev(models[0]))
        out = torch.empty((3, c.height, c.width), device="cuda")
        with pytest.raises(VegError) as ei:
            srv.submit(mid, c, tf, out)
        assert ei.value.status == 3          # VEG_ERR_OUT_OF_BUDGET
        with pytest.raises(VegError) as ei:
            srv.submit(7, c, tf, out)
        assert ei.value.status == 4          # VEG_ERR_NOT_FOUND
        big = synth.look_at_camera(np.array([0, 0, 1.0]), 3.0, 512, 512)
        with pytest.raises(VegError) as ei:
            srv.submit(mid, big, tf, out)
        assert ei.value.status == 1          # VEG_ERR_INVALID_ARG
        assert srv.stats()["rejected"] == 1
