"""Blinn-Phong lighting (Eq. 2-3, headlight): the HIP path against the oracle, for the image
and for every parameter gradient including the lighting attributes; exact identities."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import compare_image, hip, image_pixels, luts_to_dev, rel_err, to_dev

pytestmark = pytest.mark.gpu

OPTS = dict(synth.DEFAULT_OPTS)


def _lit_workload(n=1000, res=64, seed=40):
    w = synth.workload(0, n_override=n, res_override=res)
    w.gaussians.shading = synth.random_shading(synth.rng_for(0, seed), w.gaussians.n)
    return w


def test_lit_image_matches_oracle():
    V, R = hip()
    w = _lit_workload()
    cam, tf = w.cameras[0], w.tfs[0]
    st = R.render(to_dev(w.gaussians), [cam], luts_to_dev([tf]), OPTS)
    res, *_ = oracle.render_image(w.gaussians, cam, tf, OPTS)
    compare_image(image_pixels(st.image[0]), res)


def test_lit_gradients_match_oracle_adjoint():
    V, R = hip()
    w = _lit_workload(seed=41)
    cam, tf = w.cameras[0], w.tfs[0]
    g = to_dev(w.gaussians)
    st = R.render(g, [cam], luts_to_dev([tf]), OPTS)
    res, *_ = oracle.render_image(w.gaussians, cam, tf, OPTS)
    d = np.random.default_rng(42).standard_normal((cam.width * cam.height, 3))
    d[res.flag | res.flag_grad] = 0.0
    d_img = torch.as_tensor(d.T.reshape(1, 3, cam.height, cam.width).copy(), dtype=torch.float32).cuda()
    grads = R.Grads.zeros(g)
    R.render_backward(g, st, d_img, grads)
    torch.cuda.synchronize()
    ref = oracle.gradients(w.gaussians, cam, tf, OPTS, d)
    for name in ("d_means", "d_log_scales", "d_quats", "d_scalars", "d_normals", "d_k_ambient", "d_k_diffuse",
                 "d_k_specular", "d_shininess"):
        assert rel_err(getattr(grads, name).cpu().numpy(), getattr(ref, name)) <= 1e-3, name


def test_ambient_only_lighting_equals_the_unlit_image_bitwise():
    V, R = hip()
    w = synth.workload(0)
    g = w.gaussians
    cam, tf = w.cameras[0], w.tfs[0]
    plain = R.render(to_dev(g), [cam], luts_to_dev([tf]), OPTS).image
    g.shading = synth.random_shading(synth.rng_for(0, 43), g.n, k_ambient=(1.0, 1.0), k_diffuse=(0.0, 0.0),
                                     k_specular=(0.0, 0.0))
    lit = R.render(to_dev(g), [cam], luts_to_dev([tf]), OPTS).image
    assert torch.equal(plain, lit)


def test_lit_model_through_the_server_equals_the_stateless_path():
    V, R = hip()
    from paper_2504_13339_amd.serve import Server
    w = _lit_workload(n=20000, res=128, seed=44)
    g = to_dev(w.gaussians)
    cam, tf = w.cameras[0], w.tfs[0]
    ref = R.render(g, [cam], luts_to_dev([tf]), OPTS).image[0]
    with Server(max_gaussians=20000, max_entries=2_000_000, max_batch=2, n_streams=1, max_width=128,
                max_height=128) as srv:
        mid = srv.add_model(g)
        out = torch.empty((3, cam.height, cam.width), device="cuda")
        srv.wait(srv.submit(mid, cam, tf, out))
    assert torch.equal(out, ref)


def test_autograd_function_carries_lighting_gradients():
    V, R = hip()
    w = _lit_workload(n=2000, seed=45)
    cam, tf = w.cameras[0], w.tfs[0]
    g = to_dev(w.gaussians)
    leaves = [t.clone().requires_grad_(True) for t in (g.means, g.log_scales, g.quats, g.scalars)]
    lit = [getattr(g, k).clone().requires_grad_(True) for k in V.LIGHTING]
    img = R.render_autograd(*leaves, None, [cam], luts_to_dev([tf]), OPTS, lighting=lit)
    d = torch.randn(img.shape, generator=torch.Generator().manual_seed(46)).cuda()
    (img * d).sum().backward()
    st = R.render(g, [cam], luts_to_dev([tf]), OPTS)
    grads = R.Grads.zeros(g)
    R.render_backward(g, st, d, grads)
    torch.cuda.synchronize()
    for t, name in zip(lit, ("d_normals", "d_k_ambient", "d_k_diffuse", "d_k_specular", "d_shininess")):
        assert rel_err(t.grad.cpu().numpy(), getattr(grads, name).cpu().numpy()) <= 1e-5, name
