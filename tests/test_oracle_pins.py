"""Pins of the CPU oracle against closed forms, invariants and finite differences.

None of these re-types an oracle formula: each checks the oracle against something the
paper or the mathematics fixes independently (Eq. 1's closed form for a few samples, the
single-Gaussian EWA closed form, orthonormality of R(q), the pinhole map's finite-difference
Jacobian, libm's exp/log, brute-force pixel enumeration, central finite differences).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

OPTS = dict(synth.DEFAULT_OPTS)


def _axis_camera(z, W=64, H=64, f=None):
    """Camera at the world origin looking down +z (identity rotation), translated by z."""
    f = f if f is not None else (0.5 * H) / math.tan(math.radians(25.0))
    view = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, z], np.float32)
    return synth.Camera(view=view, fx=float(np.float32(f)), fy=float(np.float32(f)),
                        cx=0.5 * W, cy=0.5 * H, width=W, height=H)


def _gaussians(means, scales, v, quats=None, w=None):
    n = len(means)
    q = np.tile(np.array([[1, 0, 0, 0]], np.float32), (n, 1)) if quats is None else np.asarray(quats, np.float32)
    return synth.Gaussians(np.asarray(means, np.float32), np.log(np.asarray(scales, np.float64)).astype(np.float32),
                           q, np.asarray(v, np.float32), None if w is None else np.asarray(w, np.float32))


# ----------------------------------------------------------------------------- exp / log

def _ulps(x32, ref64):
    sp = np.spacing(np.abs(ref64).astype(np.float32)).astype(np.float64)
    return np.abs(x32.astype(np.float64) - ref64) / sp


def test_exp32_within_two_ulp_of_libm():
    rng = np.random.default_rng(1)
    x = np.concatenate([np.linspace(-86.9, 87.9, 400001), rng.uniform(-10, 10, 200000),
                        [0.0, 1.0, -1.0, math.log(2), 1e-8, -1e-8]]).astype(np.float32)
    got = oracle.exp32(x)
    ref = np.exp(x.astype(np.float64))
    assert _ulps(got, ref).max() <= 2.0
    assert oracle.exp32(np.float32(0.0)) == np.float32(1.0)
    assert np.isinf(oracle.exp32(np.float32(88.5)))
    assert oracle.exp32(np.float32(-90.0)) == 0.0


def test_log32_within_two_ulp_of_libm():
    rng = np.random.default_rng(2)
    x = np.concatenate([np.exp(np.linspace(-85, 85, 400001)), rng.uniform(0.5, 2.0, 200000),
                        [1.0, 2.0, 0.5, 255.0, 1.0000001]]).astype(np.float32)
    got = oracle.log32(x)
    ref = np.log(x.astype(np.float64))
    nz = np.abs(ref) > 1e-3
    assert _ulps(got[nz], ref[nz]).max() <= 2.0
    # near 1 the relative error can exceed 2 ulp only through the absolute error floor
    assert np.abs(got[~nz].astype(np.float64) - ref[~nz]).max() <= 2e-10 + 1e-7 * np.abs(ref[~nz]).max()
    assert oracle.log32(np.float32(1.0)) == 0.0


# ----------------------------------------------------------------------------- rotation

def test_quaternion_rotation_is_proper_orthonormal():
    rng = np.random.default_rng(3)
    q = torch.tensor(rng.standard_normal((1000, 4)))
    q = q / q.norm(dim=1, keepdim=True)
    R = oracle.quat_to_rot_f64(q)
    eye = torch.eye(3, dtype=torch.float64)
    assert torch.allclose(R @ R.transpose(-1, -2), eye.expand_as(R), atol=1e-13)
    assert torch.allclose(torch.linalg.det(R), torch.ones(1000, dtype=torch.float64), atol=1e-13)
    assert torch.allclose(oracle.quat_to_rot_f64(-q), R, atol=0)
    # 90 degrees about +z maps x to y
    c = math.cos(math.pi / 4)
    Rz = oracle.quat_to_rot_f64(torch.tensor([[c, 0.0, 0.0, c]], dtype=torch.float64))[0]
    assert torch.allclose(Rz @ torch.tensor([1.0, 0, 0], dtype=torch.float64),
                          torch.tensor([0.0, 1, 0], dtype=torch.float64), atol=1e-15)


# ----------------------------------------------------------------------------- EWA closed form

def test_single_isotropic_gaussian_closed_form():
    """Isotropic Gaussian at the optical axis: Sigma' = ((f s / z)^2 + lowpass) I, so the
    pixel value is c * min(0.99, A exp(-r^2 / (2 ((f s/z)^2 + lowpass))))."""
    z, s, v = 3.0, 0.05, 0.8
    cam = _axis_camera(z)
    g = _gaussians([[0, 0, 0]], [[s, s, s]], [v])
    lut = synth.identity_tf()
    res, proj, order, fp = oracle.render_image(g, cam, lut, OPTS)
    img = res.color.detach().numpy().reshape(64, 64, 3)
    f = float(np.float32(cam.fx))
    s_eff = math.exp(float(g.log_scales[0, 0]))      # the stored log-scale, exponentiated
    var = (f * s_eff / z) ** 2 + 0.3
    # identity LUT: colour = opacity = the table interpolated at v (np.interp on the table)
    vv = float(np.interp(float(np.float32(v)), np.arange(256) / 255.0, lut[:, 0].astype(np.float64)))
    ys, xs = np.mgrid[0:64, 0:64]
    r2 = (xs + 0.5 - 32.0) ** 2 + (ys + 0.5 - 32.0) ** 2
    a = vv * np.exp(-r2 / (2 * var))
    alpha = np.where(a >= float(np.float32(1 / 255)), np.minimum(a, float(np.float32(0.99))), 0.0)
    expect = vv * alpha
    assert np.abs(img[..., 0] - expect).max() < 1e-12
    # O1 footprint: the pixel columns whose centres lie within the alpha >= 1/255 ellipse
    tau = 2 * math.log(vv / float(np.float32(1 / 255)))
    ex = math.sqrt(tau * var)
    lo = math.ceil(32.0 - ex - 0.5) // 16
    hi = math.floor(32.0 + ex - 0.5) // 16
    assert tuple(fp.rect[0]) == (lo, lo, hi, hi)


def test_three_samples_eq1_closed_form():
    """Three Gaussians on the axis at different depths; at a pixel the result must be
    c1 a1 + c2 a2 (1-a1) + c3 a3 (1-a1)(1-a2) (Eq. 1) with the front one first."""
    cam = _axis_camera(3.0)
    vals = [0.3, 0.6, 0.9]
    depths = [0.5, -0.2, 0.1]      # world z; camera z = 3 + world z
    g = _gaussians([[0, 0, d] for d in depths], [[0.05] * 3] * 3, vals)
    lut = synth.identity_tf()
    px = np.array([[33, 30]])
    res, proj, order, fp = oracle.render_image(g, cam, lut, OPTS, pixels=px)
    f = float(np.float32(cam.fx))
    r2 = (33.5 - 32.0) ** 2 + (30.5 - 32.0) ** 2
    items = []
    for d, v in zip(depths, vals):
        z = 3.0 + float(np.float32(d))
        var = (f * math.exp(float(g.log_scales[0, 0])) / z) ** 2 + 0.3
        vv = float(np.interp(float(np.float32(v)), np.arange(256) / 255.0, lut[:, 0].astype(np.float64)))
        a = min(vv * math.exp(-r2 / (2 * var)), float(np.float32(0.99)))
        items.append((z, vv, a))
    items.sort()
    C, T = 0.0, 1.0
    for _, c, a in items:
        C += c * a * T
        T *= 1 - a
    assert abs(res.color[0, 0].item() - C) < 1e-12
    assert abs(res.T[0].item() - T) < 1e-12
    assert list(order) == [1, 2, 0]


def test_ewa_covariance_matches_fd_jacobian_of_pinhole_map():
    """Sigma' - lowpass I = J_pi Sigma J_pi^T with J_pi the (finite-difference) Jacobian of
    the pinhole map mu -> (fx x/z + cx, fy y/z + cy) in world coordinates."""
    rng = np.random.default_rng(4)
    w = synth.workload(0)
    cam = w.cameras[0]
    g = w.gaussians.subset(np.arange(40))
    proj = oracle.project_f64(g.means, g.log_scales, g.quats, g.scalars, None, cam, w.tfs[0], OPTS)
    V = np.asarray(cam.view, np.float64).reshape(3, 4)
    fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy

    def pinhole(mu):
        t = V[:, :3] @ mu + V[:, 3]
        return np.array([fx * t[0] / t[2] + cx, fy * t[1] / t[2] + cy])
    lim = 1.3 * 0.5 * cam.width / fx
    for i in range(g.n):
        mu = g.means[i].astype(np.float64)
        t = V[:, :3] @ mu + V[:, 3]
        if abs(t[0] / t[2]) > lim or abs(t[1] / t[2]) > lim:
            continue
        h = 1e-6
        Jp = np.stack([(pinhole(mu + h * e) - pinhole(mu - h * e)) / (2 * h) for e in np.eye(3)], 1)
        q = g.quats[i].astype(np.float64)
        q /= np.linalg.norm(q)
        R = oracle.quat_to_rot_f64(torch.tensor(q[None]))[0].numpy()
        Sig = R @ np.diag(np.exp(2 * g.log_scales[i].astype(np.float64))) @ R.T
        ref = Jp @ Sig @ Jp.T
        got = proj.cov2d[i].detach().numpy()
        got_m = np.array([[got[0] - 0.3, got[1]], [got[1], got[2] - 0.3]])
        assert np.abs(got_m - ref).max() <= 1e-6 * np.abs(ref).max()


def test_rotated_anisotropic_gaussian_matches_matrix_form():
    """One rotated, anisotropic, off-axis Gaussian: every pixel must equal
    c * min(0.99, A exp(-1/2 d^T S^-1 d)) with S = J_pi Sigma J_pi^T + lowpass I, J_pi the
    finite-difference Jacobian of the pinhole map and S^-1 from numpy.linalg.inv (matrix
    form, so a wrong sign or factor on the conic's cross term fails)."""
    cam = synth.look_at_camera(np.array([0.3, -0.5, 0.8]), 3.0, 48, 40)
    q = np.array([[0.8, 0.3, -0.4, 0.33]], np.float32)
    g = _gaussians([[0.12, -0.07, 0.05]], [[0.25, 0.08, 0.03]], [0.42], quats=q)
    lut = synth.random_tf(np.random.default_rng(11))
    lut[:, 3] = 0.95
    res, proj, order, fp = oracle.render_image(g, cam, lut, OPTS)
    V = np.asarray(cam.view, np.float64).reshape(3, 4)

    def pinhole(mu):
        t = V[:, :3] @ mu + V[:, 3]
        return np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])
    mu = g.means[0].astype(np.float64)
    h = 1e-5
    Jp = np.stack([(pinhole(mu + h * e) - pinhole(mu - h * e)) / (2 * h) for e in np.eye(3)], 1)
    qq = q[0].astype(np.float64) / np.linalg.norm(q[0].astype(np.float64))
    R = oracle.quat_to_rot_f64(torch.tensor(qq[None]))[0].numpy()
    Sig = R @ np.diag(np.exp(2 * g.log_scales[0].astype(np.float64))) @ R.T
    S = Jp @ Sig @ Jp.T + 0.3 * np.eye(2)
    Si = np.linalg.inv(S)
    m2 = pinhole(mu)
    xg = np.arange(256) / 255.0
    v = float(g.scalars[0])
    A = float(np.interp(v, xg, lut[:, 3].astype(np.float64)))
    c = np.array([np.interp(v, xg, lut[:, k].astype(np.float64)) for k in range(3)])
    ys, xs = np.mgrid[0:40, 0:48]
    d = np.stack([xs.reshape(-1) + 0.5 - m2[0], ys.reshape(-1) + 0.5 - m2[1]], 1)
    a = A * np.exp(-0.5 * np.einsum("pi,ij,pj->p", d, Si, d))
    alpha = np.where(a >= float(np.float32(1 / 255)), np.minimum(a, float(np.float32(0.99))), 0.0)
    expect = alpha[:, None] * c[None]
    assert (alpha > 0.1).sum() > 20
    assert np.abs(res.color.detach().numpy() - expect).max() < 1e-7
    con = proj.conic.detach().numpy()[0]
    cov = proj.cov2d.detach().numpy()[0]
    M = np.array([[con[0], con[1]], [con[1], con[2]]]) @ np.array([[cov[0], cov[1]], [cov[1], cov[2]]])
    assert np.abs(M - np.eye(2)).max() < 1e-12


# ----------------------------------------------------------------------------- compositing invariants

def test_white_tf_identity_image_equals_one_minus_T():
    w = synth.workload(0)
    lut = w.tfs[0].copy()
    lut[:, :3] = 1.0
    res, *_ = oracle.render_image(w.gaussians, w.cameras[0], lut, OPTS)
    img = res.color.detach().numpy()
    T = res.T.detach().numpy()
    assert np.abs(img - (1.0 - T)[:, None]).max() < 1e-12
    assert (T >= 0).all() and (T <= 1).all()


def test_permutation_invariance():
    w = synth.workload(0)
    g = w.gaussians
    perm = np.random.default_rng(5).permutation(g.n)
    res_a, *_ = oracle.render_image(g, w.cameras[0], w.tfs[0], OPTS)
    res_b, *_ = oracle.render_image(g.subset(perm), w.cameras[0], w.tfs[0], OPTS)
    da = res_a.color.detach().numpy()
    db = res_b.color.detach().numpy()
    # distinct depths => the same front-to-back sequence => the same sums
    assert np.array_equal(da, db)


def test_transmittance_is_monotone_along_the_list():
    w = synth.workload(0)
    fp = oracle.footprint_f32(w.gaussians, w.cameras[0], w.tfs[0], OPTS)
    proj = oracle.project_f64(w.gaussians.means, w.gaussians.log_scales, w.gaussians.quats,
                              w.gaussians.scalars, None, w.cameras[0], w.tfs[0], OPTS)
    order = oracle.depth_order(fp, proj.kept)
    px = synth.sample_pixels(np.random.default_rng(6), 64, 64, 32)
    prev = np.ones(32)
    for k in range(0, len(order) + 1, 25):
        r = oracle.render_pixels(proj, order[:k], px, OPTS, t_min=0.0)
        T = r.T.detach().numpy()
        assert (T <= prev + 1e-15).all() and (T >= 0).all()
        prev = T


def test_early_stop_bound():
    """Stopping once T < t_min changes the image by at most T_final * max|c|."""
    w = synth.workload(0, n_override=4000)
    lut = w.tfs[0].copy()
    lut[:, 3] = np.maximum(lut[:, 3], 0.6)   # dense enough that many pixels reach t_min
    res_s, *_ = oracle.render_image(w.gaussians, w.cameras[0], lut, OPTS)
    res_n, *_ = oracle.render_image(w.gaussians, w.cameras[0], lut, OPTS, t_min=0.0)
    d = np.abs(res_s.color.detach().numpy() - res_n.color.detach().numpy()).max(1)
    T = res_s.T.detach().numpy()
    assert (d <= T + 1e-15).all()
    stopped = T < 1e-4
    assert stopped.sum() > 0      # the case is exercised
    assert d.max() <= 1e-4


def test_culled_gaussian_changes_nothing():
    w = synth.workload(0)
    g = w.gaussians
    res_a, *_ = oracle.render_image(g, w.cameras[0], w.tfs[0], OPTS)
    # an extra Gaussian in front of everything whose opacity is below the skip threshold
    extra = _gaussians([[0, 0, 0]], [[0.3, 0.3, 0.3]], [0.5], w=[0.9 * (1 / 255) / 1.0])
    lut = w.tfs[0].copy()
    lut[:, 3] = np.maximum(lut[:, 3], 1.0)  # opacity 1, so A = w < 1/255
    g2 = synth.Gaussians(np.concatenate([g.means, extra.means]), np.concatenate([g.log_scales, extra.log_scales]),
                         np.concatenate([g.quats, extra.quats]), np.concatenate([g.scalars, extra.scalars]),
                         np.concatenate([np.ones(g.n, np.float32), extra.weights]))
    res_b, *_ = oracle.render_image(g2, w.cameras[0], lut, OPTS)
    g1 = synth.Gaussians(g.means, g.log_scales, g.quats, g.scalars, np.ones(g.n, np.float32))
    res_c, *_ = oracle.render_image(g1, w.cameras[0], lut, OPTS)
    assert np.array_equal(res_b.color.detach().numpy(), res_c.color.detach().numpy())


# ----------------------------------------------------------------------------- transfer function

def test_identity_lut_gives_value_colour_and_unit_slope():
    v = np.array([0.0, 0.1, 0.25, 0.5, 0.77, 1.0], np.float32)
    g = _gaussians([[0, 0, 0]] * 6, [[0.05] * 3] * 6, v)
    vt = torch.tensor(v.astype(np.float64), requires_grad=True)
    proj = oracle.project_f64(g.means, g.log_scales, g.quats, vt, None, _axis_camera(3.0),
                              synth.identity_tf(), OPTS)
    lutv = synth.identity_tf()[:, 0].astype(np.float64)
    assert np.allclose(proj.rgb.detach().numpy(), np.interp(v, np.arange(256) / 255, lutv)[:, None], atol=1e-7)
    proj.A.sum().backward()
    assert np.allclose(vt.grad.numpy(), 1.0, atol=1e-5)


def test_constant_lut_has_zero_scalar_gradient():
    w = synth.workload(0, n_override=50)
    lut = synth.constant_tf()
    d = np.random.default_rng(7).standard_normal((64 * 64, 3))
    gr = oracle.gradients(w.gaussians, w.cameras[0], lut, OPTS, d)
    assert np.abs(gr.d_scalars).max() == 0.0
    assert np.abs(gr.d_means).max() > 0


def test_knot_derivative_is_right_hand_slope_and_clamped_values_have_none():
    K = 5
    lut = np.zeros((K, 4), np.float32)
    lut[:, 3] = [0.0, 0.1, 0.5, 0.6, 1.0]   # slopes per segment: 0.4, 1.6, 0.4, 1.6
    v = np.array([0.25, 0.5, 1.0, -0.2, 1.3, 0.0], np.float32)
    vt = torch.tensor(v.astype(np.float64), requires_grad=True)
    g = _gaussians([[0, 0, 0]] * 6, [[0.05] * 3] * 6, v)
    proj = oracle.project_f64(g.means, g.log_scales, g.quats, vt, None, _axis_camera(3.0), lut, OPTS)
    proj.A.sum().backward()
    assert np.allclose(vt.grad.numpy(), [1.6, 0.4, 1.6, 0.0, 0.0, 0.4], atol=1e-12)


# ----------------------------------------------------------------------------- O1 footprint and keys

def test_footprint_is_lossless_against_pixel_enumeration():
    """Every pixel where the float64 alpha reaches alpha_min (with a 1e-5 relative margin)
    lies inside O1's tile rectangle, and the rectangle's pixel range is within one pixel of
    the continuous alpha >= alpha_min ellipse's bounding box."""
    w = synth.workload(0)
    g, cam, lut = w.gaussians, w.cameras[0], w.tfs[0]
    fp = oracle.footprint_f32(g, cam, lut, OPTS)
    proj = oracle.project_f64(g.means, g.log_scales, g.quats, g.scalars, None, cam, lut, OPTS)
    ys, xs = np.mgrid[0:64, 0:64]
    pxc, pyc = xs.reshape(-1) + 0.5, ys.reshape(-1) + 0.5
    amin = float(np.float32(1 / 255))
    mu = proj.mean2d.detach().numpy()
    con = proj.conic.detach().numpy()
    A = proj.A.detach().numpy()
    cov = proj.cov2d.detach().numpy()
    checked = 0
    for i in np.nonzero(proj.kept)[0]:
        dx, dy = pxc - mu[i, 0], pyc - mu[i, 1]
        a = A[i] * np.exp(-0.5 * (con[i, 0] * dx * dx + 2 * con[i, 1] * dx * dy + con[i, 2] * dy * dy))
        hit = a >= amin * (1 + 1e-5)
        if not hit.any():
            continue
        assert fp.keep[i]
        tx, ty = xs.reshape(-1)[hit] // 16, ys.reshape(-1)[hit] // 16
        x0, y0, x1, y1 = fp.rect[i]
        assert tx.min() >= x0 and tx.max() <= x1 and ty.min() >= y0 and ty.max() <= y1
        tau = 2 * math.log(A[i] / amin)
        ex, ey = math.sqrt(tau * cov[i, 0]), math.sqrt(tau * cov[i, 2])
        assert abs(fp.ex[i] - ex) <= 1e-5 * ex + 1e-6 and abs(fp.ey[i] - ey) <= 1e-5 * ey + 1e-6
        checked += 1
    assert checked > 100


def test_key_list_invariants():
    w = synth.workload(1, n_override=3000, views_override=2, tfs_override=2, res_override=128)
    fps, cams = [], []
    for (ci, ti) in w.frames:
        fps.append(oracle.footprint_f32(w.gaussians, w.cameras[ci], w.tfs[ti], OPTS))
        cams.append(w.cameras[ci])
    tiles, depths, pairs, ranges, bases = oracle.key_list(fps, cams)
    n = w.gaussians.n
    # sorted by (tile, depth, pair)
    key = (tiles.astype(np.uint64) << np.uint64(32)) | depths.astype(np.uint64)
    assert (np.diff(key.astype(np.float64)) >= 0).all()
    same = np.diff(key) == 0
    assert (np.diff(pairs)[same] > 0).all()
    # pair i appears count_i times
    cnt = np.bincount(pairs, minlength=n * len(fps))
    assert np.array_equal(cnt, np.concatenate([fp.count for fp in fps]))
    # ranges partition [0, E)
    nz = ranges[:, 1] > ranges[:, 0]
    assert (ranges[nz, 1] - ranges[nz, 0]).sum() == tiles.shape[0]
    for t in np.nonzero(nz)[0][:200]:
        assert (tiles[ranges[t, 0]:ranges[t, 1]] == t).all()


# ----------------------------------------------------------------------------- gradients

def _loss(g, cam, lut, d):
    res, *_ = oracle.render_image(g, cam, lut, OPTS)
    return float((res.color.detach().numpy() * d).sum())


@pytest.mark.parametrize("with_weights", [False, True])
def test_autograd_gradients_match_central_finite_differences(with_weights):
    rng = np.random.default_rng(8)
    n = 12
    g = synth.uniform_gaussians(rng, n, 0.08, 0.25, box=0.5)
    g.means = g.means.astype(np.float32)
    if with_weights:
        g.weights = rng.uniform(0.3, 1.0, n).astype(np.float32)
    cam = synth.look_at_camera(synth.random_direction(rng), 3.0, 32, 32)
    lut = synth.random_tf(rng)
    lut[:, 3] = np.clip(lut[:, 3] + 0.3, 0, 0.8)
    d = rng.standard_normal((32 * 32, 3))
    gr = oracle.gradients(g, cam, lut, OPTS, d)
    res, *_ = oracle.render_image(g, cam, lut, OPTS)
    assert not res.flag.any() and not res.flag_grad.any()

    def fd(field, idx):
        base = getattr(g, field)
        x0 = float(base[idx])
        h = 1e-6 * max(1.0, abs(x0))
        out = []
        for sgn in (1, -1):
            gg = synth.Gaussians(g.means.astype(np.float64), g.log_scales.astype(np.float64),
                                 g.quats.astype(np.float64), g.scalars.astype(np.float64),
                                 None if g.weights is None else g.weights.astype(np.float64))
            arr = getattr(gg, field)
            arr[idx] = x0 + sgn * h
            out.append(_loss_f64(gg, cam, lut, d))
        return (out[0] - out[1]) / (2 * h)

    fields = [("means", gr.d_means), ("log_scales", gr.d_log_scales), ("quats", gr.d_quats), ("scalars", gr.d_scalars)]
    if with_weights:
        fields.append(("weights", gr.d_weights))
    for field, grad in fields:
        flat = [np.unravel_index(k, grad.shape) for k in range(grad.size)]
        scale = np.abs(grad).max()
        assert scale > 0
        for idx in flat[:: max(1, len(flat) // 16)]:
            num = fd(field, idx)
            assert abs(num - grad[idx]) <= 1e-6 * scale + 1e-9, (field, idx, num, grad[idx])


def _loss_f64(g, cam, lut, d):
    """Loss with float64 parameters (FD needs perturbations below float32 resolution).
    The depth order and cull decisions of the unperturbed float32 inputs are kept."""
    g32 = synth.Gaussians(g.means.astype(np.float32), g.log_scales.astype(np.float32), g.quats.astype(np.float32),
                          g.scalars.astype(np.float32), None if g.weights is None else g.weights.astype(np.float32),
                          None if g.shading is None else g.shading.astype(np.float32))
    fp = oracle.footprint_f32(g32, cam, lut, OPTS)
    sh = None if g.shading is None else (g.shading.normals, g.shading.k_ambient, g.shading.k_diffuse,
                                         g.shading.k_specular, g.shading.shininess)
    proj = oracle.project_f64(g.means, g.log_scales, g.quats, g.scalars, g.weights, cam, lut, OPTS, shading=sh)
    order = oracle.depth_order(fp, proj.kept)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    px = np.stack([xs.reshape(-1), ys.reshape(-1)], 1)
    r = oracle.render_pixels(proj, order, px, OPTS)
    return float((r.color.detach().numpy() * d).sum())


def test_flagged_fraction_is_small_on_the_small_workload():
    w = synth.workload(0)
    res, *_ = oracle.render_image(w.gaussians, w.cameras[0], w.tfs[0], OPTS)
    assert res.flag.mean() <= 1e-2


# ----------------------------------------------------------------------------- lighting

def _shading(n, normals=None, ka=0.2, kd=0.6, ks=0.3, beta=3.0):
    nrm = np.tile(np.array([[0, 0, 1]], np.float32), (n, 1)) if normals is None else np.asarray(normals, np.float32)
    full = lambda x: np.full(n, x, np.float32)
    return synth.Shading(nrm, full(ka), full(kd), full(ks), full(beta))


def _proj_rgb(g, cam, lut):
    sh = None if g.shading is None else (g.shading.normals, g.shading.k_ambient, g.shading.k_diffuse,
                                         g.shading.k_specular, g.shading.shininess)
    p = oracle.project_f64(g.means, g.log_scales, g.quats, g.scalars, g.weights, cam, lut, OPTS, shading=sh)
    return p.rgb.detach().numpy()


def test_shading_with_only_ambient_light_is_the_tf_colour():
    rng = np.random.default_rng(31)
    g = synth.uniform_gaussians(rng, 50, 0.02, 0.1, box=0.5)
    cam = synth.look_at_camera(synth.random_direction(rng), 3.0, 48, 48)
    lut = synth.random_tf(rng)
    plain = _proj_rgb(g, cam, lut)
    g.shading = _shading(g.n, normals=rng.standard_normal((g.n, 3)), ka=1.0, kd=0.0, ks=0.0, beta=5.0)
    assert np.array_equal(_proj_rgb(g, cam, lut), plain)


def test_shading_headlight_closed_forms():
    """Camera on the z axis looking at the origin (its centre at (0, 0, -3)), identity TF at
    v = 1 so that C(v) = 1 exactly: with k_a = 1/4, k_d = 1/2, k_s = 3/8 and beta = 3, Eq. 2-3
    give c = 1/4 + s/2 + 3/8 s^3 with s = |n . l| for the unit direction l from the camera:
    9/8 at s = 1, 35/64 at s = 1/2, 1/4 at s = 0 (no specular term)."""
    cam = _axis_camera(3.0)
    lut = synth.identity_tf(256)
    c60, s60 = math.cos(math.radians(60.0)), math.sin(math.radians(60.0))
    normals = [[0, 0, 1], [0, 0, -2], [s60, 0, c60], [0, -s60, -c60], [1, 0, 0], [0, 3, 0]]
    n = len(normals)
    g = _gaussians([[0, 0, 0]] * n, [[0.05] * 3] * n, [1.0] * n)
    g.shading = _shading(n, normals=normals, ka=0.25, kd=0.5, ks=0.375, beta=3.0)
    rgb = _proj_rgb(g, cam, lut)
    want = [9 / 8, 9 / 8, 35 / 64, 35 / 64, 1 / 4, 1 / 4]
    for i, w in enumerate(want):
        assert np.allclose(rgb[i], w, atol=1e-7, rtol=0), (i, rgb[i], w)
    # off-axis centre: the light direction is the centre's own direction from the camera
    mu = np.array([[0.6, -0.4, 0.5]])
    towards_camera = np.array([0.0, 0.0, -3.0]) - mu
    g2 = _gaussians(mu, [[0.05] * 3], [1.0])
    g2.shading = _shading(1, normals=towards_camera, ka=0.25, kd=0.5, ks=0.375, beta=3.0)
    assert np.allclose(_proj_rgb(g2, cam, lut)[0], 9 / 8, atol=1e-6)


def test_shading_gradients_match_central_finite_differences():
    rng = np.random.default_rng(32)
    n = 10
    g = synth.uniform_gaussians(rng, n, 0.08, 0.25, box=0.5)
    g.shading = synth.random_shading(rng, n, shininess=(1.5, 8.0))
    cam = synth.look_at_camera(synth.random_direction(rng), 3.0, 32, 32)
    lut = synth.random_tf(rng)
    lut[:, 3] = np.clip(lut[:, 3] + 0.3, 0, 0.8)
    d = rng.standard_normal((32 * 32, 3))
    gr = oracle.gradients(g, cam, lut, OPTS, d)
    res, *_ = oracle.render_image(g, cam, lut, OPTS)
    assert not res.flag.any() and not res.flag_grad.any()

    def fd(field, idx):
        sub, name = field.split(".") if "." in field else (None, field)
        x0 = float((getattr(g.shading, name) if sub else getattr(g, name))[idx])
        h = 1e-6 * max(1.0, abs(x0))
        out = []
        for sgn in (1, -1):
            gg = synth.Gaussians(g.means.astype(np.float64), g.log_scales.astype(np.float64),
                                 g.quats.astype(np.float64), g.scalars.astype(np.float64), None,
                                 g.shading.astype(np.float64))
            arr = getattr(gg.shading, name) if sub else getattr(gg, name)
            arr[idx] = x0 + sgn * h
            out.append(_loss_f64(gg, cam, lut, d))
        return (out[0] - out[1]) / (2 * h)

    fields = [("shading.normals", gr.d_normals), ("shading.k_ambient", gr.d_k_ambient),
              ("shading.k_diffuse", gr.d_k_diffuse), ("shading.k_specular", gr.d_k_specular),
              ("shading.shininess", gr.d_shininess), ("means", gr.d_means), ("scalars", gr.d_scalars)]
    for field, grad in fields:
        flat = [np.unravel_index(k, grad.shape) for k in range(grad.size)]
        scale = np.abs(grad).max()
        assert scale > 0, field
        for idx in flat[:: max(1, len(flat) // 12)]:
            num = fd(field, idx)
            assert abs(num - grad[idx]) <= 1e-6 * scale + 1e-9, (field, idx, num, grad[idx])


# ----------------------------------------------------------------------------- training-loop neighbours

def test_ssim_of_an_image_with_itself_is_one_and_has_zero_gradient():
    rng = np.random.default_rng(50)
    x = rng.uniform(0, 1, (3, 20, 24))
    s = oracle.ssim_map(x, x).numpy()
    assert np.abs(s - 1.0).max() < 1e-12
    loss, grad = oracle.ssim_loss(x, x, 0.7)
    assert abs(loss) < 1e-10 and np.abs(grad).max() < 1e-10


def test_ssim_of_constant_images_in_the_interior():
    """Away from the border (5 px) the windowed mean of a constant image a is a and both
    variances and the covariance vanish, so SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    s = oracle.ssim_map(np.full((1, 16, 18), a), np.full((1, 16, 18), b)).numpy()[0]
    want = (2 * a * b + oracle.SSIM_C1) / (a * a + b * b + oracle.SSIM_C1)
    assert np.abs(s[5:-5, 5:-5] - want).max() < 1e-12
    assert np.abs(s[0, 0] - want) > 1e-3          # zero padding shows at the border


def test_ssim_map_matches_a_brute_force_window_sum():
    rng = np.random.default_rng(51)
    x, y = rng.uniform(0, 1, (1, 9, 8)), rng.uniform(0, 1, (1, 9, 8))
    g = oracle.ssim_window_1d()
    assert abs(g.sum() - 1.0) < 1e-15
    H, W = x.shape[1:]
    ref = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            acc = np.zeros(5)
            for u in range(11):
                for v in range(11):
                    ii, jj = i + u - 5, j + v - 5
                    if 0 <= ii < H and 0 <= jj < W:
                        wgt = g[u] * g[v]
                        a, b = x[0, ii, jj], y[0, ii, jj]
                        acc += wgt * np.array([a, b, a * a, b * b, a * b])
            mx, my, ex2, ey2, exy = acc
            sx, sy, sxy = ex2 - mx * mx, ey2 - my * my, exy - mx * my
            ref[i, j] = ((2 * mx * my + 1e-4) * (2 * sxy + 9e-4)) / ((mx * mx + my * my + 1e-4) * (sx + sy + 9e-4))
    assert np.abs(oracle.ssim_map(x, y).numpy()[0] - ref).max() < 1e-12


def test_ssim_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(52)
    x, y = rng.uniform(0.1, 0.9, (2, 12, 13)), rng.uniform(0.1, 0.9, (2, 12, 13))
    loss, grad = oracle.ssim_loss(x, y, 0.25)
    for idx in [(0, 0, 0), (0, 6, 7), (1, 11, 12), (1, 3, 9), (0, 11, 0)]:
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        num = (oracle.ssim_loss(xp, y, 0.25)[0] - oracle.ssim_loss(xm, y, 0.25)[0]) / (2 * h)
        assert abs(num - grad[idx]) <= 1e-7 * max(1.0, abs(grad[idx])), (idx, num, grad[idx])


def test_adam_closed_forms():
    """Bias correction makes the first update lr * g / (|g| + eps) for any beta; with a
    constant gradient m^ = g and v^ = g^2 at every step, so each step moves by the same
    amount; with beta1 = beta2 = 0 Adam is sign descent."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    lr, eps = 0.01, 1e-15
    p1, m, v = oracle.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, lr, eps=eps)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    p = p0
    m = v = np.zeros(4)
    for t in range(1, 6):
        p, m, v = oracle.adam_step(p, g, m, v, t, lr, eps=eps)
    assert np.allclose(p, p0 - 5 * lr * np.sign(g), rtol=0, atol=1e-12)
    q, _, _ = oracle.adam_step(p0, g, np.ones(4), np.ones(4), 7, lr, beta1=0.0, beta2=0.0, eps=eps)
    assert np.allclose(q, p0 - lr * np.sign(g), rtol=0, atol=1e-12)


def test_densify_stats_of_a_constructed_gradient():
    g2d = np.zeros((2, 3, 9))
    g2d[0, 0, :2] = (3.0, 4.0)
    g2d[1, 0, :2] = (-6.0, 8.0)
    g2d[0, 1, :2] = (1.0, 0.0)
    g2d[1, 2, :2] = (5.0, 12.0)
    kept = np.array([[True, True, False], [True, False, False]])
    acc, cnt = oracle.densify_stats(g2d, kept)
    assert np.allclose(acc, [15.0, 1.0, 0.0]) and list(cnt) == [2, 1, 0]


# ---------------------------------------------------------------------------------------
# Opacity-guided training family and the key list shared by a view's transfer functions
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("n_steps", [5, 10, 20])
def test_tent_opacity_maps_follow_the_stated_rule(n_steps):
    """Section "Training": one map per step of the scalar range, centred in its step, linear
    drop-off with slope equal to the number of steps; together they weight the range
    equally (partition of unity between the first and last centres)."""
    x = np.linspace(0, 1, 20001)
    maps = np.stack([synth.tent_opacity(x, n_steps, j) for j in range(n_steps)])
    assert maps.min() >= 0 and maps.max() <= 1
    for j in range(n_steps):
        c = (j + 0.5) / n_steps
        assert synth.tent_opacity(c, n_steps, j) == 1.0
        h = 0.25 / n_steps
        slope = (synth.tent_opacity(c - h, n_steps, j) - synth.tent_opacity(c - 2 * h, n_steps, j)) / h
        assert abs(slope - n_steps) <= 1e-9 * n_steps
        far = np.abs(x - c) >= 1.0 / n_steps
        assert np.all(maps[j][far] == 0)
    inner = (x >= 0.5 / n_steps) & (x <= 1 - 0.5 / n_steps)
    assert np.allclose(maps.sum(0)[inner], 1.0, atol=1e-12)
    lut = synth.tent_tfs(n_steps)
    assert len(lut) == n_steps and lut[0].shape == (256, 4)
    assert np.allclose(lut[3][:, 3], synth.tent_opacity(np.arange(256) / 255, n_steps, 3), atol=1e-7)


def _shared_case(n=1000, res=64):
    w = synth.workload(0, n_override=n, res_override=res)
    luts = [synth.random_tf(synth.rng_for(0, 70 + k)) for k in range(3)] + synth.tent_tfs(10)[2:5]
    return w.gaussians, w.cameras[0], luts


def test_shared_footprint_contains_every_frames_footprint():
    g, cam, luts = _shared_case()
    union = oracle.footprint_shared_f32(g, cam, luts, OPTS)
    fps = [oracle.footprint_f32(g, cam, lut, OPTS) for lut in luts]
    assert np.array_equal(union.keep, np.any([fp.keep for fp in fps], axis=0))
    for fp in fps:
        k = fp.keep
        assert np.all(union.rect[k, 0] <= fp.rect[k, 0]) and np.all(union.rect[k, 1] <= fp.rect[k, 1])
        assert np.all(union.rect[k, 2] >= fp.rect[k, 2]) and np.all(union.rect[k, 3] >= fp.rect[k, 3])
        assert np.all(union.count >= fp.count)
    assert np.array_equal(union.depth_bits, fps[0].depth_bits)
    # with one table the shared footprint is that table's own, field for field
    one = oracle.footprint_shared_f32(g, cam, luts[:1], OPTS)
    for name in ("keep", "rect", "count", "ex", "ey"):
        assert np.array_equal(getattr(one, name), getattr(fps[0], name)), name
    # some Gaussians are kept by some tables only, so the shared list is a strict union
    some = np.any([fp.keep for fp in fps], axis=0) & ~np.all([fp.keep for fp in fps], axis=0)
    assert some.sum() > 50


def test_shared_footprint_is_lossless_for_every_table():
    """Every pixel where any table's float64 alpha reaches alpha_min lies in the shared
    rectangle (pixel enumeration, as for a single table)."""
    g, cam, luts = _shared_case()
    union = oracle.footprint_shared_f32(g, cam, luts, OPTS)
    ys, xs = np.mgrid[0:64, 0:64]
    pxc, pyc = xs.reshape(-1) + 0.5, ys.reshape(-1) + 0.5
    amin = float(np.float32(1 / 255))
    checked = 0
    for lut in luts:
        proj = oracle.project_f64(g.means, g.log_scales, g.quats, g.scalars, None, cam, lut, OPTS)
        mu, con, A = (proj.mean2d.detach().numpy(), proj.conic.detach().numpy(), proj.A.detach().numpy())
        for i in np.nonzero(proj.kept)[0]:
            dx, dy = pxc - mu[i, 0], pyc - mu[i, 1]
            a = A[i] * np.exp(-0.5 * (con[i, 0] * dx * dx + 2 * con[i, 1] * dx * dy + con[i, 2] * dy * dy))
            hit = a >= amin * (1 + 1e-5)
            if not hit.any():
                continue
            assert union.keep[i]
            tx, ty = xs.reshape(-1)[hit] // 16, ys.reshape(-1)[hit] // 16
            x0, y0, x1, y1 = union.rect[i]
            assert tx.min() >= x0 and tx.max() <= x1 and ty.min() >= y0 and ty.max() <= y1
            checked += 1
    assert checked > 300


# ---------------------------------------------------------------------------------------
# Vector-quantised model storage
# ---------------------------------------------------------------------------------------

def test_vq_round_trip_recovers_a_model_built_from_codewords():
    """A model whose rows are codewords encodes to its own indices (nearest row at distance
    0) and decodes back bit for bit; the fields split the row in order."""
    rng = np.random.default_rng(3)
    book = rng.standard_normal((50, 7)).astype(np.float32)
    idx = rng.integers(0, 50, 2000)
    x = book[idx]
    enc, b2 = synth.vq_encode(np.random.default_rng(4), x, 50, iters=3)
    ls, q = oracle.vq_decode(enc, b2, [3, 4])
    assert np.array_equal(np.concatenate([ls, q], 1), x)
    # a codebook of one row decodes every Gaussian to that row; widths of one give [n] arrays
    a, b, c = oracle.vq_decode(np.zeros(5, np.uint16), np.array([[1.0, 2.0, 3.0]], np.float32), [1, 1, 1])
    assert a.shape == (5,) and np.all(a == 1) and np.all(b == 2) and np.all(c == 3)


def test_vq_out_of_range_index_culls_the_gaussian():
    g = synth.workload(0, n_override=200).gaussians
    book = np.concatenate([g.log_scales[:10], g.quats[:10]], 1).astype(np.float32)
    idx = np.arange(200) % 12                # rows 10 and 11 do not exist
    ls, q = oracle.vq_decode(idx, book, [3, 4])
    bad = idx >= 10
    assert np.all(np.isnan(ls[bad])) and np.all(np.isnan(q[bad])) and np.isfinite(ls[~bad]).all()
    g2 = synth.Gaussians(g.means, ls, q, g.scalars, g.weights)
    cam, lut = synth.workload(0).cameras[0], synth.workload(0).tfs[0]
    fp = oracle.footprint_f32(g2, cam, lut, OPTS)
    assert not fp.keep[bad].any()


def test_vq_encoding_reduces_distortion_with_iterations():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3000, 7)).astype(np.float32)

    def distortion(iters):
        idx, book = synth.vq_encode(np.random.default_rng(6), x, 64, iters=iters)
        (rows,) = oracle.vq_decode(idx, book, [7])
        return float(((rows - x) ** 2).sum())
    d0, d4 = distortion(0), distortion(4)
    assert d4 < d0


# ---------------------------------------------------------------------------------------
# Adaptive density control
# ---------------------------------------------------------------------------------------

def test_densify_plan_decisions_by_hand():
    """Six Gaussians built to land in each branch (thresholds: gradient 0.5, log-scale -2,
    weight 0.005)."""
    acc = np.array([0.0, 3.0, 3.0, 0.9, 3.0, 10.0], np.float32)
    vis = np.array([0, 4, 4, 2, 4, 1], np.int32)          # means: 0, .75, .75, .45, .75, 10
    ls = np.full((6, 3), -3.0, np.float32)
    ls[2, 1] = -1.0                                        # large: split instead of clone
    w = np.array([0.5, 0.5, 0.5, 0.5, 0.001, np.nan], np.float32)
    act, cnt = oracle.densify_plan(acc, vis, ls, w, 0.5, -2.0, 0.005)
    assert list(act) == [oracle.KEEP, oracle.CLONE, oracle.SPLIT, oracle.KEEP, oracle.PRUNE, oracle.PRUNE]
    assert list(cnt) == [2, 1, 1, 2]
    act2, _ = oracle.densify_plan(acc, vis, ls, None, 0.5, -2.0, 0.005)   # no weights: no pruning
    assert list(act2) == [0, 1, 2, 0, 1, 1]


def test_densify_apply_layout_and_split_children_closed_form():
    """Survivors, then clone copies, then split children; with z = +e_x and -e_x the two
    children of a Gaussian rotated 90 degrees about z sit at mu +- s_x e_y, and their scales
    are the parent's divided by 1.6; new Gaussians get zero optimizer moments."""
    act = np.array([oracle.KEEP, oracle.SPLIT, oracle.CLONE, oracle.PRUNE, oracle.SPLIT], np.uint8)
    means = np.arange(15, dtype=np.float64).reshape(5, 3)
    ls = np.log(np.array([[0.1, 0.2, 0.3]] * 5))
    c = math.cos(math.pi / 4)
    quats = np.array([[1, 0, 0, 0], [c, 0, 0, c], [1, 0, 0, 0], [1, 0, 0, 0], [2, 0, 0, 0]], np.float64)
    z = np.zeros((5, 2, 3))
    z[1, 0, 0], z[1, 1, 0] = 1.0, -1.0
    z[4, 0, 1], z[4, 1, 2] = 1.0, 1.0
    w = np.arange(5, dtype=np.float64)
    mom = np.ones((5, 3))
    m2, ls2, w2, mom2 = oracle.densify_apply(act, means, ls, quats, z, [(means, 1), (ls, 2), (w, 0), (mom, 3)])
    # n + clones + splits - prunes = 5 + 1 + 2 - 1
    assert m2.shape == (7, 3) and ls2.shape == (7, 3) and mom2.shape == (7, 3)
    # survivors 0 and 2, the copy of 2, the children of 1 and of 4
    assert list(w2) == [0.0, 2.0, 2.0, 1.0, 1.0, 4.0, 4.0]
    assert np.array_equal(m2[:3], means[[0, 2, 2]]) and np.array_equal(ls2[:3], ls[[0, 2, 2]])
    assert np.all(mom2[:2] == 1.0) and np.all(mom2[2:] == 0.0)
    # a rotation of 90 degrees about z maps e_x to e_y
    assert np.allclose(m2[3], means[1] + [0, 0.1, 0]) and np.allclose(m2[4], means[1] - [0, 0.1, 0])
    # the unnormalised quaternion (2, 0, 0, 0) is the identity: mu + 0.2 e_y and mu + 0.3 e_z
    assert np.allclose(m2[5], means[4] + [0, 0.2, 0]) and np.allclose(m2[6], means[4] + [0, 0, 0.3])
    assert np.allclose(np.exp(ls2[3:]), np.array([[0.1, 0.2, 0.3]]) / 1.6)
