"""Pins of the oracle's decision margins, of the key list's tile membership and of the L1
term, each against something fixed independently of the oracle's own code:

* decision margins (``render_pixels``' ``slack`` and flags): hand-built Gaussians sit on a
  pixel centre (sigma = 0, so a = A exactly), next to the skip or the stop threshold; the
  decision is flipped by nudging alpha_min or t_min, and the pixel must move by no more
  than ``slack``, which must equal its closed form (the per-evaluation error bound of the
  float32 renderer, the transmittance in front of the Gaussian, the sum over decisions);
  the error bound itself is checked against a float32 emulation of the exponent;
* the key list: every tile's list equals a brute-force enumeration of the Gaussians whose
  tile rectangle covers it, and every pixel a Gaussian reaches is in a tile whose list
  holds it (two frames of different, non-square sizes);
* L1: a hand-computed case, central differences, sign(0) = 0.
"""
import math

import numpy as np
import torch

import oracle
import synth
from oracle import veg_oracle as vo

OPTS = dict(synth.DEFAULT_OPTS)
U = 2.0 ** -24
AMIN = float(np.float32(OPTS["alpha_min"]))
TMIN = float(np.float32(OPTS["t_min"]))


def _proj(As, rgbs, px=(5, 7), var=4.0):
    """Gaussians centred on pixel ``px``'s centre (sigma = 0 there), front to back in list
    order, isotropic screen covariance ``var`` px^2."""
    n = len(As)
    mean2d = torch.tensor([[px[0] + 0.5, px[1] + 0.5]] * n, dtype=torch.float64)
    conic = torch.tensor([[1.0 / var, 0.0, 1.0 / var]] * n, dtype=torch.float64)
    cov = torch.tensor([[var, 0.0, var]] * n, dtype=torch.float64)
    return vo.OracleProjection(mean2d=mean2d, conic=conic, cov2d=cov,
                               rgb=torch.tensor(np.asarray(rgbs, np.float64)),
                               A=torch.tensor(np.asarray(As, np.float64)),
                               depth=torch.arange(1, n + 1, dtype=torch.float64), kept=np.ones(n, bool))


def _eps(a):
    """The float32 error bound on ln a at sigma = 0 (centre offset zero)."""
    return vo.ERR_COEF * U * (1.0 + abs(math.log(a)))


def _render(proj, opts, t_min=None, px=(5, 7)):
    order = np.arange(proj.A.shape[0])
    return oracle.render_pixels(proj, order, np.array([px]), opts, t_min=t_min)


def _opts(**kw):
    o = dict(OPTS)
    o.update(kw)
    return o


# ------------------------------------------------------------------------------- skip

def test_skip_flip_just_above_threshold_is_within_slack_and_slack_is_its_closed_form():
    """One Gaussian with a = alpha_min (1 + 4e-6), inside the float32 bound: blended here,
    skipped once alpha_min is nudged above a.  The pixel moves by c a <= slack, and slack =
    alpha_min (1 + eps) T_before with T_before = 1."""
    A = AMIN * (1 + 4e-6)
    assert math.log(A / AMIN) < _eps(A)
    c = [0.9, 0.4, 0.1]
    p = _proj([A], [c])
    r = _render(p, OPTS)
    assert r.last[0] == 0                    # blended
    slack = AMIN * (1 + _eps(A))
    assert abs(r.slack[0] - slack) <= 1e-15
    assert r.flag[0] and r.flag_grad[0]
    amin_up = float(np.nextafter(np.float32(A), np.float32(1)))
    r2 = _render(p, _opts(alpha_min=amin_up))
    assert r2.last[0] == -1                  # skipped
    move = (r.color - r2.color).abs().max().item()
    assert abs(move - 0.9 * A) <= 1e-15
    assert move <= r.slack[0]


def test_skip_flip_just_below_threshold_behind_a_front_gaussian():
    """The near-threshold Gaussian sits behind one of alpha 0.5: its slack carries the
    transmittance in front of it (0.5), and a flip moves the pixel by at most that."""
    A = AMIN * (1 - 4e-6)
    c_front, c_back = [0.2, 0.3, 0.4], [1.0, 0.0, 0.5]
    p = _proj([0.5, A], [c_front, c_back])
    r = _render(p, OPTS)
    assert r.last[0] == 0                    # the back one is skipped
    slack = AMIN * (1 + _eps(A)) * 0.5
    assert abs(r.slack[0] - slack) <= 1e-15
    amin_down = float(np.nextafter(np.float32(A), np.float32(0)))
    r2 = _render(p, _opts(alpha_min=amin_down))
    assert r2.last[0] == 1                   # now blended
    move = (r.color - r2.color).abs().max().item()
    assert abs(move - 1.0 * A * 0.5) <= 1e-15
    assert move <= r.slack[0]


def test_slack_sums_the_near_threshold_decisions_of_a_pixel():
    """Two near-threshold Gaussians in one pixel (the second behind the first): slack is
    the sum of both bounds, each with the transmittance in front of it; flipping both
    moves the pixel by no more."""
    A1, A2 = AMIN * (1 + 3e-6), AMIN * (1 + 5e-6)
    p = _proj([A1, A2], [[1.0, 1.0, 1.0], [1.0, 1.0, 1.0]])
    r = _render(p, OPTS)
    expect = AMIN * (1 + _eps(A1)) + AMIN * (1 + _eps(A2)) * (1 - A1)
    assert abs(r.slack[0] - expect) <= 1e-15
    amin_up = float(np.nextafter(np.float32(max(A1, A2)), np.float32(1)))
    r2 = _render(p, _opts(alpha_min=amin_up))
    assert r2.last[0] == -1
    move = (r.color - r2.color).abs().max().item()
    assert move <= r.slack[0]
    assert move > 0.5 * r.slack[0]           # the bound is not loose by more than 2x here


def test_no_slack_outside_the_error_bound():
    """a 1e-3 (relative) away from alpha_min, far outside the float32 bound: no slack, no
    flags."""
    for A in (AMIN * (1 + 1e-3), AMIN * (1 - 1e-3)):
        r = _render(_proj([A], [[1.0, 0.5, 0.2]]), OPTS)
        assert r.slack[0] == 0.0 and not r.flag[0] and not r.flag_grad[0]


# ------------------------------------------------------------------------------- stop

def _stop_stack(delta):
    """Alphas 0.95, 0.95, then one that leaves T = t_min e^delta, then 0.5 and 0.3."""
    T2 = 0.05 * 0.05
    a3 = 1.0 - TMIN * math.exp(delta) / T2
    As = [0.95, 0.95, a3, 0.5, 0.3]
    rgbs = [[0.1, 0.2, 0.3], [0.3, 0.2, 0.1], [0.5, 0.5, 0.5], [1.0, 0.8, 0.6], [0.2, 0.9, 0.4]]
    return As, rgbs


def _m_after(As, k):
    """Bound on the relative float32 error of T after the first k + 1 blends (closed form of
    the oracle's stop margin; every alpha here is unclamped and at sigma = 0)."""
    return sum(U + a / (1 - a) * (_eps(a) + 2 * U) for a in As[:k + 1])


def test_stop_flip_just_above_t_min_is_within_slack():
    """T after the third Gaussian is t_min (1 + 3e-5), inside its float32 bound: the oracle
    blends the fourth and stops there; with t_min nudged above that T it stops after the
    third.  The pixel moves by c4 alpha4 T3 <= slack = (m3 + max alpha after) T3 (1 + m3)."""
    As, rgbs = _stop_stack(3e-5)
    m3 = _m_after(As, 2)
    assert 3e-5 < m3
    p = _proj(As, rgbs)
    r = _render(p, OPTS)
    assert r.last[0] == 3 and r.n_eval[0] == 4
    T3 = 0.05 * 0.05 * (1 - As[2])
    slack = (m3 + 0.5) * T3 * (1 + m3)
    assert abs(r.slack[0] - slack) <= 1e-12 * slack
    assert r.flag[0] and r.flag_grad[0]
    r2 = _render(p, OPTS, t_min=float(np.nextafter(np.float32(T3), np.float32(1))))
    assert r2.last[0] == 2
    move = (r.color - r2.color).abs().max().item()
    assert abs(move - 1.0 * 0.5 * T3) <= 1e-15
    assert move <= r.slack[0]


def test_stop_flip_just_below_t_min_is_within_slack():
    """T after the third Gaussian is t_min (1 - 3e-5): the oracle stops there; with t_min
    nudged below that T it blends the fourth too (and then stops)."""
    As, rgbs = _stop_stack(-3e-5)
    m3 = _m_after(As, 2)
    p = _proj(As, rgbs)
    r = _render(p, OPTS)
    assert r.last[0] == 2 and r.n_eval[0] == 3
    T3 = 0.05 * 0.05 * (1 - As[2])
    slack = (m3 + 0.5) * T3 * (1 + m3)
    assert abs(r.slack[0] - slack) <= 1e-12 * slack
    r2 = _render(p, OPTS, t_min=float(np.nextafter(np.float32(T3), np.float32(0))))
    assert r2.last[0] == 3
    move = (r.color - r2.color).abs().max().item()
    assert move <= r.slack[0]


def test_no_stop_slack_far_from_t_min():
    As, rgbs = _stop_stack(1e-2)
    r = _render(_proj(As, rgbs), OPTS)
    assert r.slack[0] == 0.0 and not r.flag_grad[0]


# ------------------------------------------------------------ the error bound, emulated

def _fma32(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def test_error_bound_covers_a_float32_emulation_of_the_exponent():
    """The float32 exponent ln a, computed the way a tiled float32 renderer does (float32
    screen covariance and determinant from O1, conic = adj / det in float32, tile-local centre, quadratic
    form by fused multiply-adds, float32 log2 of A), differs from the float64 value by less
    than half the oracle's bound, at every pixel of the footprints of the 1k-Gaussian
    workload and of a reduced shell-clustered one (elongated ellipses included)."""
    f32 = np.float32
    l2e = f32(1.0 / math.log(2.0))
    worst = 0.0
    for widx, n, res in ((0, None, None), (2, 4000, 256)):
        w = synth.workload(widx, n_override=n, res_override=res)
        cam, lut, g = w.cameras[0], w.tfs[0], w.gaussians
        fp = oracle.footprint_f32(g, cam, lut, OPTS)
        proj = oracle.project_f64(g.means, g.log_scales, g.quats, g.scalars, None, cam, lut, OPTS)
        mu, con = proj.mean2d.detach().numpy(), proj.conic.detach().numpy()
        cov, A64 = proj.cov2d.detach().numpy(), proj.A.detach().numpy()
        S00, S01, S11 = fp.cov[:, 0], fp.cov[:, 1], fp.cov[:, 2]
        c0, c1, c2 = S11 / fp.det, -S01 / fp.det, S00 / fp.det
        for i in np.nonzero(fp.keep & proj.kept)[0]:
            x0, y0, x1, y1 = fp.rect[i]
            ys, xs = np.mgrid[16 * y0:min(16 * y1 + 16, cam.height), 16 * x0:min(16 * x1 + 16, cam.width)]
            xs, ys = xs.reshape(-1), ys.reshape(-1)
            dx64, dy64 = xs + 0.5 - mu[i, 0], ys + 0.5 - mu[i, 1]
            sig = 0.5 * (con[i, 0] * dx64 ** 2 + 2 * con[i, 1] * dx64 * dy64 + con[i, 2] * dy64 ** 2)
            ln64 = math.log(A64[i]) - sig
            near = np.abs(ln64 - math.log(AMIN)) < 0.5
            if not near.any():
                continue
            tx, ty = xs // 16, ys // 16
            mxr, myr = f32(fp.mx[i] - 16.0 * x0), f32(fp.my[i] - 16.0 * y0)
            smx = mxr - (16 * (tx - x0)).astype(f32)
            smy = myr - (16 * (ty - y0)).astype(f32)
            q0, q1, q2 = c0[i] * (f32(0.5) * l2e), c1[i] * l2e, c2[i] * (f32(0.5) * l2e)
            l2A = f32(math.log2(float(fp.A[i])))
            dx = ((xs % 16).astype(f32) + f32(0.5)) - smx
            dy = ((ys % 16).astype(f32) + f32(0.5)) - smy
            base = _fma32(-q0 * dx, dx, np.full_like(dx, l2A))
            e = _fma32(-dy, _fma32(np.full_like(dy, q2), dy, q1 * dx), base)
            ln32 = e.astype(np.float64) * math.log(2.0)
            y0v = con[i, 0] * dx64 + con[i, 1] * dy64
            y1v = con[i, 1] * dx64 + con[i, 2] * dy64
            eps = vo.ERR_COEF * U * (1 + abs(math.log(A64[i])) +
                                    (np.abs(y0v) * math.sqrt(cov[i, 0]) + np.abs(y1v) * math.sqrt(cov[i, 2])) ** 2)
            worst = max(worst, float((np.abs(ln32 - ln64) / eps)[near].max()))
    assert 0.0 < worst <= 0.5, worst


# ------------------------------------------------------------------- key-list tiles

def _two_frames():
    rng = np.random.default_rng(31)
    g = synth.clustered_gaussians(rng, 1500, scale_lo=0.01, scale_hi=0.08)
    cams = [synth.look_at_camera(synth.random_direction(rng), 3.0, 96, 56),
            synth.look_at_camera(synth.random_direction(rng), 3.0, 72, 104)]
    luts = [synth.random_tf(rng), synth.random_tf(rng)]
    return g, cams, luts


def test_key_list_tiles_equal_a_cover_enumeration():
    """Each tile's list holds exactly the Gaussians whose tile rectangle covers the tile,
    ordered by (depth bits, index), with tile ids numbered per frame from that frame's
    base, row-major over its (non-square) tile grid."""
    g, cams, luts = _two_frames()
    fps = [oracle.footprint_f32(g, c, l, OPTS) for c, l in zip(cams, luts)]
    tiles, depths, pairs, ranges, bases = oracle.key_list(fps, cams)
    n = g.n
    grids = [((c.width + 15) // 16, (c.height + 15) // 16) for c in cams]
    assert grids == [(6, 4), (5, 7)]
    assert list(bases) == [0, 24] and ranges.shape[0] == 24 + 35
    total = 0
    for f, (fp, (gx, gy)) in enumerate(zip(fps, grids)):
        for ty in range(gy):
            for tx in range(gx):
                cover = [i for i in range(n) if fp.count[i] > 0 and fp.rect[i, 0] <= tx <= fp.rect[i, 2]
                         and fp.rect[i, 1] <= ty <= fp.rect[i, 3]]
                cover.sort(key=lambda i: (int(fp.depth_bits[i]), i))
                s, e = ranges[bases[f] + ty * gx + tx]
                assert list(pairs[s:e]) == [f * n + i for i in cover], (f, tx, ty)
                total += len(cover)
    assert total == tiles.shape[0] and total > 1000


def test_key_list_tile_of_every_reached_pixel_holds_the_gaussian():
    """Every pixel where a Gaussian's float64 alpha reaches alpha_min (with a 1e-5 relative
    margin) lies in a tile, (x // 16, y // 16) of its own frame, whose list holds it."""
    g, cams, luts = _two_frames()
    fps = [oracle.footprint_f32(g, c, l, OPTS) for c, l in zip(cams, luts)]
    tiles, depths, pairs, ranges, bases = oracle.key_list(fps, cams)
    n = g.n
    checked = 0
    for f, (cam, lut) in enumerate(zip(cams, luts)):
        gx = (cam.width + 15) // 16
        members = {}
        for t in range((cam.width + 15) // 16 * ((cam.height + 15) // 16)):
            s, e = ranges[bases[f] + t]
            members[t] = set(int(p) for p in pairs[s:e])
        proj = oracle.project_f64(g.means, g.log_scales, g.quats, g.scalars, None, cam, lut, OPTS)
        mu, con, A = proj.mean2d.detach().numpy(), proj.conic.detach().numpy(), proj.A.detach().numpy()
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        xs, ys = xs.reshape(-1), ys.reshape(-1)
        for i in np.nonzero(proj.kept)[0]:
            dx, dy = xs + 0.5 - mu[i, 0], ys + 0.5 - mu[i, 1]
            a = A[i] * np.exp(-0.5 * (con[i, 0] * dx * dx + 2 * con[i, 1] * dx * dy + con[i, 2] * dy * dy))
            hit = a >= AMIN * (1 + 1e-5)
            for t in np.unique((ys[hit] // 16) * gx + xs[hit] // 16):
                assert f * n + i in members[int(t)], (f, i, t)
                checked += 1
    assert checked > 1000


# ------------------------------------------------------------------------------- L1

def test_l1_hand_computed_case():
    img = np.array([[1.0, -2.0, 0.0], [0.5, 0.0, -0.25]])
    loss, grad = oracle.l1_loss(img, np.zeros_like(img))
    assert loss == 3.75 / 6
    assert np.array_equal(grad, np.array([[1, -1, 0], [1, 0, -1]]) / 6.0)
    loss2, grad2 = oracle.l1_loss(img, np.zeros_like(img), scale=0.5)
    assert loss2 == 0.5 * 3.75 and np.array_equal(grad2, 0.5 * np.sign(img))


def test_l1_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (3, 5, 4))
    tgt = img + rng.choice([-1.0, 1.0], img.shape) * rng.uniform(0.01, 0.2, img.shape)
    _, grad = oracle.l1_loss(img, tgt)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (2, 4, 1), (0, 3, 2)]:
        up, dn = img.copy(), img.copy()
        up[idx] += h
        dn[idx] -= h
        num = (oracle.l1_loss(up, tgt)[0] - oracle.l1_loss(dn, tgt)[0]) / (2 * h)
        assert abs(num - grad[idx]) <= 1e-8


def test_tile_occupancy_equals_the_key_list_tile_lengths():
    g, cams, luts = _two_frames()
    fps = [oracle.footprint_f32(g, c, l, OPTS) for c, l in zip(cams, luts)]
    tiles, depths, pairs, ranges, bases = oracle.key_list(fps, cams)
    for f, (fp, cam) in enumerate(zip(fps, cams)):
        occ = oracle.tile_occupancy(fp, cam)
        nt = occ.size
        lens = ranges[bases[f]:bases[f] + nt, 1] - ranges[bases[f]:bases[f] + nt, 0]
        assert occ.shape == ((cam.height + 15) // 16, (cam.width + 15) // 16)
        assert np.array_equal(occ.reshape(-1), lens)
