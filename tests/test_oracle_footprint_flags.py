"""Pins of the oracle's footprint box, tile lists and decision flags (Sec. 4.4
compositing and tiling contract), against brute force and closed forms.

* The opacity box of each splat is the exact bounding box of
  {alpha_c exp(-q/2) >= 1/255}: its edges equal the extreme points of that
  ellipse found by an independent parametrization (eigenvectors of the conic,
  numerical maximization), and no sample of a dense grid outside the box
  reaches the threshold.
* tile_lists() equals a brute-force scan over every (tile, Gaussian) pair, in
  (depth, index) order, and holds every Gaussian that reaches 1/255 at a pixel
  centre of the tile.
* Each flag bit fires on a constructed case inside its band and not outside
  it, and the per-pixel bound covers the change the flipped decision makes
  (checked by flipping it in FP64).
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
import scenegen
from tests.helpers import axis_view, scene_from

Y00 = 0.5 / math.sqrt(math.pi)


def _scene_view():
    sc = scenegen.make_scene(1500, 31, h=1.0, sigma_off=0.1)
    v = scenegen.make_views(1, 31, r=3.0, W=96, H=80)[0]
    return sc, v


def _ellipse_extreme(a, b, c, k, axis):
    """max over the ellipse a x^2 + 2 b x y + c y^2 = k of coordinate `axis`,
    by parametrizing the ellipse through the conic's eigenvectors and
    maximizing numerically (no closed form of the extent involved)."""
    lam, V = np.linalg.eigh(np.array([[a, b], [b, c]]))
    r = np.sqrt(k / lam)

    def f(t):
        p = V @ (r * np.array([math.cos(t), math.sin(t)]))
        return -p[axis]

    ts = np.linspace(0.0, 2 * math.pi, 4097)
    t0 = ts[int(np.argmin([f(t) for t in ts]))]
    res = minimize_scalar(f, bounds=(t0 - 2e-3, t0 + 2e-3), method="bounded",
                          options={"xatol": 1e-12})
    return -res.fun


def test_o10_box_edges_touch_the_opacity_ellipse():
    sc, v = _scene_view()
    sl = oracle.slice_(sc, v)
    pr = oracle.project(sl, sc.sh, v)
    vis = np.nonzero(pr.visible)[0]
    assert len(vis) > 300
    for g in vis[:: max(1, len(vis) // 150)]:
        a, b, c = pr.conic[:, g]
        k = 2.0 * math.log(sl.alpha_c[g] / oracle.ALPHA_MIN)
        u, vv = pr.mean2d[:, g]
        ex = _ellipse_extreme(a, b, c, k, 0)
        ey = _ellipse_extreme(a, b, c, k, 1)
        assert abs((pr.box[2, g] - u) - ex) < 1e-9 * max(1.0, ex)
        assert abs((u - pr.box[0, g]) - ex) < 1e-9 * max(1.0, ex)
        assert abs((pr.box[3, g] - vv) - ey) < 1e-9 * max(1.0, ey)
        assert abs((vv - pr.box[1, g]) - ey) < 1e-9 * max(1.0, ey)


def test_o10_no_sample_outside_the_box_reaches_the_threshold():
    """Dense quarter-pixel grid around each box: every sample with
    alpha_c e^{-q/2} >= 1/255 lies in the box (that the box is no larger than
    the ellipse is pinned by the edge test above)."""
    sc, v = _scene_view()
    sl = oracle.slice_(sc, v)
    pr = oracle.project(sl, sc.sh, v)
    vis = np.nonzero(pr.visible)[0]
    for g in vis[:: max(1, len(vis) // 120)]:
        x0, y0, x1, y1 = pr.box[:, g]
        xs = np.arange(math.floor(x0) - 3, math.ceil(x1) + 3, 0.25)
        ys = np.arange(math.floor(y0) - 3, math.ceil(y1) + 3, 0.25)
        X, Y = np.meshgrid(xs, ys)
        dx, dy = X - pr.mean2d[0, g], Y - pr.mean2d[1, g]
        a, b, c = pr.conic[:, g]
        al = sl.alpha_c[g] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
        hit = al >= oracle.ALPHA_MIN
        assert hit.any()
        assert np.all((X[hit] >= x0 - 1e-9) & (X[hit] <= x1 + 1e-9))
        assert np.all((Y[hit] >= y0 - 1e-9) & (Y[hit] <= y1 + 1e-9))


def test_rect_is_the_tile_range_of_the_box():
    sc, v = _scene_view()
    sl = oracle.slice_(sc, v)
    pr = oracle.project(sl, sc.sh, v)
    tx, ty = (v.W + 15) // 16, (v.H + 15) // 16
    for g in range(sc.n):
        if not pr.visible[g]:
            continue
        x0, y0, x1, y1 = pr.box[:, g]
        # tiles whose extent [16 t, 16 t + 16) meets [x0, x1], clipped to the grid
        cols = [t for t in range(tx) if 16 * t <= x1 and x0 < 16 * (t + 1)]
        rows = [t for t in range(ty) if 16 * t <= y1 and y0 < 16 * (t + 1)]
        assert cols and rows
        assert list(pr.rect[:, g]) == [cols[0], rows[0], cols[-1] + 1, rows[-1] + 1]


def test_culled_splats_have_an_empty_or_offscreen_box():
    sc, v = _scene_view()
    sl = oracle.slice_(sc, v)
    pr = oracle.project(sl, sc.sh, v)
    for g in np.nonzero(~pr.visible)[0]:
        x0, y0, x1, y1 = pr.box[:, g]
        offscreen = x1 < 0 or y1 < 0 or x0 >= 16 * ((v.W + 15) // 16) or y0 >= 16 * ((v.H + 15) // 16)
        assert sl.alpha_c[g] < oracle.ALPHA_MIN or offscreen or (x0, y0, x1, y1) == (0, 0, 0, 0)


def test_tile_lists_equal_brute_force_and_hold_every_reaching_gaussian():
    sc, v = _scene_view()
    sl = oracle.slice_(sc, v)
    pr = oracle.project(sl, sc.sh, v)
    lists = oracle.tile_lists(pr, v)
    tx, ty = (v.W + 15) // 16, (v.H + 15) // 16
    vis = [g for g in range(sc.n) if pr.visible[g]]
    for t_y in range(ty):
        for t_x in range(tx):
            inside = [g for g in vis
                      if 16 * t_x <= pr.box[2, g] and pr.box[0, g] < 16 * (t_x + 1)
                      and 16 * t_y <= pr.box[3, g] and pr.box[1, g] < 16 * (t_y + 1)]
            ref = sorted(inside, key=lambda g: (pr.depth[g], g))
            got = lists.get(t_y * tx + t_x, [])
            assert got == ref, (t_x, t_y)
            # every Gaussian reaching 1/255 at a pixel centre of the tile is listed
            px = np.arange(16 * t_x, min(16 * t_x + 16, v.W)) + 0.5
            py = np.arange(16 * t_y, min(16 * t_y + 16, v.H)) + 0.5
            X, Y = np.meshgrid(px, py)
            listed = set(got)
            for g in vis:
                dx, dy = X - pr.mean2d[0, g], Y - pr.mean2d[1, g]
                a, b, c = pr.conic[:, g]
                al = sl.alpha_c[g] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
                if (al >= oracle.ALPHA_MIN).any():
                    assert g in listed, (t_x, t_y, g)


# ---- decision flags and their bounds ---------------------------------------

def _iso(s_list, z_list, alpha_list, dc_list):
    n = len(s_list)
    Ld = np.zeros((n, 7, 7))
    sh = np.zeros((n, 48))
    for g in range(n):
        Ld[g] = np.eye(7)
        Ld[g][:3, :3] = s_list[g] * np.eye(3)
        sh[g, 0:3] = dc_list[g]
    return scene_from(np.array([[0.0, 0.0, z] for z in z_list]), [0.5] * n, [(0, 0, 1)] * n, Ld,
                      alpha_list, sh)


def _alpha_at(view, sc, g, px, py):
    sl = oracle.slice_(sc, view)
    pr = oracle.project(sl, sc.sh, view)
    dx, dy = pr.mean2d[0, g] - (px + 0.5), pr.mean2d[1, g] - (py + 0.5)
    a, b, c = pr.conic[:, g]
    return sl.alpha_c[g] * math.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)), sl.alpha_c[g]


def _opacity_for(view, s, target, px, py):
    """Base opacity that gives alpha = target at pixel (px, py) for the
    on-axis isotropic Gaussian of scale s (the modulations are 1 here)."""
    a_pix, a_c = _alpha_at(view, _iso([s], [0.0], [0.5], [(1, 1, 1)]), 0, px, py)
    return 0.5 * target / a_pix


def test_alpha_flag_fires_inside_its_band_and_bounds_the_flip():
    v = axis_view(W=32, H=32, z0=3.0, bg=(0.2, 0.4, 0.6))
    px, py = 25, 16
    dc = (1.5, -0.5, 0.2)
    rgb = np.maximum(0.0, 0.5 + np.float32(dc).astype(np.float64) * Y00)
    bg = np.array([0.2, 0.4, 0.6], np.float32).astype(np.float64)
    for rel in (1e-9, -1e-9):
        base = _opacity_for(v, 0.05, oracle.ALPHA_MIN * (1 + rel), px, py)
        sc = _iso([0.05], [0.0], [np.float32(base)], [dc])
        a_pix, _ = _alpha_at(v, sc, 0, px, py)
        assert abs(math.log(a_pix / oracle.ALPHA_MIN)) < 1e-6
        im = oracle.render(sc, v)
        assert im.flags[py, px] & oracle.FLAG_ALPHA
        assert not im.flags[py, px] & (oracle.FLAG_T | oracle.FLAG_DEPTH)
        # first-order effect: a (rgb - bg) with a at the threshold
        d = np.abs(rgb - bg).max() * max(a_pix, oracle.ALPHA_MIN)
        assert im.fbound[py, px] == pytest.approx(1.01 * d, rel=2e-4)
        # flip the decision in FP64 by nudging the opacity across the threshold
        sc2 = _iso([0.05], [0.0], [np.float32(base * (1 - 1e-6 if rel > 0 else 1 + 1e-6))], [dc])
        flipped = oracle.render(sc2, v, banded=False)
        assert np.abs(flipped.image[:, py, px] - im.image[:, py, px]).max() <= im.fbound[py, px]
    # well outside the band: no opacity flag at that pixel
    for rel in (3e-3, -3e-3):
        sc = _iso([0.05], [0.0], [np.float32(_opacity_for(v, 0.05, oracle.ALPHA_MIN * (1 + rel), px, py))], [dc])
        im = oracle.render(sc, v)
        assert not im.flags[py, px]
        assert im.fbound[py, px] == 0.0


def test_t_flag_fires_inside_its_band_and_bounds_the_flip():
    """k coincident wide Gaussians with per-pixel alpha a at the centre pixel
    and (1 - a)^k = T_MIN (1 + rel): the k-th step lands at T_MIN."""
    v = axis_view(W=16, H=16, z0=3.0, bg=(1.0, 1.0, 1.0))
    k, px, py = 10, 8, 8
    dc = (-2.0, -2.0, -2.0)   # rgb = 0.5 - 2 Y00 ~ -0.06 -> clamped to 0
    for rel, inside in ((1e-9, True), (-1e-9, True), (2e-2, False), (-2e-2, False)):
        target = 1.0 - (oracle.T_MIN * (1 + rel)) ** (1.0 / k)
        base = _opacity_for(v, 50.0, target, px, py)
        sc = _iso([50.0] * k, [0.0] * k, [base] * k, [dc] * k)
        # the FP32 base opacity moves alpha slightly: recompute the landing point
        a_pix, _ = _alpha_at(v, sc, 0, px, py)
        land = (1 - a_pix) ** k
        im = oracle.render(sc, v)
        fired = bool(im.flags[py, px] & oracle.FLAG_T)
        if inside:
            assert abs(land / oracle.T_MIN - 1) < 1e-5
            assert fired
            # the flip changes the pixel by a T_{k-1} |rgb - bg| = a T_{k-1}
            # (rgb = 0, bg = 1): the step either is or is not taken
            T_before = (1 - a_pix) ** (k - 1)
            assert im.fbound[py, px] == pytest.approx(1.01 * a_pix * T_before, rel=1e-6)
        else:
            assert not fired


def test_depth_flag_fires_on_near_ties_and_bounds_the_swap():
    v = axis_view(W=24, H=24, z0=3.0)
    dcs = [(1.0, 0.0, -1.0), (-1.0, 1.0, 0.0)]
    for dz, inside in ((1e-12, True), (2e-4, False)):
        sc = _iso([0.2, 0.2], [0.0, dz], [0.6, 0.6], dcs)
        im = oracle.render(sc, v)
        if inside:
            assert im.flags[12, 12] & oracle.FLAG_DEPTH
            # swapping the two changes the pixel by T a1 a2 |rgb1 - rgb2| (T = 1)
            a, _ = _alpha_at(v, sc, 0, 12, 12)
            rgb = [np.maximum(0, 0.5 + np.float32(d).astype(np.float64) * Y00) for d in dcs]
            assert im.fbound[12, 12] == pytest.approx(1.01 * a * a * np.abs(rgb[0] - rgb[1]).max(), rel=1e-6)
            # and the swap, made in FP64 by moving the second one in front, stays within it
            sc2 = _iso([0.2, 0.2], [0.0, -dz], [0.6, 0.6], dcs)
            sw = oracle.render(sc2, v, banded=False)
            assert np.all(np.abs(sw.image - im.image).max(0) <= im.fbound + 1e-15)
        else:
            assert not (im.flags & oracle.FLAG_DEPTH).any()


# ---- value band: opacities moving within their bands, decisions kept -----

# only the constant term of the band: ln alpha's band is 1e-3 at every
# (Gaussian, pixel), whatever the geometry
CONST_BAND = dict(k_mu=0.0, k_uv=0.0, k_s=0.0, k_eval=0.0, k_ac=1e-3 * 2.0 ** 24, k_T=0.0, k_z=0.0)


def test_value_band_of_one_splat_is_its_opacity_derivative_times_the_band():
    """One splat over the background: C = a rgb + (1 - a) bg, so
    d C / d ln a = a (rgb - bg) and the value bound is 1.01 x 1e-3 x a
    max|rgb - bg|.  Scaling the splat's opacity by e^(+-1e-3) (every decision
    kept) moves the pixel by that much to first order."""
    v = axis_view(W=32, H=32, z0=3.0, bg=(0.2, 0.4, 0.6))
    dc = (1.5, -0.5, 0.2)
    rgb = np.maximum(0.0, 0.5 + np.float32(dc).astype(np.float64) * Y00)
    bg = np.array([0.2, 0.4, 0.6], np.float32).astype(np.float64)
    sc = _iso([0.3], [0.0], [0.5], [dc])
    im = oracle.render(sc, v, flags=CONST_BAND)
    for px, py in ((16, 16), (19, 14), (21, 17)):
        a_pix, _ = _alpha_at(v, sc, 0, px, py)
        assert oracle.ALPHA_MIN * 1.01 < a_pix < oracle.ALPHA_MAX
        assert im.vbound[py, px] == pytest.approx(1.01 * 1e-3 * a_pix * np.abs(rgb - bg).max(), rel=1e-9)
        for sgn in (1.0, -1.0):
            moved = oracle.render(_iso([0.3], [0.0], [0.5 * math.exp(sgn * 1e-3)], [dc]), v, banded=False)
            d = np.abs(moved.image[:, py, px] - im.image[:, py, px]).max()
            assert im.vbound[py, px] / 1.01 * (1 - 2e-3) <= d <= im.vbound[py, px]
    # no contributor, no value bound
    assert im.vbound[0, 0] == 0.0 and im.ncontrib[0, 0] == 0


def test_value_band_of_two_splats_sums_both_derivatives():
    """Two splats in depth order at one pixel: C = a1 c1 + (1 - a1)(a2 c2 +
    (1 - a2) bg), so d C / d ln a1 = a1 (c1 - a2 c2 - (1 - a2) bg) and
    d C / d ln a2 = (1 - a1) a2 (c2 - bg); the bound is 1.01 x 1e-3 x the sum
    of their largest channels."""
    v = axis_view(W=24, H=24, z0=3.0, bg=(1.0, 0.5, 0.0))
    dcs = [(1.0, 0.0, -1.0), (-1.0, 1.0, 0.5)]
    sc = _iso([0.2, 0.25], [0.0, 0.1], [0.6, 0.7], dcs)
    im = oracle.render(sc, v, flags=CONST_BAND)
    px, py = 13, 11
    a1, _ = _alpha_at(v, sc, 0, px, py)
    a2, _ = _alpha_at(v, sc, 1, px, py)
    c1, c2 = (np.maximum(0.0, 0.5 + np.float32(d).astype(np.float64) * Y00) for d in dcs)
    bg = np.array([1.0, 0.5, 0.0])
    d1 = np.abs(a1 * (c1 - a2 * c2 - (1 - a2) * bg)).max()
    d2 = np.abs((1 - a1) * a2 * (c2 - bg)).max()
    assert im.vbound[py, px] == pytest.approx(1.01 * 1e-3 * (d1 + d2), rel=1e-9)


def test_value_band_bounds_any_opacity_moves_within_the_band():
    """A random scene with the constant band: scaling every Gaussian's
    opacity by e^(s_i 1e-3), s_i = +-1 at random, moves each pixel by at most
    fbound + vbound (decisions taken the other way are in fbound)."""
    sc = scenegen.make_scene(400, 41, h=1.0, sigma_off=0.1)
    v = scenegen.make_views(1, 41, r=3.0, W=48, H=40, bg=(0.3, 0.6, 0.9))[0]
    im = oracle.render(sc, v, flags=CONST_BAND)
    assert (im.vbound > 0).mean() > 0.5
    rng = np.random.default_rng(7)
    for _ in range(3):
        s = rng.choice([-1.0, 1.0], size=sc.n)
        sc2 = scene_from(sc.mu_p.T, sc.mu_t, sc.mu_d.T, scenegen.unpack_L(sc.L.T.astype(np.float64)),
                         sc.alpha.astype(np.float64) * np.exp(s * 1e-3), sc.sh.T)
        moved = oracle.render(sc2, v, banded=False)
        d = np.abs(moved.image - im.image).max(0)
        assert np.all(d <= im.fbound + im.vbound + 1e-12)
        # and the bound is not loose by orders of magnitude
        assert d.max() >= 0.05 * (im.fbound + im.vbound).max()


def test_unbanded_render_has_no_flags_and_the_same_image():
    sc, views = scenegen.config0()
    a = oracle.render(sc, views[0])
    b = oracle.render(sc, views[0], banded=False)
    np.testing.assert_array_equal(a.image, b.image)
    assert not b.flags.any() and not b.fbound.any() and not b.vbound.any()


def test_fp32_model_scales_on_axis():
    """On the optical axis with R = I: e_mu = f/z max|mu|, |J R| = diag(f/z),
    so Sabs is (f/z)^2 |Sigma_c| restricted to x, y."""
    v = axis_view(W=64, H=64, z0=3.0)
    mu = np.array([[0.0], [0.0], [0.5]])
    cov = np.array([[0.01], [0.002], [-0.003], [0.02], [0.001], [0.03]])
    sl = oracle.Sliced(mu, cov, np.array([0.8]), None, None, None)
    e = oracle.fp32_model(sl, v)[:, 0]
    fz = float(v.fx) / 3.5
    np.testing.assert_allclose(e, [fz * 0.5, fz * fz * 0.01, fz * fz * 0.002, fz * fz * 0.02, 0.5 + 3.5],
                               rtol=1e-12)
