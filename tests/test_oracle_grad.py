"""Pins of the gradient reference (PyTorch FP64 autograd of the plain forward):
central finite differences of the independent C forward, and closed forms."""
import math

import numpy as np
import pytest

import oracle
import oracle.grad as og
import scenegen
from tests.helpers import axis_view, scene_from

GROUPS = og.PARAMS


def _loss_c(arrs, v, w, crop):
    sc = scenegen.Scene(**arrs)
    im = oracle.render(sc, v, crop=crop)
    return float((im.image * w).sum()), im.chash.copy()


def _fd_check(scene, v, crop, params, rel_h=1e-6, seed=0):
    """Returns (fd, ad) arrays over the listed (group, index) parameters whose
    +-h perturbations keep every pixel's contributor set."""
    x0, y0, w_, h_ = crop
    w = np.random.default_rng(seed).normal(size=(3, h_, w_))
    g_ad, _ = og.grad(scene, v, w, crop=crop)
    base = {k: np.asarray(getattr(scene, k), np.float32).astype(np.float64) for k in GROUPS}
    _, h0 = _loss_c(base, v, w, crop)
    fd, ad = [], []
    for grp, idx in params:
        th = base[grp][idx]
        h = rel_h * max(1.0, abs(th))
        arr_p = {k: a.copy() for k, a in base.items()}
        arr_m = {k: a.copy() for k, a in base.items()}
        arr_p[grp][idx] = th + h
        arr_m[grp][idx] = th - h
        lp, hp = _loss_c(arr_p, v, w, crop)
        lm, hm = _loss_c(arr_m, v, w, crop)
        if not (np.array_equal(hp, h0) and np.array_equal(hm, h0)):
            continue
        fd.append((lp - lm) / (2 * h))
        ad.append(g_ad[grp][idx])
    return np.array(fd), np.array(ad)


def _all_params(scene):
    out = []
    for grp in GROUPS:
        a = np.asarray(getattr(scene, grp))
        for idx in np.ndindex(a.shape):
            out.append((grp, idx))
    return out


def test_x18_fd_all_parameters_small_scene():
    """Every parameter of a 16-Gaussian 16x16 scene: FD of the C forward equals
    the autograd gradient."""
    sc = scenegen.make_scene(16, 40, h=0.4, sigma_off=0.1)
    v = scenegen.make_views(1, 40, r=2.5, W=16, H=16, bg=(0.2, 0.4, 0.6))[0]
    fd, ad = _fd_check(sc, v, (0, 0, 16, 16), _all_params(sc))
    assert len(fd) > 0.9 * 16 * 84
    assert np.abs(ad).max() > 1e-3
    err = np.abs(fd - ad)
    assert np.all(err <= 1e-6 * np.maximum(np.abs(ad), 1e-3 * np.abs(ad).max())), err.max()


def test_x18_fd_sampled_parameters_training_subset():
    """Sampled parameters (all groups) of the 2,000-Gaussian 64x64 subset of
    the training workload (same camera, first 2,000 Gaussians)."""
    sc_full, views, _ = scenegen.config2(n=2000)
    v = views[0]
    v = scenegen.make_view(v.c, 64, 64, v.t, d=v.d, lambda_t=v.lambda_t, lambda_d=v.lambda_d)
    sub = sc_full
    rng = np.random.default_rng(1)
    # sample among Gaussians that contribute somewhere
    g_ad, _ = og.grad(sub, v, np.ones((3, 64, 64)))
    live = np.nonzero(np.abs(g_ad["alpha"]) > 0)[0]
    params = []
    for grp in GROUPS:
        a = np.asarray(getattr(sub, grp))
        rows = a.shape[0] if a.ndim == 2 else 1
        for _ in range(16 if grp != "sh" else 24):
            gidx = int(rng.choice(live))
            idx = (int(rng.integers(rows)), gidx) if a.ndim == 2 else (gidx,)
            params.append((grp, idx))
    fd, ad = _fd_check(sub, v, (0, 0, 64, 64), params)
    assert len(fd) > 0.8 * len(params)
    err = np.abs(fd - ad)
    scale = np.maximum(np.abs(ad), 1e-3 * np.abs(ad).max())
    assert np.all(err <= 1e-5 * scale), (err / scale).max()


def test_x20_closed_form_gradients_single_gaussian():
    """One on-axis Gaussian (f_temp = f_dir = 1): dC_ch/d beta_0,ch =
    alpha(p) Y_00, dC_ch/d alpha = (rgb_ch - bg_ch) exp(-q/2) where unclamped."""
    v = axis_view(W=32, H=32, z0=3.0, bg=(0.25, 0.5, 0.75))
    Ld = np.eye(7)[None].copy()
    Ld[0, :3, :3] = 0.12 * np.eye(3)
    sh = np.zeros((1, 48))
    sh[0, :3] = [0.4, -0.2, 0.9]
    sc = scene_from([[0, 0, 0]], [0.5], [(0, 0, 1)], Ld, [0.6], sh)
    w = np.random.default_rng(2).normal(size=(3, 32, 32))
    g, _ = og.grad(sc, v, w)
    f = float(v.fx)
    var = f * f * float(np.float32(0.12)) ** 2 / 9.0 + oracle.DILATION
    ys, xs = np.mgrid[0:32, 0:32] + 0.5
    e = np.exp(-0.5 * ((xs - v.cx) ** 2 + (ys - v.cy) ** 2) / var)
    a = float(np.float32(0.6)) * e
    live = a >= oracle.ALPHA_MIN
    Y00 = 0.5 / math.sqrt(math.pi)
    rgb = 0.5 + np.array([0.4, -0.2, 0.9], np.float32).astype(np.float64) * Y00
    bg = np.array([0.25, 0.5, 0.75], np.float32).astype(np.float64)
    for ch in range(3):
        expect = (w[ch] * np.where(live, a, 0.0)).sum() * Y00
        assert g["sh"][ch, 0] == pytest.approx(expect, rel=1e-12)
    expect_a = sum((w[ch] * np.where(live, e, 0.0)).sum() * (rgb[ch] - bg[ch]) for ch in range(3))
    assert g["alpha"][0] == pytest.approx(expect_a, rel=1e-12)


def _scene64(sc):
    """The scene with FP64 planes (so perturbations are not rounded)."""
    return scenegen.Scene(*(np.asarray(getattr(sc, k), np.float64).copy()
                            for k in ("mu_p", "mu_t", "mu_d", "L", "alpha", "sh")))


def _splat_values(s, v):
    o = oracle.slice_(s, v)
    pr = oracle.project(o, s.sh, v)
    return np.concatenate([pr.mean2d, pr.conic, o.alpha_c[None], pr.rgb], 0)


def test_splat_jacobian_matches_central_differences_of_the_c_path():
    """og.splat_jacobian (autograd of the PyTorch slice and projection)
    against FP64 central differences of the independent C slice and
    projection, for every parameter of a few Gaussians of a correlated scene."""
    sc = scenegen.make_scene(40, 71, sigma_off=0.15)
    v = scenegen.make_views(1, 71, r=3.0, W=32, H=32)[0]
    J = og.splat_jacobian(sc, v)
    base = _scene64(sc)
    vis = oracle.project(oracle.slice_(sc, v), sc.sh, v).visible
    checked = 0
    for g in np.nonzero(vis)[0][:4]:
        for k in og.PARAMS:
            arr = getattr(base, k)
            planes = 1 if arr.ndim == 1 else arr.shape[0]
            for p in range(planes):
                idx = (g,) if arr.ndim == 1 else (p, g)
                h = 1e-6 * max(1.0, abs(arr[idx]))
                sp, sm = _scene64(sc), _scene64(sc)
                getattr(sp, k)[idx] += h
                getattr(sm, k)[idx] -= h
                fd = (_splat_values(sp, v)[:, g] - _splat_values(sm, v)[:, g]) / (2 * h)
                np.testing.assert_allclose(J[k][:, p, g], fd, rtol=1e-5, atol=1e-6 * max(1.0, np.abs(fd).max()))
                checked += 1
    assert checked == 4 * 84


def test_splat_gradients_match_central_differences_and_the_chain_rule():
    """og.grad_splats against FP64 central differences of the C compositing
    in each splat value, and chained through og.splat_jacobian it gives
    og.grad's parameter gradients."""
    sc, views = scenegen.config0()
    v = views[0]
    dL = np.random.default_rng(5).normal(size=(3, v.H, v.W))
    d = og.grad_splats(sc, v, dL)
    sl = oracle.slice_(sc, v)
    pr = oracle.project(sl, sc.sh, v)

    def loss(s2, p2):
        return float((oracle.composite(s2, p2, v, banded=False).image * dL).sum())

    rng = np.random.default_rng(6)
    checked = 0
    for g in rng.choice(np.nonzero(pr.visible)[0], 12, replace=False):
        for j in range(len(og.SPLAT)):
            scale = [1.0, 1.0, *([float(np.abs(pr.conic[:, g]).max())] * 3), float(sl.alpha_c[g]), 1.0, 1.0, 1.0][j]
            h = 1e-5 * scale
            vals = []
            for sgn in (1, -1, 0.5, -0.5):
                s2 = oracle.Sliced(sl.mu_c, sl.cov_c, sl.alpha_c.copy(), None, None, None)
                p2 = oracle.Projected(pr.mean2d.copy(), pr.conic.copy(), pr.depth, pr.rgb.copy(), pr.rect,
                                      pr.visible, pr.box)
                tgt = [p2.mean2d[0], p2.mean2d[1], p2.conic[0], p2.conic[1], p2.conic[2], s2.alpha_c,
                       p2.rgb[0], p2.rgb[1], p2.rgb[2]][j]
                tgt[g] += sgn * h
                vals.append(loss(s2, p2))
            fd, fd2 = (vals[0] - vals[1]) / (2 * h), (vals[2] - vals[3]) / h
            if abs(fd - fd2) > 1e-5 * max(1e-3, abs(fd)):
                continue   # a discrete decision moved within the step
            assert d[j, g] == pytest.approx(fd, rel=1e-4, abs=1e-8)
            checked += 1
    assert checked > 80
    J = og.splat_jacobian(sc, v)
    g_full, _ = og.grad(sc, v, dL)
    for k in og.PARAMS:
        chain = np.einsum("jpn,jn->pn", J[k], d).reshape(g_full[k].shape)
        np.testing.assert_allclose(chain, g_full[k], rtol=0, atol=1e-12 * np.abs(g_full[k]).max())
