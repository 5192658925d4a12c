"""Pins of the slice variants around Algorithm 1: conditioning each Gaussian
on its own direction unit(mu_p - c), and the gradients with respect to the
modulation strengths lambda_t, lambda_d (trainable in the paper's schedule)."""
import numpy as np

import oracle
import oracle.grad as og
import scenegen
from tests.test_oracle_grad import _all_params, _fd_check, _loss_c


def _scene_view(per_gaussian=True, n=30, seed=50):
    sc = scenegen.make_scene(n, seed, h=0.5, sigma_off=0.1)
    v = scenegen.make_views(1, seed, r=2.5, W=24, H=16, bg=(0.1, 0.2, 0.3))[0]
    return sc, v.replace(d_per_gaussian=per_gaussian)


def test_per_gaussian_direction_is_the_fixed_direction_slice_per_gaussian():
    """Slicing with d_i = unit(mu_p,i - c) equals slicing each Gaussian alone
    with that d as the view's direction (up to the FP32 rounding of a view's d)."""
    sc, v = _scene_view()
    s_all = oracle.slice_(sc, v)
    mu_p = np.asarray(sc.mu_p, np.float64)
    c = np.asarray(v.c, np.float64)
    for g in range(sc.n):
        e = mu_p[:, g] - c
        vg = v.replace(d_per_gaussian=False, d=e / np.linalg.norm(e))
        s_g = oracle.slice_(sc, vg)
        assert np.allclose(s_all.mu_c[:, g], s_g.mu_c[:, g], rtol=1e-6, atol=1e-8), g
        assert np.allclose(s_all.alpha_c[g], s_g.alpha_c[g], rtol=1e-5, atol=1e-12), g
        assert np.array_equal(s_all.cov_c[:, g], s_g.cov_c[:, g])   # Sigma_cond has no d in it
    # and the mode matters: the view's own d gives other opacities
    s_fix = oracle.slice_(sc, v.replace(d_per_gaussian=False))
    assert np.abs(s_fix.alpha_c - s_all.alpha_c).max() > 1e-3


def test_c_and_torch_forwards_agree_with_per_gaussian_direction():
    import torch
    sc, v = _scene_view(n=60, seed=51)
    a = oracle.render(sc, v).image
    P = og.scene_tensors(sc, requires_grad=False)
    with torch.no_grad():
        b = og.render_t(P, v).numpy()
    assert np.abs(a - b).max() < 1e-11


def test_fd_gradients_with_per_gaussian_direction():
    """With d depending on mu_p, central differences of the C forward still
    equal autograd for every parameter of a small scene."""
    sc, v = _scene_view(n=12, seed=52)
    v = v.replace(W=16, H=16)
    fd, ad = _fd_check(sc, v, (0, 0, 16, 16), _all_params(sc))
    assert len(fd) > 0.9 * 12 * 84
    err = np.abs(fd - ad)
    assert np.all(err <= 1e-6 * np.maximum(np.abs(ad), 1e-3 * np.abs(ad).max())), err.max()


def test_lambda_gradients_match_central_differences():
    for per_gaussian in (False, True):
        sc, v = _scene_view(per_gaussian, n=40, seed=53)
        v = v.replace(lambda_t=0.3, lambda_d=0.2)
        w = np.random.default_rng(5).normal(size=(3, v.H, v.W))
        g, _ = og.grad(sc, v, w)
        arrs = {k: np.asarray(getattr(sc, k), np.float32).astype(np.float64) for k in og.PARAMS}
        for j, name in enumerate(("lambda_t", "lambda_d")):
            h = 1e-6
            lp, hp = _loss_c(arrs, v.replace(**{name: getattr(v, name) + h}), w, (0, 0, v.W, v.H))
            lm, hm = _loss_c(arrs, v.replace(**{name: getattr(v, name) - h}), w, (0, 0, v.W, v.H))
            assert np.array_equal(hp, hm)          # same contributor sets
            # the view stores lambda in FP32: difference over the stored values
            hp_eff = float(np.float32(getattr(v, name) + h)) - float(np.float32(getattr(v, name) - h))
            fd = (lp - lm) / hp_eff
            assert abs(g["lambda"][j]) > 1e-4
            assert abs(fd - g["lambda"][j]) <= 1e-4 * abs(g["lambda"][j]), (per_gaussian, name, fd, g["lambda"][j])
