"""Pins of the oracle's projection and compositing (Sec. 4.4) and SH colour
(Sec. 3, eq. 2) against analytic images, library routines and symmetries."""
import math

import numpy as np
import pytest

import oracle
import oracle.grad as og
import scenegen
from tests.helpers import axis_view, scene_from

pi = math.pi
Y00 = 0.5 / math.sqrt(pi)


def _iso_scene(s_list, z_list, alpha_list, dc_list, mu_t=0.5):
    """Isotropic Gaussians on the optical axis of axis_view(): spatial factor
    s I, no coupling to (t, d), mu_d = (0, 0, 1), DC-only colour."""
    n = len(s_list)
    Ld = np.zeros((n, 7, 7))
    sh = np.zeros((n, 48))
    for g in range(n):
        Ld[g] = np.eye(7)
        Ld[g][:3, :3] = s_list[g] * np.eye(3)
        sh[g, 0:3] = dc_list[g]
    mu_p = np.array([[0.0, 0.0, z] for z in z_list])
    return scene_from(mu_p, [mu_t] * n, [(0, 0, 1)] * n, Ld, alpha_list, sh)


def _analytic_alpha(view, s, z_world, alpha):
    """alpha(p) of an on-axis isotropic Gaussian: Sigma_2D = (f^2 s^2 / z^2 + 0.3) I."""
    z = float(z_world) - float(view.c[2])
    f = float(view.fx)
    s = float(np.float32(s))
    var = f * f * s * s / (z * z) + oracle.DILATION
    ys, xs = np.mgrid[0:view.H, 0:view.W] + 0.5
    q = ((xs - view.cx) ** 2 + (ys - view.cy) ** 2) / var
    a = np.minimum(oracle.ALPHA_MAX, float(np.float32(alpha)) * np.exp(-0.5 * q))
    return np.where(a >= oracle.ALPHA_MIN, a, 0.0)


def test_x7_ewa_on_axis_closed_form():
    v = axis_view(W=64, H=48, z0=3.0)
    sl = oracle.Sliced(mu_c=np.zeros((3, 1)), cov_c=np.array([[0.01], [0], [0], [0.01], [0], [0.01]]),
                       alpha_c=np.array([0.8]), f_temp=None, f_dir=None, status=None)
    pr = oracle.project(sl, np.zeros((48, 1)), v)
    assert pr.visible[0]
    np.testing.assert_allclose(pr.mean2d[:, 0], [v.cx, v.cy], atol=1e-12)
    var = v.fx ** 2 * 0.01 / 9.0 + oracle.DILATION
    np.testing.assert_allclose(pr.conic[:, 0], [1 / var, 0, 1 / var], rtol=1e-13, atol=1e-16)
    assert pr.depth[0] == pytest.approx(3.0, abs=1e-15)


def test_x7_ewa_jacobian_by_finite_differences():
    """Off axis (J unclamped), Sigma_2D - 0.3 I equals J_fd Sigma_c J_fd^T with
    J_fd the central-difference Jacobian of the projected mean w.r.t. the
    world position."""
    sc = scenegen.make_scene(1, 3)
    v = scenegen.make_view([1.0, -2.5, 1.2], 80, 60, 0.5)
    mu = np.array([[0.2], [0.1], [-0.3]])
    cov = np.array([[0.02], [0.004], [-0.003], [0.01], [0.002], [0.03]])
    sl = oracle.Sliced(mu, cov, np.array([0.9]), None, None, None)
    pr = oracle.project(sl, sc.sh, v)
    h = 1e-6
    J = np.zeros((2, 3))
    for k in range(3):
        mp_, mm = mu.copy(), mu.copy()
        mp_[k] += h
        mm[k] -= h
        up = oracle.project(oracle.Sliced(mp_, cov, np.array([0.9]), None, None, None), sc.sh, v).mean2d[:, 0]
        um = oracle.project(oracle.Sliced(mm, cov, np.array([0.9]), None, None, None), sc.sh, v).mean2d[:, 0]
        J[:, k] = (up - um) / (2 * h)
    S = np.array([[cov[0, 0], cov[1, 0], cov[2, 0]], [cov[1, 0], cov[3, 0], cov[4, 0]],
                  [cov[2, 0], cov[4, 0], cov[5, 0]]])
    S2 = J @ S @ J.T + oracle.DILATION * np.eye(2)
    a, b, c = pr.conic[:, 0]
    S2_oracle = np.linalg.inv(np.array([[a, b], [b, c]]))
    np.testing.assert_allclose(S2_oracle, S2, rtol=1e-7)


def test_x8_sh_orthonormal_and_matches_scipy():
    """The 16 real SH functions are orthonormal on the sphere (exact Gauss-
    Legendre x uniform-phi quadrature) and equal the real combinations of
    scipy's complex Y_l^m (Condon-Shortley phase): sqrt2 Re Y_l^m for m > 0,
    sqrt2 Im Y_l^|m| for m < 0."""
    from scipy.special import sph_harm_y
    xg, wg = np.polynomial.legendre.leggauss(10)
    nphi = 20
    gram = np.zeros((16, 16))
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for j in range(nphi):
            ph = 2 * pi * j / nphi
            Y = oracle.sh_basis(st * math.cos(ph), st * math.sin(ph), ct)
            gram += w * (2 * pi / nphi) * np.outer(Y, Y)
            theta = math.acos(ct)
            for l in range(4):
                for m in range(-l, l + 1):
                    k = l * l + l + m
                    if m == 0:
                        ref = sph_harm_y(l, 0, theta, ph).real
                    elif m > 0:
                        ref = math.sqrt(2) * sph_harm_y(l, m, theta, ph).real
                    else:
                        ref = math.sqrt(2) * sph_harm_y(l, -m, theta, ph).imag
                    assert Y[k] == pytest.approx(ref, abs=1e-13)
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-13)


def test_x10_single_gaussian_analytic_image():
    """One Gaussian: C(p) = rgb alpha(p) + (1 - alpha(p)) bg with the analytic
    on-axis alpha(p); never terminates since 1 - alpha >= 0.01 > T_MIN."""
    v = axis_view(W=64, H=64, z0=3.0, bg=(0.25, 0.5, 1.0))
    sc = _iso_scene([0.15], [0.0], [0.9], [(0.8, -0.3, 2.0)])
    im = oracle.render(sc, v)
    a = _analytic_alpha(v, 0.15, 0.0, 0.9)
    rgb = np.maximum(0.0, 0.5 + np.array([np.float32(0.8), np.float32(-0.3), np.float32(2.0)],
                                         np.float64) * Y00)
    bg = np.array([0.25, 0.5, 1.0])
    expect = rgb[:, None, None] * a[None] + (1 - a[None]) * bg[:, None, None]
    np.testing.assert_allclose(im.image, expect, atol=1e-14)
    np.testing.assert_allclose(im.final_T, 1 - a, atol=1e-14)
    assert (a > 0).sum() > 100 and (a == 0).sum() > 100


def test_x11_two_gaussians_front_to_back():
    """C = c1 a1 + c2 a2 (1 - a1) + bg (1 - a1)(1 - a2), nearer Gaussian first
    whatever the index order."""
    v = axis_view(W=48, H=48, z0=3.0, bg=(0.1, 0.2, 0.3))
    # index 0 is the far one
    sc = _iso_scene([0.2, 0.1], [0.5, -0.5], [0.7, 0.6], [(1.0, 0.0, 0.0), (0.0, 1.0, -1.0)])
    im = oracle.render(sc, v)
    a_far = _analytic_alpha(v, 0.2, 0.5, 0.7)
    a_near = _analytic_alpha(v, 0.1, -0.5, 0.6)
    c_far = np.maximum(0, 0.5 + np.array([1.0, 0.0, 0.0]) * Y00)
    c_near = np.maximum(0, 0.5 + np.array([0.0, 1.0, -1.0]) * Y00)
    bg = np.array([0.1, 0.2, 0.3])
    expect = (c_near[:, None, None] * a_near + c_far[:, None, None] * a_far * (1 - a_near)
              + bg[:, None, None] * (1 - a_near) * (1 - a_far))
    np.testing.assert_allclose(im.image, expect, atol=1e-14)


def test_x12_termination_excludes_the_saturating_gaussian():
    """16 coincident wide Gaussians with alpha ~ 0.5 at the centre: the first 13
    contribute and the 14th would push T below 1e-4 (0.5^14 < 1e-4 <= 0.5^13),
    so it and all later ones are excluded."""
    v = axis_view(W=16, H=16, z0=3.0, bg=(1.0, 1.0, 1.0))
    k = 16
    sc = _iso_scene([50.0] * k, [0.0] * k, [0.5] * k, [(2.0, 2.0, 2.0)] * k)
    im = oracle.render(sc, v)
    a = _analytic_alpha(v, 50.0, 0.0, 0.5)[8, 8]
    assert 0.4999 < a < 0.5
    T13 = (1 - a) ** 13
    rgb = 0.5 + float(np.float32(2.0)) * Y00
    expect = rgb * (1 - T13) + 1.0 * T13
    assert im.ncontrib[8, 8] == 13
    assert im.final_T[8, 8] == pytest.approx(T13, rel=1e-12)
    np.testing.assert_allclose(im.image[:, 8, 8], expect, rtol=1e-12)
    assert abs(T13 - 2.0 ** -13) < 1e-8


def test_x13_transparent_scene_is_background_and_order_invariant():
    sc, views = scenegen.config0()
    v = views[0].replace(bg=np.array([0.3, 0.6, 0.9], np.float32))
    clear = scenegen.Scene(sc.mu_p, sc.mu_t, sc.mu_d, sc.L, np.full_like(sc.alpha, 1e-4), sc.sh)
    im = oracle.render(clear, v)
    bg = np.array([0.3, 0.6, 0.9], np.float32).astype(np.float64)
    np.testing.assert_array_equal(im.image, np.broadcast_to(bg[:, None, None], im.image.shape))
    perm = np.random.default_rng(3).permutation(sc.n)
    a = oracle.render(sc, v)
    b = oracle.render(sc.subset(perm), v)
    np.testing.assert_allclose(a.image, b.image, atol=1e-15)


def test_x9_rotation_about_z_by_pi_is_exact():
    """Rotating world, camera and view direction by pi about z (a sign flip of
    x and y: exact in FP32) and the SH coefficients by (-1)^m leaves the image
    unchanged.  L transforms as B L B with B = diag(-1,-1,1, 1, -1,-1,1)."""
    sc, views = scenegen.config0()
    v = views[0]
    Q = np.diag([-1.0, -1.0, 1.0]).astype(np.float32)
    B = np.array([-1, -1, 1, 1, -1, -1, 1], np.float32)
    L2 = sc.L.copy()
    for i in range(7):
        for j in range(i + 1):
            L2[scenegen.tri_index(i, j)] *= B[i] * B[j]
    sh2 = sc.sh.copy()
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            sh2[3 * k:3 * k + 3] *= (-1) ** abs(m)
    sc2 = scenegen.Scene(Q @ sc.mu_p, sc.mu_t.copy(), Q @ sc.mu_d, L2, sc.alpha.copy(), sh2)
    v2 = v.replace(R_wc=v.R_wc @ Q.T, c=Q @ v.c, d=Q @ v.d)
    a, b = oracle.render(sc, v), oracle.render(sc2, v2)
    np.testing.assert_allclose(a.image, b.image, atol=1e-12)
    np.testing.assert_array_equal(a.ncontrib, b.ncontrib)


def test_c_and_torch_forwards_agree():
    """The two independent FP64 forwards (C and PyTorch) produce the same image."""
    for lam in (0.05, 0.5):
        sc, views = scenegen.config0(lam=lam)
        im = oracle.render(sc, views[0])
        P = og.scene_tensors(sc, requires_grad=False)
        img = og.render_t(P, views[0]).numpy()
        np.testing.assert_allclose(img, im.image, atol=1e-11)
    sc = scenegen.make_scene(3000, 21, h=1.0, sigma_off=0.15)
    v = scenegen.make_views(1, 21, r=3.0, W=256, H=192)[0]
    crop = (96, 64, 48, 40)
    im = oracle.render(sc, v, crop=crop)
    img = og.render_t(og.scene_tensors(sc, requires_grad=False), v, crop=crop).numpy()
    np.testing.assert_allclose(img, im.image, atol=1e-11)
