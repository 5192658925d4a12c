"""Pins of the oracle's conditional slicing (Sec. 4.2, Algorithm 1 steps 3-6)
against closed forms, identities and sampling -- never against itself."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import scenegen
from tests.helpers import axis_view, dense_cov, scene_from

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _one(L_entries, mu_p=(0, 0, 0), mu_t=0.0, mu_d=(0, 0, 1), alpha=0.5):
    Ld = np.eye(7)
    for (i, j), val in L_entries.items():
        Ld[i, j] = val
    return scene_from([mu_p], [mu_t], [mu_d], Ld[None], [alpha])


def test_x1_time_coupled_x_closed_form():
    """L = I except L00 = s, L30 = a, L33 = b couples x and t only.  By hand from
    eq. cond_mean/cond_cov: mu_x' = mu_x + s a/(a^2+b^2) (t - mu_t),
    Sigma_xx' = s^2 b^2/(a^2+b^2); other entries unchanged; f_temp =
    exp(-lambda_t (t-mu_t)^2 / (2 (a^2+b^2)))."""
    with open(os.path.join(GOLDEN, "slice_x1.json")) as f:
        cases = json.load(f)["cases"]
    for cs in cases:
        s, a, b = cs["s"], cs["a"], cs["b"]
        sc = _one({(0, 0): s, (3, 0): a, (3, 3): b}, mu_t=cs["mu_t"])
        v = axis_view(t=cs["t"], lam=cs["lambda"])
        out = oracle.slice_(sc, v)
        # closed form, evaluated from the FP32-rounded inputs
        s32, a32, b32 = (float(np.float32(x)) for x in (s, a, b))
        t32, mt32 = float(np.float32(cs["t"])), float(np.float32(cs["mu_t"]))
        den = a32 ** 2 + b32 ** 2
        exp_mu = np.array([s32 * a32 / den * (t32 - mt32), 0.0, 0.0])
        exp_cov = np.array([s32 ** 2 * b32 ** 2 / den, 0, 0, 1, 0, 1])
        lam32 = float(np.float32(cs["lambda"]))
        exp_ft = math.exp(-0.5 * lam32 * (t32 - mt32) ** 2 / den)
        np.testing.assert_allclose(out.mu_c[:, 0], exp_mu, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(out.cov_c[:, 0], exp_cov, rtol=1e-13, atol=1e-15)
        assert out.f_temp[0] == pytest.approx(exp_ft, rel=1e-13)
        assert out.f_dir[0] == pytest.approx(1.0, rel=1e-15)
        # the stored worked values (exactly representable cases)
        if cs.get("exact"):
            np.testing.assert_allclose(out.mu_c[:, 0], cs["mu_c"], rtol=1e-14)
            np.testing.assert_allclose(out.cov_c[:, 0], cs["cov_c"], rtol=1e-14)
            assert out.f_temp[0] == pytest.approx(cs["f_temp"], rel=1e-14)


def test_x2_zero_cross_covariance_is_3dgs():
    """L_QP = 0: the slice leaves mu_p and L_PP L_PP^T untouched (a 3DGS
    Gaussian) and only the opacity is modulated; lambda = 0 leaves alpha too."""
    rng = np.random.default_rng(5)
    n = 64
    Ld = np.zeros((n, 7, 7))
    for g in range(n):
        A = np.tril(rng.normal(0, 0.1, (7, 7)))
        A[np.diag_indices(7)] = np.exp(rng.uniform(-4, -1, 7))
        A[3:, :3] = 0.0
        Ld[g] = A
    sc = scene_from(rng.uniform(-1, 1, (n, 3)), rng.uniform(0, 1, n),
                    rng.normal(size=(n, 3)), Ld, rng.uniform(0.1, 0.9, n))
    for lam in (0.0, 0.3):
        v = axis_view(lam=lam, t=0.7)
        out = oracle.slice_(sc, v)
        np.testing.assert_array_equal(out.mu_c, sc.mu_p.astype(np.float64))
        S = dense_cov(sc)
        np.testing.assert_allclose(out.cov_c, np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2],
                                                        S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]]),
                                   rtol=1e-14, atol=1e-18)
        if lam == 0.0:
            np.testing.assert_array_equal(out.alpha_c, sc.alpha.astype(np.float64))


def test_x3_time_decoupled_is_6dgs():
    """Sigma_pt = 0 and Sigma_td = 0: the slice equals the 6DGS conditional on
    the direction alone (Sec. 3), and f_dir equals the 6DGS modulation with
    lambda_6D = lambda_d / 2 (the 6DGS exponent has no 1/2)."""
    rng = np.random.default_rng(6)
    n = 32
    Ld = np.zeros((n, 7, 7))
    for g in range(n):
        A = np.tril(rng.normal(0, 0.15, (7, 7)))
        A[np.diag_indices(7)] = np.exp(rng.uniform(-3, -1, 7))
        A[3, :3] = 0.0       # t row decoupled from p
        A[4:, 3] = 0.0       # d rows decoupled from t
        Ld[g] = A
    sc = scene_from(rng.uniform(-1, 1, (n, 3)), rng.uniform(0, 1, n),
                    rng.normal(size=(n, 3)), Ld, rng.uniform(0.1, 0.9, n))
    v = axis_view(lam=0.2, t=0.6)
    out = oracle.slice_(sc, v)
    S = dense_cov(sc)
    P, D = [0, 1, 2], [4, 5, 6]
    d = np.asarray(v.d, np.float64)
    for g in range(n):
        Sp, Spd, Sd = S[g][np.ix_(P, P)], S[g][np.ix_(P, D)], S[g][np.ix_(D, D)]
        delta = d - sc.mu_d[:, g].astype(np.float64)
        mu6 = sc.mu_p[:, g] + Spd @ np.linalg.solve(Sd, delta)
        cov6 = Sp - Spd @ np.linalg.solve(Sd, Spd.T)
        np.testing.assert_allclose(out.mu_c[:, g], mu6, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(out.cov_c[:, g], cov6[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]],
                                   rtol=1e-11, atol=1e-15)
        lam6 = v.lambda_d / 2
        fcond = math.exp(-lam6 * delta @ np.linalg.solve(Sd, delta))
        assert out.f_dir[g] == pytest.approx(fcond, rel=1e-12)


def _cov3(cov6):
    xx, xy, xz, yy, yz, zz = cov6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def test_x4_precision_block_determinant_and_loewner():
    """Sigma_cond^{-1} = (Sigma^{-1})_PP; det Sigma_cond = prod L_ii^2 / det
    Sigma_QQ; Sigma_cond <= Sigma_PP (Loewner); Sigma_cond does not depend on
    (t, d).  Tolerances scale with the conditioning of Sigma."""
    sc = scenegen.make_scene(200, 11, sigma_off=0.15)
    v1 = axis_view(t=0.1)
    v2 = v1.replace(t=0.9, d=np.array([0.6, 0.0, 0.8], np.float32))
    o1, o2 = oracle.slice_(sc, v1), oracle.slice_(sc, v2)
    np.testing.assert_array_equal(o1.cov_c, o2.cov_c)
    S = dense_cov(sc)
    Lp = sc.L.astype(np.float64)
    for g in range(sc.n):
        C = _cov3(o1.cov_c[:, g])
        prec = np.linalg.inv(S[g])[:3, :3]
        kappa = np.linalg.cond(S[g])
        resid = np.abs(C @ prec - np.eye(3)).max()
        assert resid < 1e-14 * kappa + 1e-12
        diag = np.array([Lp[scenegen.tri_index(i, i), g] for i in range(7)])
        det_expect = np.prod(diag ** 2) / np.linalg.det(S[g][3:, 3:])
        det_c = np.linalg.det(C)
        assert abs(det_c - det_expect) <= 1e-14 * kappa * abs(det_expect) + 1e-15 * np.abs(C).max() ** 3
        ev = np.linalg.eigvalsh(S[g][:3, :3] - C)
        assert ev.min() > -1e-13 * np.abs(S[g][:3, :3]).max()


def test_x4_against_50_digit_reference():
    """The FP64 slice agrees with the same conditional statistics evaluated in
    50-digit arithmetic (mpmath) to a few FP64 ulps of the entry scale,
    including nearly degenerate conditional covariances."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    sc = scenegen.make_scene(40, 13, sigma_off=0.15)
    v = axis_view(t=0.3).replace(d=np.array([0.0, 0.6, 0.8], np.float32))
    o = oracle.slice_(sc, v)
    Ld = scenegen.unpack_L(sc.L.T.astype(np.float64))
    d = [mp.mpf(float(x)) for x in np.asarray(v.d, np.float32)]
    for g in range(sc.n):
        L = mp.matrix(Ld[g].tolist())
        Sm = L * L.T
        SPP, SPQ, SQQ = Sm[0:3, 0:3], Sm[0:3, 3:7], Sm[3:7, 3:7]
        r = mp.matrix([mp.mpf(float(np.float32(v.t))) - mp.mpf(float(sc.mu_t[g]))] +
                      [d[k] - mp.mpf(float(sc.mu_d[k, g])) for k in range(3)])
        K = SPQ * mp.inverse(SQQ)
        mu = [float(mp.mpf(float(sc.mu_p[k, g])) + (K * r)[k]) for k in range(3)]
        Sc = SPP - K * SPQ.T
        c6 = [float(Sc[i, j]) for i, j in [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]]
        scale = float(max(abs(x) for x in SPP))
        np.testing.assert_allclose(o.cov_c[:, g], c6, rtol=0, atol=64 * 2.2e-16 * scale)
        np.testing.assert_allclose(o.mu_c[:, g], mu, rtol=0, atol=64 * 2.2e-16 * (1 + max(abs(x) for x in mu)))


def test_x4_affine_mean_matches_regression_coefficients():
    """mu_cond is affine in r = (t - mu_t, d - mu_d) with slope K = Sigma_PQ
    Sigma_QQ^{-1}; K estimated by least-squares regression of X_p on X_q over
    Monte-Carlo draws of the 7D Gaussian agrees within sampling error, and so
    does the residual covariance with Sigma_cond."""
    sc = scenegen.make_scene(3, 12, sigma_off=0.15)
    Ld = scenegen.unpack_L(sc.L.T.astype(np.float64))
    rng = np.random.default_rng(0)
    M = 400_000
    for g in range(3):
        mu = np.concatenate([sc.mu_p[:, g], [sc.mu_t[g]], sc.mu_d[:, g]]).astype(np.float64)
        X = mu[None, :] + rng.normal(size=(M, 7)) @ Ld[g].T
        Xq = np.concatenate([X[:, 3:] - mu[3:], np.ones((M, 1))], 1)
        coef, *_ = np.linalg.lstsq(Xq, X[:, :3], rcond=None)
        K_hat = coef[:4].T
        resid = X[:, :3] - Xq @ coef
        C_hat = resid.T @ resid / M
        # the oracle's mean at two conditioning points gives K along r1 - r0
        v0 = axis_view(t=float(sc.mu_t[g]), lam=0.0).replace(d=sc.mu_d[:, g])
        v1 = axis_view(t=float(sc.mu_t[g]) + 0.25, lam=0.0).replace(
            d=sc.mu_d[:, g] + np.array([0.5, -0.25, 0.125], np.float32))
        o0, o1 = oracle.slice_(sc, v0), oracle.slice_(sc, v1)
        dr = np.array([np.float32(v1.t) - np.float32(v0.t)] +
                      list(np.asarray(v1.d, np.float64) - np.asarray(v0.d, np.float64)))
        slope = o1.mu_c[:, g] - o0.mu_c[:, g]
        tol = 6 * np.sqrt(np.diag(C_hat)) / np.sqrt(M) * np.abs(dr).sum() / np.sqrt(
            np.diag(np.cov((X[:, 3:] - mu[3:]).T)).min())
        np.testing.assert_allclose(slope, K_hat @ dr, atol=float(tol.max()) + 1e-4)
        C = _cov3(o0.cov_c[:, g])
        np.testing.assert_allclose(C, C_hat, atol=6 * np.abs(C).max() * np.sqrt(2 / M) * 3)


def test_x5_latent_whitening_identity():
    """A second derivation of the slice: write X = mu + L z, z ~ N(0, I7), and
    condition the latent z.  With G = L_QQ^{-1} L_QP, w = L_QQ^{-1} r and
    M = I + G^T G = C C^T:  mu_c = mu_p + L_PP M^{-1} G^T w and
    Sigma_c = (L_PP C^{-T})(L_PP C^{-T})^T.  This route shares no algebra with
    the Schur complement; its own rounding grows with cond(M), so the tolerance
    does too."""
    sc = scenegen.make_scene(500, 13, sigma_off=0.15)
    v = axis_view(t=0.3).replace(d=np.array([0.0, 0.6, 0.8], np.float32))
    o = oracle.slice_(sc, v)
    Ld = scenegen.unpack_L(sc.L.T.astype(np.float64))
    d = np.asarray(v.d, np.float64)
    for g in range(sc.n):
        L = Ld[g]
        LPP, LQP, LQQ = L[:3, :3], L[3:, :3], L[3:, 3:]
        r = np.concatenate([[np.float64(v.t) - sc.mu_t[g]], d - sc.mu_d[:, g]])
        G = np.linalg.solve(LQQ, LQP)
        w = np.linalg.solve(LQQ, r)
        Mm = np.eye(3) + G.T @ G
        Cm = np.linalg.cholesky(Mm)
        mu = sc.mu_p[:, g] + LPP @ np.linalg.solve(Mm, G.T @ w)
        B = LPP @ np.linalg.inv(Cm).T
        cov = B @ B.T
        amp = 1e-14 * np.linalg.cond(Mm) * max(1.0, np.linalg.cond(LQQ))
        np.testing.assert_allclose(o.mu_c[:, g], mu, rtol=0, atol=amp * (1 + np.abs(mu).max()))
        c6 = cov[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
        np.testing.assert_allclose(o.cov_c[:, g], c6, rtol=0, atol=amp * np.abs(LPP @ LPP.T).max())


def test_modulation_marginal_blocks():
    """f_temp uses the marginal variance Sigma_t and f_dir the marginal block
    Sigma_d (Sec. 4.1 defines both as marginals), not blocks of the
    inverse of Sigma_(t,d)."""
    sc = scenegen.make_scene(50, 14, sigma_off=0.15)
    v = axis_view(t=0.9, lam=0.3).replace(d=np.array([0.0, 0.0, -1.0], np.float32))
    o = oracle.slice_(sc, v)
    S = dense_cov(sc)
    for g in range(sc.n):
        dt = np.float64(v.t) - sc.mu_t[g]
        dl = np.asarray(v.d, np.float64) - sc.mu_d[:, g]
        ft = math.exp(-0.5 * 0.3 * dt * dt / S[g, 3, 3])
        fd = math.exp(-0.5 * 0.3 * dl @ np.linalg.inv(S[g, 4:, 4:]) @ dl)
        lam = float(np.float32(0.3))
        ft = math.exp(-0.5 * lam * dt * dt / S[g, 3, 3])
        fd = math.exp(-0.5 * lam * dl @ np.linalg.inv(S[g, 4:, 4:]) @ dl)
        assert o.f_temp[g] == pytest.approx(ft, rel=1e-12)
        assert o.f_dir[g] == pytest.approx(fd, rel=1e-10)
        assert o.alpha_c[g] == pytest.approx(float(sc.alpha[g]) * ft * fd, rel=1e-10)


def test_nonpositive_diagonal_is_reported():
    sc = _one({(5, 5): -0.1})
    o = oracle.slice_(sc, axis_view())
    assert o.status[0] & 1
