"""Pins of the oracle's adaptive Gaussian refinement (Sec. 4.3; Algorithm 1
steps 1-2): values of gamma(t) known in closed form, the identity of zero
weights, networks small enough to evaluate by hand, and the affine regime
checked against the composed weight matrices."""
import math

import numpy as np
import pytest

import oracle
import scenegen

OUT = (3, 1, 3, 28)
H, IN = 64, 27


def blocks(w):
    """Views (W1, b1, W2, b2) of each MLP in a packed weight vector."""
    out, off = [], 0
    for c in OUT:
        W1 = w[off:off + H * IN].reshape(H, IN); off += H * IN
        b1 = w[off:off + H]; off += H
        W2 = w[off:off + c * H].reshape(c, H); off += c * H
        b2 = w[off:off + c]; off += c
        out.append((W1, b1, W2, b2))
    assert off == w.size
    return out


def zeros():
    return np.zeros(oracle.AGR_WEIGHTS)


@pytest.mark.parametrize("t,expect", [
    (0.0, [(0.0, 1.0)] * 10),
    (0.5, [(1.0, 0.0), (0.0, -1.0)] + [(0.0, 1.0)] * 8),
    (1.0 / 3.0, [(math.sqrt(3) / 2, 0.5), (math.sqrt(3) / 2, -0.5), (-math.sqrt(3) / 2, -0.5)]),
    (1.0 / 6.0, [(0.5, math.sqrt(3) / 2), (math.sqrt(3) / 2, 0.5), (math.sqrt(3) / 2, -0.5),
                 (-math.sqrt(3) / 2, -0.5)]),
])
def test_encoding_closed_form_values(t, expect):
    g = oracle.agr_encoding(t)
    assert g.shape == (20,)
    for k, (s, c) in enumerate(expect):
        assert abs(g[2 * k] - s) < 1e-12 and abs(g[2 * k + 1] - c) < 1e-12, k


def test_zero_weights_are_the_identity():
    sc, views = scenegen.config0()
    r = oracle.agr(sc, 0.3, zeros())
    for k in ("mu_p", "mu_t", "mu_d", "L"):
        assert np.array_equal(getattr(r, k), np.asarray(getattr(sc, k), np.float64)), k
    a = oracle.render(sc, views[0])
    b = oracle.render(sc, views[0], agr_weights=zeros())
    assert np.array_equal(a.image, b.image) and np.array_equal(a.final_T, b.final_T)


def test_output_biases_land_on_their_parameters():
    """W1 = W2 = 0: each MLP adds its b2, entry by entry, to its own parameter
    (the L output in the packed order of L)."""
    sc = scenegen.make_scene(40, 3)
    w = zeros()
    bl = blocks(w)
    shifts = [np.array([0.1, -0.2, 0.3]), np.array([0.05]), np.array([-0.01, 0.02, 0.03]),
              np.arange(28) * 1e-3 + 1e-3]
    for (W1, b1, W2, b2), s in zip(bl, shifts):
        b2[:] = s
    r = oracle.agr(sc, 0.7, w)
    base = {k: np.asarray(getattr(sc, k), np.float64) for k in ("mu_p", "mu_t", "mu_d", "L")}
    assert np.allclose(r.mu_p - base["mu_p"], shifts[0][:, None], atol=1e-15)
    assert np.allclose(r.mu_t - base["mu_t"], shifts[1][0], atol=1e-15)
    assert np.allclose(r.mu_d - base["mu_d"], shifts[2][:, None], atol=1e-15)
    assert np.allclose(r.L - base["L"], shifts[3][:, None], atol=1e-15)


def test_hand_evaluated_units():
    """MLP t, unit 0: h = relu(mu_t - 0.5), phi_t = 2 h + 0.1.  MLP p, unit 5:
    h = relu(cos(2 pi t) + 1.5) (input 10 = cos(2^1 pi t)), phi_p[0] = 4 h.
    MLP d, unit 9: h = relu(mu_d[1]) (input 5), phi_d[2] = h."""
    sc = scenegen.make_scene(3, 8)
    sc.mu_t[:] = np.array([0.8, 0.3, 0.5], np.float32)
    sc.mu_d[1, :] = np.array([0.25, -0.5, 0.0], np.float32)
    w = zeros()
    (pW1, pb1, pW2, pb2), (tW1, tb1, tW2, tb2), (dW1, db1, dW2, db2), _ = blocks(w)
    tW1[0, 3] = 1.0; tb1[0] = -0.5; tW2[0, 0] = 2.0; tb2[0] = 0.1
    pW1[5, 10] = 1.0; pb1[5] = 1.5; pW2[0, 5] = 4.0
    dW1[9, 5] = 1.0; dW2[2, 9] = 1.0
    t = 0.5                                   # cos(2 pi t) = -1
    r = oracle.agr(sc, t, w)
    mt = np.asarray(sc.mu_t, np.float64)
    assert np.allclose(r.mu_t - mt, [2 * 0.3 + 0.1, 0.1, 0.1], atol=1e-7)
    assert np.allclose(r.mu_p[0] - np.asarray(sc.mu_p[0], np.float64), 4 * 0.5, atol=1e-12)
    assert np.allclose(r.mu_p[1:] - np.asarray(sc.mu_p[1:], np.float64), 0.0, atol=0)
    md = np.asarray(sc.mu_d, np.float64)
    assert np.allclose(r.mu_d[2] - md[2], [0.25, 0.0, 0.0], atol=1e-12)
    assert np.array_equal(r.mu_d[:2], md[:2])


def test_all_units_active_equals_the_composed_affine_map():
    """With every hidden pre-activation positive the MLP is affine:
    phi = (W2 W1) f + (W2 b1 + b2).  Evaluated here with the products taken
    in the other order, so a transposed or misindexed operand shows."""
    rng = np.random.default_rng(11)
    sc = scenegen.make_scene(25, 12)
    w = rng.normal(0, 0.3, oracle.AGR_WEIGHTS)
    bl = blocks(w)
    for W1, b1, W2, b2 in bl:
        b1[:] = 50.0 + rng.uniform(0, 1, H)   # |W1 f| < 50 for these inputs
    t = 0.37
    r = oracle.agr(sc, t, w)
    f = np.concatenate([np.asarray(sc.mu_p, np.float64), np.asarray(sc.mu_t, np.float64)[None],
                        np.asarray(sc.mu_d, np.float64),
                        np.repeat(oracle.agr_encoding(t)[:, None], sc.n, 1)])
    assert f.shape == (27, sc.n)
    names = ("mu_p", "mu_t", "mu_d", "L")
    for (W1, b1, W2, b2), k in zip(bl, names):
        assert np.all(W1 @ f + b1[:, None] > 0)
        phi = (W2 @ W1) @ f + (W2 @ b1 + b2)[:, None]
        got = getattr(r, k).reshape(phi.shape[0], -1) - np.asarray(getattr(sc, k), np.float64).reshape(
            phi.shape[0], -1)
        assert np.allclose(got, phi, rtol=1e-12, atol=1e-9), k


def test_refinement_happens_before_the_slice():
    """Rendering with AGR equals rendering the refined parameters."""
    sc, views = scenegen.config0()
    w = scenegen.agr_weights(7)
    v = views[0]
    r = oracle.agr(sc, v.t, w)
    a = oracle.render(sc, v, agr_weights=w)
    b = oracle.render(r, v)
    assert np.array_equal(a.image, b.image)
    s1 = oracle.slice_(sc, v, agr_weights=w)
    s2 = oracle.slice_(r, v)
    assert np.array_equal(s1.mu_c, s2.mu_c) and np.array_equal(s1.alpha_c, s2.alpha_c)
    # and it is not the identity for these weights
    assert np.abs(a.image - oracle.render(sc, v).image).max() > 1e-2
