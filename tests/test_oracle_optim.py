"""Pins of the oracle's optimizer step and pruning: Adam's bias-corrected
steps in closed form, the projections, and pruning by the opacity floor."""
import numpy as np

from oracle.optim import DIAG, GROUPS, adam_step, prune

SH = {"mu_p": 3, "mu_t": 1, "mu_d": 3, "L": 28, "alpha": 1, "sh": 48}


def _zeros(n):
    return {k: np.zeros((SH[k], n)) if SH[k] > 1 else np.zeros(n) for k in GROUPS}


def test_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step moves a value by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(0)
    n = 17
    p0 = {k: rng.uniform(0.2, 0.8, a.shape) for k, a in _zeros(n).items()}
    g = {k: rng.normal(0, 1e-2, a.shape) for k, a in _zeros(n).items()}
    lr = {k: 1e-3 * (i + 1) for i, k in enumerate(GROUPS)}
    p, m, v = p0, _zeros(n), _zeros(n)
    for t in range(1, 6):
        p, m, v = adam_step(p, g, m, v, lr, t, alpha_bounds=(-1e9, 1e9), diag_min=-1e9)
        for k in GROUPS:
            want = p0[k] - t * lr[k] * g[k] / (np.abs(g[k]) + 1e-15)
            assert np.allclose(p[k], want, rtol=0, atol=1e-12 * t), (k, t)


def test_zero_gradient_changes_nothing_and_projections_hold():
    n = 9
    p0 = {k: np.full(a.shape, 0.5) for k, a in _zeros(n).items()}
    p0["alpha"][:] = [0.0, 1.0, 0.5, 2.0, -1.0, 0.3, 0.99999, 1e-6, 0.7]
    p0["L"][DIAG[3]] = -0.2
    p, m, v = adam_step(p0, _zeros(n), _zeros(n), _zeros(n), {k: 1.0 for k in GROUPS}, 1)
    assert np.array_equal(p["alpha"], np.clip(p0["alpha"], 1e-4, 0.9999))
    assert np.all(p["L"][DIAG] >= 1e-4) and np.all(p["L"][DIAG[3]] == 1e-4)
    for k in ("mu_p", "mu_t", "mu_d", "sh"):
        assert np.array_equal(p[k], p0[k])
        assert not m[k].any() and not v[k].any()


def test_prune_keeps_the_gaussians_at_or_above_the_floor_in_order():
    a = np.array([0.5, 0.009, 0.01, 0.2, 0.0099999, 1.0])
    arr = {"alpha": a, "x": np.arange(12.0).reshape(2, 6)}
    out = prune(arr, a, 0.01)
    assert np.array_equal(out["alpha"], [0.5, 0.01, 0.2, 1.0])
    assert np.array_equal(out["x"], [[0, 2, 3, 5], [6, 8, 9, 11]])
