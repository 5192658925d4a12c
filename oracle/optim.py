"""Optimizer step and pruning of the oracle -- TEST INFRASTRUCTURE.

Sec. 4.4 keeps the 3DGS optimizer (Adam) and prunes Gaussians below the
opacity floor tau_min = 0.01.  Adam written out in FP64 numpy, in PyTorch's
order: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
p -= lr/(1-b1^t) * m / (sqrt(v)/sqrt(1-b2^t) + eps); then the projections the
library applies (opacity into [alpha_lo, alpha_hi], L's diagonal >= diag_min).
"""
from __future__ import annotations

import numpy as np

GROUPS = ("mu_p", "mu_t", "mu_d", "L", "alpha", "sh")
DIAG = [i * (i + 1) // 2 + i for i in range(7)]


def adam_step(p: dict, g: dict, m: dict, v: dict, lr: dict, t: int, beta1=0.9, beta2=0.999, eps=1e-15,
              alpha_bounds=(1e-4, 0.9999), diag_min=1e-4):
    """Returns new (p, m, v) dicts of FP64 arrays."""
    P, M, V = {}, {}, {}
    for k in GROUPS:
        gk = np.asarray(g[k], np.float64)
        M[k] = beta1 * np.asarray(m[k], np.float64) + (1 - beta1) * gk
        V[k] = beta2 * np.asarray(v[k], np.float64) + (1 - beta2) * gk * gk
        denom = np.sqrt(V[k]) / np.sqrt(1 - beta2 ** t) + eps
        P[k] = np.asarray(p[k], np.float64) - lr[k] / (1 - beta1 ** t) * M[k] / denom
    P["alpha"] = np.clip(P["alpha"], alpha_bounds[0], alpha_bounds[1])
    P["L"][DIAG] = np.maximum(P["L"][DIAG], diag_min)
    return P, M, V


def prune(arrays: dict, alpha, tau: float) -> dict:
    """The Gaussians with alpha >= tau, in their order (last axis)."""
    keep = np.asarray(alpha) >= tau
    return {k: np.asarray(a)[..., keep] for k, a in arrays.items()}
