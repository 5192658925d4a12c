"""Densification helpers of the oracle -- TEST INFRASTRUCTURE.

Algorithm 1's optional step and Sec. 4.4: Sigma_cond = U D U^T, scale
S = sqrt(diag D), rotation R = U with its last column multiplied by
sign(det R); the temporal split test |Sigma_pt| > 0.05 extent and a
normalized temporal scale sqrt(Sigma_t) / time_span > 0.25.  FP64 numpy;
shares nothing with the HIP library.
"""
from __future__ import annotations

import numpy as np


def cov_decompose(cov6: np.ndarray):
    """cov6 [6][n] packed (xx, xy, xz, yy, yz, zz) -> scale [3][n] (descending),
    rot [3][3][n] (R[:, :, i] with det +1), eigenvalues [3][n]."""
    c = np.asarray(cov6, np.float64)
    n = c.shape[1]
    A = np.empty((n, 3, 3))
    A[:, 0, 0], A[:, 0, 1], A[:, 0, 2] = c[0], c[1], c[2]
    A[:, 1, 0], A[:, 1, 1], A[:, 1, 2] = c[1], c[3], c[4]
    A[:, 2, 0], A[:, 2, 1], A[:, 2, 2] = c[2], c[4], c[5]
    w, U = np.linalg.eigh(A)                  # ascending
    w, U = w[:, ::-1], U[:, :, ::-1]          # descending, as an SVD orders them
    det = np.linalg.det(U)
    U[:, :, 2] *= np.sign(det)[:, None]
    S = np.sqrt(np.maximum(w, 0.0))
    return S.T.copy(), np.transpose(U, (1, 2, 0)).copy(), w.T.copy()


def split_test(L_packed: np.ndarray, extent: float, time_span: float = 1.0):
    """Returns (split [n] bool, m1, m2) with m1 = |Sigma_pt| - 0.05 extent and
    m2 = sqrt(Sigma_t) / time_span - 0.25 (split iff both are > 0)."""
    Lp = np.asarray(L_packed, np.float64)
    n = Lp.shape[1]
    L = np.zeros((n, 7, 7))
    for i in range(7):
        for j in range(i + 1):
            L[:, i, j] = Lp[i * (i + 1) // 2 + j]
    S = L @ np.transpose(L, (0, 2, 1))
    spt = np.linalg.norm(S[:, :3, 3], axis=1)
    m1 = spt - 0.05 * extent
    m2 = np.sqrt(S[:, 3, 3]) / time_span - 0.25
    return (m1 > 0) & (m2 > 0), m1, m2
