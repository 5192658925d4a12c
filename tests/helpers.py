"""Small builders shared by the tests (inputs only; no method arithmetic)."""
import numpy as np

import scenegen
from scenegen import Scene, tri_index


def pack_L(Ld: np.ndarray) -> np.ndarray:
    """[n][7][7] dense lower-triangular -> [28][n] packed planes (FP32)."""
    n = Ld.shape[0]
    out = np.zeros((28, n), np.float32)
    for i in range(7):
        for j in range(i + 1):
            out[tri_index(i, j)] = Ld[:, i, j]
    return out


def scene_from(mu_p, mu_t, mu_d, Ld, alpha, sh=None) -> Scene:
    mu_p = np.asarray(mu_p, np.float32).reshape(-1, 3)
    n = mu_p.shape[0]
    if sh is None:
        sh = np.zeros((n, 48), np.float32)
    return Scene(mu_p=np.ascontiguousarray(mu_p.T),
                 mu_t=np.asarray(mu_t, np.float32).reshape(n),
                 mu_d=np.ascontiguousarray(np.asarray(mu_d, np.float32).reshape(n, 3).T),
                 L=pack_L(np.asarray(Ld, np.float64).reshape(n, 7, 7)),
                 alpha=np.asarray(alpha, np.float32).reshape(n),
                 sh=np.ascontiguousarray(np.asarray(sh, np.float32).reshape(n, 48).T))


def dense_cov(scene: Scene) -> np.ndarray:
    """FP64 Sigma = L L^T per Gaussian, [n][7][7] (test-side, via numpy)."""
    Ld = scenegen.unpack_L(scene.L.T.astype(np.float64))
    return Ld @ np.transpose(Ld, (0, 2, 1))


def axis_view(W=64, H=64, z0=3.0, t=0.5, lam=0.05, bg=(0, 0, 0)):
    """Camera at (0, 0, -z0) looking at the origin along world +z... expressed
    with an explicit rotation so that camera axes equal world axes."""
    R = np.eye(3, dtype=np.float32)
    f = (W / 2.0) / scenegen.TAN_HALF_FOV
    v = scenegen.View(R_wc=R, c=np.array([0, 0, -z0], np.float32), fx=f, fy=f, cx=W / 2.0,
                      cy=H / 2.0, W=W, H=H, t=t, d=np.array([0, 0, 1], np.float32),
                      lambda_t=lam, lambda_d=lam, bg=np.asarray(bg, np.float32))
    v._cast()
    return v
