"""Pins of the oracle's densification helpers: decompositions of covariances
built from known scales and rotations, and split decisions on hand-built
factors."""
import numpy as np

from oracle.densify import cov_decompose, split_test


def pack(A):
    return np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]])[:, None]


def rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def test_diagonal_covariance():
    S, R, _ = cov_decompose(pack(np.diag([4.0, 9.0, 1.0])))
    assert np.allclose(S[:, 0], [3.0, 2.0, 1.0], atol=1e-14)
    R = R[:, :, 0]
    # columns: +-e_y, +-e_x, then the sign that makes R proper
    assert np.allclose(np.abs(R), [[0, 1, 0], [1, 0, 0], [0, 0, 1]], atol=1e-14)
    assert abs(np.linalg.det(R) - 1.0) < 1e-14


def test_rotated_covariance_recovers_its_scales_and_axes():
    Q = rot(0.3, -0.7, 1.1)
    s = np.array([0.5, 0.2, 0.1])
    S, R, _ = cov_decompose(pack(Q @ np.diag(s * s) @ Q.T))
    R = R[:, :, 0]
    assert np.allclose(S[:, 0], s, rtol=1e-12)
    for k in range(3):  # each axis up to sign
        assert min(np.abs(R[:, k] - Q[:, k]).max(), np.abs(R[:, k] + Q[:, k]).max()) < 1e-12
    assert abs(np.linalg.det(R) - 1.0) < 1e-12
    assert np.allclose(R @ np.diag(S[:, 0] ** 2) @ R.T, Q @ np.diag(s * s) @ Q.T, atol=1e-14)


def test_split_decisions_on_hand_built_factors():
    def packed(entries):
        Lp = np.zeros((28, 1))
        for (i, j), v in entries.items():
            Lp[i * (i + 1) // 2 + j, 0] = v
        return Lp
    base = {(k, k): 1.0 for k in range(7)}
    # Sigma_xt = L00 L30 = 0.3; Sigma_t = 0.3^2 + 1: split at extent 1
    a = packed({**base, (3, 0): 0.3})
    split, m1, m2 = split_test(a, extent=1.0)
    assert split[0] and abs(m1[0] - 0.25) < 1e-15 and abs(m2[0] - (np.sqrt(1.09) - 0.25)) < 1e-15
    # the same coupling against a 10x larger extent: not split (0.3 < 0.5)
    assert not split_test(a, extent=10.0)[0][0]
    # narrow in time (Sigma_t = 0.01 + 0.2^2 -> sqrt = 0.2236 < 0.25): not split
    b = packed({**base, (3, 3): 0.1, (3, 1): 0.2})
    split, m1, m2 = split_test(b, extent=1.0)
    assert not split[0] and m1[0] > 0 and m2[0] < 0
    # and the time span normalizes the temporal scale: over a 0.5-long range it splits
    assert split_test(b, extent=1.0, time_span=0.5)[0][0]
