"""Densification helpers on the GPU against the oracle: scale and rotation of
sliced covariances (scales to FP32 rounding; rotations up to the sign of
axes whose eigenvalue is well separated, always proper and reconstructing
Sigma), degenerate inputs, and the split test's decisions."""
import numpy as np
import pytest

import scenegen
from oracle.densify import cov_decompose as ora_decompose
from oracle.densify import split_test as ora_split

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


def _check(cov32, scale, rot, report=None, tag=""):
    S0, R0, w0 = ora_decompose(cov32.astype(np.float64))
    S = scale.astype(np.float64)
    Rg = rot.astype(np.float64).reshape(3, 3, -1)
    smax = np.maximum(S0[0], 1e-30)
    err_s = np.abs(S - S0).max(0) / smax
    assert np.all(err_s <= 1e-6), err_s.max()
    n = S.shape[1]
    RR = np.einsum("ikn,jkn->ijn", Rg, Rg)
    assert np.abs(RR - np.eye(3)[:, :, None]).max() <= 1e-6
    det = np.array([np.linalg.det(Rg[:, :, i]) for i in range(n)])
    assert np.all(np.abs(det - 1.0) <= 1e-5)
    # reconstruction of the (FP64-promoted) input
    A = np.einsum("ikn,kn,jkn->ijn", Rg, S * S, Rg)
    c = cov32.astype(np.float64)
    A0 = np.stack([np.stack([c[0], c[1], c[2]]), np.stack([c[1], c[3], c[4]]), np.stack([c[2], c[4], c[5]])])
    assert np.abs(A - A0).max(axis=(0, 1)).max() <= 1e-6 * np.abs(w0).max()
    # axes of well separated eigenvalues agree up to sign
    gap = np.minimum(np.abs(w0[0] - w0[1]), np.abs(w0[1] - w0[2])) / np.maximum(np.abs(w0[0]), 1e-30)
    for k in range(3):
        sep = np.ones(n, bool)
        if k == 0:
            sep = np.abs(w0[0] - w0[1]) > 1e-3 * np.abs(w0[0])
        elif k == 1:
            sep = gap > 1e-3
        else:
            sep = np.abs(w0[1] - w0[2]) > 1e-3 * np.abs(w0[0])
        d = np.minimum(np.abs(Rg[:, k] - R0[:, k]).max(0), np.abs(Rg[:, k] + R0[:, k]).max(0))
        assert np.all(d[sep] <= 1e-4), (k, d[sep].max())
    if report:
        report("cov_decompose_parity", case=tag, n=int(n), scale_rel=float(err_s.max()))


def test_decompose_sliced_covariances(R, report):
    from paper_2503_07946_amd.render import GaussianScene, cov_decompose
    sc = scenegen.make_scene(6000, 61, sigma_off=0.15)
    v = scenegen.make_views(1, 61, r=3.0, W=64, H=48)[0]
    b = R.render(GaussianScene.from_host(sc), v)
    cov = b.cov_c().contiguous()
    keep = b.alpha_c().cpu().numpy() > 0
    scale, rot = cov_decompose(cov)
    torch.cuda.synchronize()
    c = cov.cpu().numpy()[:, keep]
    _check(c, scale.cpu().numpy()[:, keep], rot.cpu().numpy()[:, keep], report, "sliced")


def test_decompose_known_rotations_and_degenerate_inputs(R, report):
    from paper_2503_07946_amd.render import cov_decompose
    rng = np.random.default_rng(62)
    n = 4096
    Q, _ = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    s = np.exp(rng.uniform(np.log(1e-3), np.log(1.0), size=(n, 3)))
    A = Q @ (s[:, :, None] ** 2 * np.transpose(Q, (0, 2, 1)))
    A[0] = np.eye(3) * 0.25                       # isotropic: any proper rotation is right
    A[1] = 0.0                                    # zero covariance
    A[2] = np.diag([1.0, 1.0, 1e-4])              # two equal eigenvalues
    c = np.stack([A[:, 0, 0], A[:, 0, 1], A[:, 0, 2], A[:, 1, 1], A[:, 1, 2], A[:, 2, 2]]).astype(np.float32)
    scale, rot = cov_decompose(torch.as_tensor(c).cuda())
    torch.cuda.synchronize()
    sc, rt = scale.cpu().numpy(), rot.cpu().numpy()
    assert np.allclose(sc[:, 0], 0.5, rtol=1e-6) and np.all(sc[:, 1] == 0.0)
    _check(c, sc, rt, report, "random_rotations")


def test_split_test_matches_the_oracle(R, report):
    from paper_2503_07946_amd.render import GaussianScene, split_mask
    for seed, sigma, extent in ((63, 0.15, 1.0), (64, 0.3, 0.5), (65, 0.05, 0.2)):
        sc = scenegen.make_scene(20000, seed, sigma_off=sigma)
        got = split_mask(GaussianScene.from_host(sc), extent).cpu().numpy()
        want, m1, m2 = ora_split(np.asarray(sc.L, np.float64), extent)
        sure = (np.abs(m1) > 1e-9 * extent) & (np.abs(m2) > 1e-9)
        report("split_test_parity", case=f"seed{seed}", n=int(sc.n), split=int(want.sum()),
               borderline=int((~sure).sum()))
        assert 0 < want.sum() < sc.n
        assert np.array_equal(got[sure], want[sure])
