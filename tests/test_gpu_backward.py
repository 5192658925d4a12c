"""Gradients of the HIP backward (rasterize, project, slice reverse kernels)
against the FP64 autograd reference, and the autograd.Function wrapper."""
import numpy as np
import pytest

import oracle
import oracle.grad as og
import scenegen
from tests.gpu_helpers import check_gradients, splat_grads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GROUPS = ("mu_p", "mu_t", "mu_d", "L", "alpha", "sh")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


def _gpu_grad(R, scene, view, dL):
    from paper_2503_07946_amd.render import GaussianScene
    print(f"[backward] n={scene.n} {view.W}x{view.H}", flush=True)
    gs = GaussianScene.from_host(scene)
    b = R.render(gs, view)
    g = R.backward(b, [torch.as_tensor(dL, dtype=torch.float32, device="cuda")])[0]
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}, b


CASES = {
    "c0_random": lambda: (*scenegen.config0(0.05), None),
    "c0_l05": lambda: (*scenegen.config0(0.5), None),
    "train_subset_l1": lambda: ("l1",),
    "corr015_ragged": lambda: (scenegen.make_scene(3000, 19, sigma_off=0.15),
                               scenegen.make_views(1, 19, r=3.0, W=72, H=40, bg=(0.3, 0.2, 0.1)), None),
    "d_per_gaussian_lam03": lambda: (scenegen.make_scene(2500, 23, sigma_off=0.1),
                                     [v.replace(d_per_gaussian=True, lambda_t=0.3, lambda_d=0.2)
                                      for v in scenegen.make_views(1, 23, r=3.0, W=64, H=48)], None),
}


def _case(name):
    c = CASES[name]()
    if c[0] == "l1":
        sc, views, _ = scenegen.config2(n=2000)
        v0 = views[0]
        v = scenegen.make_view(v0.c, 64, 64, v0.t, d=v0.d, lambda_t=v0.lambda_t, lambda_d=v0.lambda_d)
        return sc, [v], "l1"
    return c


@pytest.mark.parametrize("case", list(CASES))
def test_gradients_match_oracle(R, case, report):
    scene, views, kind = _case(case)
    v = views[0]
    ora = oracle.render(scene, v)
    # no gradient through pixels where the oracle took a decision within FP32
    # reach of its threshold (the two sides may differ there by a contribution)
    mask = (ora.fbound == 0).astype(np.float64)
    if kind == "l1":
        target = scenegen.target_image(2002, v.W, v.H).astype(np.float64)
        dL = og.l1_grad_image(ora.image, target)
    else:
        dL = np.random.default_rng(7).normal(size=(3, v.H, v.W))
    dL = (dL * mask[None]).astype(np.float32)
    assert mask.mean() >= 0.99
    g_gpu, b = _gpu_grad(R, scene, v, dL)
    g_ora, _ = og.grad(scene, v, dL.astype(np.float64))
    lam_gpu, lam_ora = g_gpu.pop("lambda").astype(np.float64), g_ora.pop("lambda")
    lam_err = np.abs(lam_gpu - lam_ora) / np.maximum(np.abs(lam_ora), 1e-6 * np.abs(g_ora["alpha"]).sum())
    report("lambda_grad_parity", case=case, rel=lam_err.tolist(), gpu=lam_gpu.tolist(), oracle=lam_ora.tolist())
    assert np.all(lam_err <= 1e-3), (lam_gpu, lam_ora)
    d_ora = og.grad_splats(scene, v, dL.astype(np.float64))
    rep = check_gradients(g_gpu, splat_grads(b, 0), g_ora, d_ora, og.splat_jacobian(scene, v))
    report("grad_parity", case=case, masked_pixels=int((mask == 0).sum()), **rep)


def test_autograd_function_matches_library_backward(R):
    from paper_2503_07946_amd.render import render_image
    scene, views = scenegen.config0()
    v = views[0]
    params = {k: torch.as_tensor(getattr(scene, k)).cuda().requires_grad_(True) for k in GROUPS}
    img = render_image(params, v)
    target = torch.as_tensor(scenegen.target_image(5, v.W, v.H)).cuda()
    loss = (img - target).abs().mean()
    loss.backward()
    dL = torch.sign(img.detach() - target) / img.numel()
    g_gpu, _ = _gpu_grad(R, scene, v, dL.cpu().numpy())
    for k in GROUPS:
        a = params[k].grad.cpu().numpy()
        np.testing.assert_allclose(a, g_gpu[k], rtol=0, atol=1e-5 * np.abs(g_gpu[k]).max() + 1e-12)


def test_backward_is_deterministic_enough(R):
    """Float atomics reorder sums between runs; the gradients still agree to
    FP32 rounding of the accumulated values."""
    scene, views = scenegen.config0()
    dL = np.random.default_rng(3).normal(size=(3, 64, 64)).astype(np.float32)
    g1, _ = _gpu_grad(R, scene, views[0], dL)
    g2, _ = _gpu_grad(R, scene, views[0], dL)
    for k in GROUPS:
        s = np.abs(g1[k]).max()
        np.testing.assert_allclose(g1[k], g2[k], rtol=0, atol=1e-5 * s + 1e-12)
