"""Fused Adam step and pruning on the GPU against the oracle, and a short
synthetic training run (render, L1 loss, backward, Adam) that lowers the loss."""
import numpy as np
import pytest

import scenegen
from oracle.optim import GROUPS, adam_step, prune

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


def test_adam_steps_match_the_oracle(R, report):
    from paper_2503_07946_amd.render import Adam, GaussianScene
    sc = scenegen.make_scene(5000, 71)
    gs = GaussianScene.from_host(sc)
    opt = Adam(gs, eps=1e-8)
    rng = np.random.default_rng(72)
    p = {k: np.asarray(getattr(sc, k), np.float64) for k in GROUPS}
    m = {k: np.zeros_like(a) for k, a in p.items()}
    v = {k: np.zeros_like(a) for k, a in p.items()}
    worst = 0.0
    for t in range(1, 4):
        g = {k: rng.normal(0, 1e-2, a.shape).astype(np.float32) for k, a in p.items()}
        print(f"[optim] adam step {t}", flush=True)
        opt.step(gs, {k: torch.as_tensor(g[k]).cuda() for k in GROUPS})
        torch.cuda.synchronize()
        # the oracle continues from the GPU's FP32 state so rounding does not accumulate
        p_in = {k: np.asarray(a, np.float32).astype(np.float64) for k, a in p.items()}
        f32 = lambda x: float(np.float32(x))   # the library receives these in FP32
        P, M, V = adam_step(p_in, g, m, v, {k: f32(x) for k, x in opt.lr.items()}, t,
                            beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
        for k in GROUPS:
            gp = getattr(gs, k).cpu().numpy().astype(np.float64)
            err = np.abs(gp - P[k]).max() / max(np.abs(P[k]).max(), 1e-30)
            worst = max(worst, err)
            assert err <= 2e-6, (k, t, err)
            assert np.allclose(opt.m[k].cpu().numpy(), M[k], rtol=1e-5, atol=1e-9), k
            assert np.allclose(opt.v[k].cpu().numpy(), V[k], rtol=1e-5, atol=1e-12), k
            p[k] = gp
            m[k] = opt.m[k].cpu().numpy().astype(np.float64)
            v[k] = opt.v[k].cpu().numpy().astype(np.float64)
    report("adam_parity", rel=worst)


@pytest.mark.parametrize("n,tau", [(3000, 0.3), (1, 0.5), (2000, 2.0), (0, 0.01)])
def test_prune_matches_the_oracle(R, n, tau):
    from paper_2503_07946_amd.render import Adam, GaussianScene
    sc = scenegen.make_scene(max(n, 1), 73)
    if n == 0:
        gs = GaussianScene(*(torch.zeros((k, 0), device="cuda").reshape(-1) if k == 1 else
                             torch.zeros((k, 0), device="cuda") for k in (3, 1, 3, 28, 1, 48)))
    else:
        gs = GaussianScene.from_host(sc)
    opt = Adam(gs)
    for k in GROUPS:  # distinct moments so that their compaction is checked too
        opt.m[k].copy_(torch.rand_like(opt.m[k]))
        opt.v[k].copy_(torch.rand_like(opt.v[k]))
    before = {k: getattr(gs, k).cpu().numpy() for k in GROUPS}
    mb = {k: opt.m[k].cpu().numpy() for k in GROUPS}
    print(f"[optim] prune n={n} tau={tau}", flush=True)
    out = opt.prune(gs, tau)
    torch.cuda.synchronize()
    want = prune(before, before["alpha"], tau)
    assert out.n == (want["alpha"].shape[-1] if n else 0)
    for k in GROUPS:
        assert np.array_equal(getattr(out, k).cpu().numpy().reshape(want[k].shape), want[k]), k
    wm = prune(mb, before["alpha"], tau)
    for k in GROUPS:
        assert np.array_equal(opt.m[k].cpu().numpy().reshape(wm[k].shape), wm[k]), k


def test_short_training_run_lowers_the_loss(R, report):
    """Fit the means and colours of a perturbed copy of a scene to the scene's
    own render: 40 Adam steps of mean L1 must remove at least 30 % of it."""
    from paper_2503_07946_amd.render import Adam, GaussianScene
    sc = scenegen.make_scene(3000, 74, sigma_off=0.05)
    v = scenegen.make_views(1, 74, r=3.0, W=96, H=96)[0]
    target = R.render(GaussianScene.from_host(sc), v).frames[0].image.clone()
    rng = np.random.default_rng(75)
    noisy = scenegen.make_scene(3000, 74, sigma_off=0.05)
    noisy.mu_p += rng.normal(0, 0.02, noisy.mu_p.shape).astype(np.float32)
    noisy.sh += rng.normal(0, 0.1, noisy.sh.shape).astype(np.float32)
    gs = GaussianScene.from_host(noisy)
    opt = Adam(gs, lr={"mu_p": 2e-3, "sh": 1e-2, "L": 0.0, "alpha": 0.0, "mu_t": 0.0, "mu_d": 0.0})
    losses = []
    for it in range(40):
        b = R.render(gs, v)
        img = b.frames[0].image
        diff = img - target
        losses.append(float(diff.abs().mean()))
        dL = torch.sign(diff) / diff.numel()
        g = R.backward(b, [dL])[0]
        opt.step(gs, g)
    torch.cuda.synchronize()
    report("training_run", first=losses[0], last=losses[-1])
    print(f"[optim] L1 {losses[0]:.5f} -> {losses[-1]:.5f}", flush=True)
    assert losses[-1] < 0.7 * losses[0], losses
