"""Parity at the full workload sizes, in the launch configuration the benchmark
times (the first batch of a step: 25 of the 50 views of 800x800 over 200,000
Gaussians, in one set of launches), checked on
outputs the oracle can compute at this size: the whole slice, the integer
stage re-executed on the CPU, and sampled pixel crops of the image.  Also the
full variant with adaptive refinement in the same launch configuration, the
training workload (500,000 Gaussians at 1352x1014, forward + backward with the
upstream gradient restricted to a crop) and the ill-conditioned 4M-Gaussian
1080p stress scene."""
import numpy as np
import pytest

import oracle
import oracle.grad as og
import scenegen
from tests.gpu_helpers import (AGR_FLAGS, check_gradients, cpu_bin, flag_cap, footprint_rows, image_check,
                               splat_grads, slice_tolerance)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


@pytest.fixture(scope="module")
def c1():
    scene, views = scenegen.config1(50)
    return scene, views[:25]


@pytest.fixture(scope="module")
def c1_batch(R, c1):
    from paper_2503_07946_amd.render import GaussianScene
    scene, views = c1
    gs = GaussianScene.from_host(scene)
    print("[fullsize] 200k Gaussians, batch of 25 x 800x800", flush=True)
    b = R.render_frames(R.make_frames([(gs, v) for v in views], keep_sliced=True))
    torch.cuda.synchronize()
    return b


def test_c1_slice_all_gaussians(R, c1, c1_batch):
    scene, views = c1
    for f in (0, 24):
        ora = oracle.slice_(scene, views[f])
        mu = c1_batch.mu_c(f).cpu().numpy().astype(np.float64)
        cov = c1_batch.cov_c(f).cpu().numpy().astype(np.float64)
        ac = c1_batch.alpha_c(f).cpu().numpy().astype(np.float64)
        mscale = np.maximum(np.abs(ora.mu_c).max(0), np.abs(scene.mu_p).max(0))
        assert np.all(np.abs(mu - ora.mu_c) <= slice_tolerance(ora.mu_c, mscale))
        assert np.all(np.abs(cov - ora.cov_c) <= slice_tolerance(ora.cov_c, np.abs(ora.cov_c).max(0)))
        assert np.all(np.abs(ac - ora.alpha_c) <= slice_tolerance(ora.alpha_c, ora.alpha_c))


def test_c1_integer_stage_bitexact(R, c1, c1_batch, report):
    scene, views = c1
    counts = c1_batch.counts().cpu().numpy()
    for f in (0, 24):
        v = views[f]
        dk = c1_batch.depth_key(f).cpu().numpy().view(np.uint32)
        rect = c1_batch.rect(f).cpu().numpy().view(np.uint32)
        order, tile, g, ranges = cpu_bin(dk, rect, 50, 2500)
        kept = int(counts[f, 0])
        assert kept == len(order)
        assert np.array_equal(c1_batch.order(f).cpu().numpy()[:kept], order)
        t_gpu, g_gpu, base = c1_batch.pairs(f, counts)
        assert np.array_equal(t_gpu.cpu().numpy(), tile)
        assert np.array_equal(g_gpu.cpu().numpy(), g)
        rg = c1_batch.ranges(f).cpu().numpy().astype(np.int64)
        ne = ranges[:, 1] > ranges[:, 0]
        assert np.array_equal(rg[ne] - base, ranges[ne])
        report("c1_bin", frame=f, kept=kept, pairs=len(tile))


def test_c1_sampled_crops(R, c1, c1_batch, report):
    scene, views = c1
    rng = np.random.default_rng(11)
    for f in (0, 13):
        v = views[f]
        img = c1_batch.frames[f].image.cpu().numpy()
        for _ in range(2):
            x0, y0 = int(rng.integers(0, 800 - 32)), int(rng.integers(0, 800 - 32))
            crop = (x0, y0, 32, 32)
            ora = oracle.render(scene, v, crop=crop)
            err, nflag = image_check(img[:, y0:y0 + 32, x0:x0 + 32], ora)
            report("c1_crop", frame=f, crop=crop, max_err=err, flagged=nflag)
            assert err <= 1e-4
            assert nflag <= flag_cap(32 * 32)
        # the centre crop, where the tile lists are longest
        crop = (384, 384, 32, 32)
        ora = oracle.render(scene, v, crop=crop)
        err, nflag = image_check(img[:, 384:416, 384:416], ora)
        report("c1_crop", frame=f, crop=crop, max_err=err, flagged=nflag)
        assert err <= 1e-4
        assert nflag <= flag_cap(32 * 32)


def test_c1_agr_batch_slice_and_crop(R, c1, report):
    """The full variant with adaptive refinement in the benchmark's launch
    configuration (the same 25 views, the 200,000 Gaussians refined with
    scenegen.agr_weights(1)): the sliced statistics of every Gaussian of the
    batch's last frame and the centre crop of its first, against the FP64
    oracle with the refinement's tolerances."""
    from paper_2503_07946_amd.render import GaussianScene
    from tests.test_gpu_agr import AGR_REL, EPS_MU, log_alpha_sensitivity
    scene, views = c1
    w = scenegen.agr_weights(1)
    gs = GaussianScene.from_host(scene, agr=w)
    print("[fullsize] AGR: 200k Gaussians, batch of 25 x 800x800", flush=True)
    b = R.render_frames(R.make_frames([(gs, v) for v in views], keep_sliced=True))
    torch.cuda.synchronize()
    f = len(views) - 1
    v = views[f]
    ora = oracle.slice_(scene, v, agr_weights=w)
    ref = oracle.agr(scene, v.t, w)
    ok = ora.status == 0
    assert ok.mean() > 0.5
    mscale = np.maximum(np.abs(ora.mu_c).max(0), np.abs(ref.mu_p).max(0))
    cscale = np.abs(ora.cov_c).max(0)
    mu = b.mu_c(f).cpu().numpy().astype(np.float64)
    cov = b.cov_c(f).cpu().numpy().astype(np.float64)
    ac = b.alpha_c(f).cpu().numpy().astype(np.float64)
    tol_mu = np.maximum(slice_tolerance(ora.mu_c, mscale), AGR_REL * mscale)
    tol_cv = np.maximum(slice_tolerance(ora.cov_c, cscale), AGR_REL * cscale)
    tol_ac = np.maximum(slice_tolerance(ora.alpha_c, ora.alpha_c),
                        (AGR_REL + EPS_MU * log_alpha_sensitivity(ref, v)) * ora.alpha_c)
    e_mu = (np.abs(mu - ora.mu_c) / np.maximum(mscale, 1e-30))[:, ok].max()
    e_cv = (np.abs(cov - ora.cov_c) / np.maximum(cscale, 1e-30))[:, ok].max()
    e_ac = (np.abs(ac - ora.alpha_c) / np.maximum(ora.alpha_c, 1e-30))[ok].max()
    report("c1_agr_slice", frame=f, mu_rel=float(e_mu), cov_rel=float(e_cv), alpha_rel=float(e_ac))
    assert np.all(np.abs(mu - ora.mu_c)[:, ok] <= tol_mu[:, ok]), e_mu
    assert np.all(np.abs(cov - ora.cov_c)[:, ok] <= tol_cv[:, ok]), e_cv
    assert np.all(np.abs(ac - ora.alpha_c)[ok] <= tol_ac[ok]), e_ac
    crop = (384, 384, 32, 32)
    img = b.frames[0].image.cpu().numpy()
    o = oracle.render(scene, views[0], crop=crop, agr_weights=w, flags=AGR_FLAGS)
    err, nflag = image_check(img[:, 384:416, 384:416], o)
    report("c1_agr_crop", frame=0, crop=crop, max_err=err, flagged=nflag)
    assert err <= 1e-4


def test_c2_training_step_crop_gradients(R, report):
    """500,000 Gaussians at 1352x1014; L1 loss gradient kept on a 32x32 crop;
    every Gaussian's gradient compared with the FP64 reference."""
    from paper_2503_07946_amd.render import GaussianScene
    scene, views, target = scenegen.config2()
    v = views[0]
    gs = GaussianScene.from_host(scene)
    print("[fullsize] c2 forward", flush=True)
    b = R.render(gs, v)
    img = b.frames[0].image.cpu().numpy()
    x0, y0 = 660, 490
    crop = (x0, y0, 32, 32)
    ora = oracle.render(scene, v, crop=crop)
    err, nflag = image_check(img[:, y0:y0 + 32, x0:x0 + 32], ora)
    assert err <= 1e-4
    assert nflag <= flag_cap(32 * 32)
    dL = np.zeros_like(img)
    sub = og.l1_grad_image(img[:, y0:y0 + 32, x0:x0 + 32].astype(np.float64), target[:, y0:y0 + 32, x0:x0 + 32])
    dL[:, y0:y0 + 32, x0:x0 + 32] = sub * (ora.fbound == 0)[None]
    print("[fullsize] c2 backward", flush=True)
    g = R.backward(b, [torch.as_tensor(dL, device="cuda")])[0]
    torch.cuda.synchronize()
    d_crop = dL[:, y0:y0 + 32, x0:x0 + 32].astype(np.float64)
    g_ora, _ = og.grad(scene, v, d_crop, crop=crop)
    d_ora = og.grad_splats(scene, v, d_crop, crop=crop)
    g_gpu = {k: g[k].cpu().numpy() for k in og.PARAMS}
    rep = check_gradients(g_gpu, splat_grads(b, 0), g_ora, d_ora, og.splat_jacobian(scene, v))
    report("c2_grad", max_err=err, flagged=nflag, masked_pixels=int((ora.fbound > 0).sum()), **rep)


@pytest.fixture(scope="module")
def c4():
    print("[fullsize] generating the 4M stress scene (64 views of 1920x1080)", flush=True)
    return scenegen.config4()


def test_c4_slice_and_integer_stage(R, c4, report):
    """4,000,000 Gaussians with (t, d) blocks of condition number up to 1e4,
    1920x1080: slice on a sample of Gaussians, and the integer stage (kept
    count, pair count, sampled tile lists) of view 0."""
    from paper_2503_07946_amd.render import GaussianScene
    scene, views, _ = c4
    v = views[0]
    gs = GaussianScene.from_host(scene)
    print("[fullsize] c4 render", flush=True)
    b = R.render(gs, v)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(scene.n, 200_000, replace=False)
    sub = scene.subset(idx)
    ora = oracle.slice_(sub, v)
    mu = b.mu_c().cpu().numpy()[:, idx].astype(np.float64)
    cov = b.cov_c().cpu().numpy()[:, idx].astype(np.float64)
    mscale = np.maximum(np.abs(ora.mu_c).max(0), np.abs(sub.mu_p).max(0))
    assert np.all(np.abs(mu - ora.mu_c) <= slice_tolerance(ora.mu_c, mscale))
    assert np.all(np.abs(cov - ora.cov_c) <= slice_tolerance(ora.cov_c, np.abs(ora.cov_c).max(0)))
    counts = b.counts().cpu().numpy()
    dk = b.depth_key().cpu().numpy().view(np.uint32)
    rect = b.rect().cpu().numpy().view(np.uint32)
    kept = dk != 0xFFFFFFFF
    rect[~kept] = 0   # culled Gaussians have no footprint
    gi, ry, ra, rb = footprint_rows(rect)
    live = kept[gi] & (rb > ra)
    gi, ry, ra, rb = gi[live], ry[live], ra[live], rb[live]
    assert int(counts[0, 0]) == int(kept.sum())
    assert int(counts[0, 1]) == int((rb - ra).sum())
    # sampled tiles: the list is every kept Gaussian whose footprint holds the
    # tile, in (depth key, index) order
    rg = b.ranges(0).cpu().numpy().astype(np.int64)
    pg = b.ws[b.layout.off_pair_g:].view(torch.int32)
    for t in np.random.default_rng(1).choice(120 * 68, 48, replace=False):
        tx, ty = t % 120, t // 120
        cand = gi[(ry == ty) & (ra <= tx) & (tx < rb)]
        ref = cand[np.lexsort((cand, dk[cand]))]
        got = pg[rg[t, 0]:rg[t, 1]].cpu().numpy() if rg[t, 1] > rg[t, 0] else np.array([], np.int64)
        assert np.array_equal(got, ref), f"tile {t}"
    report("c4_bin", kept=int(counts[0, 0]), pairs=int(counts[0, 1]))


C4_CROP = (928, 508, 64, 64)   # the 64x64 centre crop of a 1920x1080 view
C4_INFLIGHT = 8                # views resident at once


def test_c4_64_views_forward_backward_and_centre_crops(R, c4, report):
    """The stress configuration as a whole: 64 views of 1920x1080 over the
    4M-Gaussian scene, rendered C4_INFLIGHT at a time, each followed by a full
    backward pass (L1 loss against the seeded target over the whole image).
    Views 0-3 are checked against the FP64 oracle on the centre crop: the
    image, and every gradient with the upstream gradient restricted to the
    crop.  The oracle takes the Gaussians whose FP64 opacity box comes within
    a pixel of the crop; every other Gaussian is below 1/255 at every crop
    pixel, adds nothing to the crop and has zero gradient, which the GPU's
    gradients must show as exact zeros."""
    from paper_2503_07946_amd.render import GaussianScene
    scene, views, target = c4
    x0, y0, cw, ch = C4_CROP
    gs = GaussianScene.from_host(scene)
    tgt = torch.as_tensor(target, device="cuda")
    checked = 0
    pairs = []
    for s0 in range(0, len(views), C4_INFLIGHT):
        vb = views[s0:s0 + C4_INFLIGHT]
        print(f"[fullsize] c4 views {s0}..{s0 + len(vb) - 1}: forward", flush=True)
        b = R.render_frames(R.make_frames([(gs, v) for v in vb], keep_sliced=True))
        c = b.counts().cpu().numpy()
        assert not np.any(c[:, 3] & 4), "pair arena overflow"
        pairs += c[:, 1].tolist()
        for f in range(len(vb)):
            k = s0 + f
            if k >= 4:
                continue
            v = vb[f]
            img = b.frames[f].image.cpu().numpy()
            sl = oracle.slice_(scene, v)
            pr = oracle.project(sl, scene.sh, v)
            near = pr.visible & (pr.box[2] >= x0 - 1) & (pr.box[0] <= x0 + cw + 1) & \
                (pr.box[3] >= y0 - 1) & (pr.box[1] <= y0 + ch + 1)
            sel = np.nonzero(near)[0]
            sub = scene.subset(sel)
            o = oracle.render(sub, v, crop=C4_CROP)
            err, nflag = image_check(img[:, y0:y0 + ch, x0:x0 + cw], o)
            assert err <= 1e-4, (k, err)
            assert nflag <= flag_cap(cw * ch), (k, nflag)
            # gradients with the upstream gradient on the crop only
            dL = np.zeros_like(img)
            dsub = og.l1_grad_image(img[:, y0:y0 + ch, x0:x0 + cw].astype(np.float64),
                                    target[:, y0:y0 + ch, x0:x0 + cw]) * (o.fbound == 0)[None]
            dL[:, y0:y0 + ch, x0:x0 + cw] = dsub
            dls = [torch.zeros_like(fr.image) for fr in b.frames]
            dls[f] = torch.as_tensor(dL, device="cuda")
            print(f"[fullsize] c4 view {k}: crop backward", flush=True)
            g = R.backward(b, dls)[f]
            torch.cuda.synchronize()
            g_ora, _ = og.grad(sub, v, dsub.astype(np.float64), crop=C4_CROP)
            d_ora = og.grad_splats(sub, v, dsub.astype(np.float64), crop=C4_CROP)
            sel_t = torch.as_tensor(sel, device="cuda")
            others = torch.ones(scene.n, dtype=torch.bool, device="cuda")
            others[sel_t] = False
            g_sub = {}
            for name in og.PARAMS:
                ga = g[name].reshape(-1, scene.n)
                g_sub[name] = ga[:, sel_t].cpu().numpy()
                assert bool((ga[:, others] == 0).all()), (k, name, "gradient outside the crop's Gaussians")
            d_gpu = splat_grads(b, f)[:, sel]
            rep = check_gradients(g_sub, d_gpu, g_ora, d_ora, og.splat_jacobian(sub, v))
            report("c4_crop", view=k, crop=list(C4_CROP), gaussians_near=int(len(sel)), max_err=err,
                   flagged=nflag, **rep)
            checked += 1
        # the workload's backward: L1 over every pixel of every view
        print(f"[fullsize] c4 views {s0}..{s0 + len(vb) - 1}: full backward", flush=True)
        dls = [torch.sign(fr.image - tgt) / fr.image.numel() for fr in b.frames]
        gl = R.backward(b, dls)
        torch.cuda.synchronize()
        for gg in gl:
            for name in og.PARAMS:
                assert bool(torch.isfinite(gg[name]).all()), name
            assert float(gg["sh"].abs().max()) > 0.0
        del b, gl
    assert checked == 4
    report("c4_views", views=len(views), inflight=C4_INFLIGHT, pairs_mean=float(np.mean(pairs)))
