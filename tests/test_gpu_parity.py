"""Parity of the HIP render path with the FP64 oracle (each stage and the
image), bit-exactness of the integer stage, and edge cases.  GPU only."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_helpers import (CULLED, cpu_bin, flag_cap, footprint_rows, image_check, oracle_rect_flags,
                               slice_tolerance, tile_reached)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


def _gs(scene):
    from paper_2503_07946_amd.render import GaussianScene
    return GaussianScene.from_host(scene)


def _render(R, scene, view, capacity=None):
    print(f"[render] n={scene.n} {view.W}x{view.H}", flush=True)
    b = R.render(_gs(scene), view, capacity=capacity)
    torch.cuda.synchronize()
    return b


CASES = {
    "c0_l005": lambda: scenegen.config0(0.05),
    "c0_l05": lambda: scenegen.config0(0.5),
    "ragged_37x23": lambda: (scenegen.make_scene(3000, 7, h=1.0, sigma_off=0.1),
                             scenegen.make_views(1, 7, r=3.0, W=37, H=23)),
    "cond_1e4_96x80": lambda: (scenegen.make_scene(4000, 8, recondition=True),
                               scenegen.make_views(1, 8, r=3.0, W=96, H=80, bg=(0.2, 0.3, 0.4))),
    "corr015_128x72": lambda: (scenegen.make_scene(5000, 9, sigma_off=0.15),
                               scenegen.make_views(1, 9, r=3.0, W=128, H=72)),
    "d_per_gaussian_80x56": lambda: (scenegen.make_scene(4000, 10, sigma_off=0.1),
                                     [v.replace(d_per_gaussian=True)
                                      for v in scenegen.make_views(1, 10, r=3.0, W=80, H=56)]),
}


@pytest.mark.parametrize("case", list(CASES))
def test_slice_parity(R, case):
    scene, views = CASES[case]()
    v = views[0]
    b = _render(R, scene, v)
    ora = oracle.slice_(scene, v)
    mu = b.mu_c().cpu().numpy().astype(np.float64)
    cov = b.cov_c().cpu().numpy().astype(np.float64)
    ac = b.alpha_c().cpu().numpy().astype(np.float64)
    ok = ora.status == 0
    mscale = np.maximum(np.abs(ora.mu_c).max(0), np.abs(scene.mu_p).max(0))
    cscale = np.abs(ora.cov_c).max(0)
    assert np.all(np.abs(mu - ora.mu_c)[:, ok] <= slice_tolerance(ora.mu_c, mscale)[:, ok])
    assert np.all(np.abs(cov - ora.cov_c)[:, ok] <= slice_tolerance(ora.cov_c, cscale)[:, ok])
    assert np.all(np.abs(ac - ora.alpha_c)[ok] <= slice_tolerance(ora.alpha_c, ora.alpha_c)[ok])


@pytest.mark.parametrize("case", list(CASES))
def test_project_parity(R, case):
    scene, views = CASES[case]()
    v = views[0]
    b = _render(R, scene, v)
    sl = oracle.slice_(scene, v)
    pr = oracle.project(sl, scene.sh, v)
    flag = oracle_rect_flags(sl, pr, v)
    dk = b.depth_key().cpu().numpy().view(np.uint32)
    gvis = dk != CULLED
    assert np.array_equal(gvis[~flag], pr.visible[~flag])
    rect = b.rect().cpu().numpy().view(np.uint32)
    both = gvis & pr.visible & ~flag
    g_rect = np.stack([rect[:, 0] & 0xFFFF, rect[:, 0] >> 16, rect[:, 1] & 0xFFFF, rect[:, 1] >> 16])
    assert np.array_equal(g_rect[:, both], pr.rect[:, both].astype(np.uint32))
    sp = b.splat().cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(sp[both, 0:2].T, pr.mean2d[:, both], rtol=2e-6, atol=2e-4)
    cscale = np.maximum(np.abs(pr.conic[0]), np.abs(pr.conic[2]))[both]
    # the record stores the exponent coefficients -log2(e) (a/2, b, c/2) and log2(alpha_c)
    log2e = 1.4426950408889634
    conic = sp[both, 2:5].T / np.array([[-0.5 * log2e], [-log2e], [-0.5 * log2e]])
    assert np.all(np.abs(conic - pr.conic[:, both]) <= 2e-4 * cscale[None, :] + 1e-9)
    np.testing.assert_allclose(sp[both, 10], sl.alpha_c[both], rtol=1e-6)
    np.testing.assert_allclose(2.0 ** sp[both, 5], sl.alpha_c[both], rtol=2e-6)
    np.testing.assert_allclose(sp[both, 6:9].T, pr.rgb[:, both], atol=2e-6)
    np.testing.assert_allclose(sp[both, 11], pr.depth[both], rtol=1e-6)
    assert np.array_equal(sp[both, 9], 16.0 * sp[both, 4])  # the band step's coefficient


@pytest.mark.parametrize("case", list(CASES))
def test_footprint_holds_every_reached_tile(R, case, report):
    """A tile dropped from a Gaussian's tile box holds no pixel centre where the
    oracle's opacity alpha_c exp(-q/2) reaches 1/255, so the trimmed tile lists
    lose no contribution; and the trims do drop tiles."""
    scene, views = CASES[case]()
    v = views[0]
    b = _render(R, scene, v)
    sl = oracle.slice_(scene, v)
    pr = oracle.project(sl, scene.sh, v)
    flag = oracle_rect_flags(sl, pr, v)
    dk = b.depth_key().cpu().numpy().view(np.uint32)
    rect = b.rect().cpu().numpy().view(np.uint32)
    use = (dk != CULLED) & pr.visible & ~flag
    rect[dk == CULLED] = 0   # culled Gaussians have no footprint
    gi, ty, a, bb = footprint_rows(rect)
    sel = use[gi]
    gi, ty, a, bb = gi[sel], ty[sel], a[sel], bb[sel]
    x0 = (rect[:, 0] & 0xFFFF).astype(np.int64)
    w = (rect[:, 1] & 0xFFFF).astype(np.int64) - x0
    wr = w[gi]
    rep = np.repeat(np.arange(len(gi)), wr)
    tx = x0[gi][rep] + np.arange(int(wr.sum())) - np.repeat(np.cumsum(wr) - wr, wr)
    g, yy = gi[rep], ty[rep]
    in_fp = (tx >= a[rep]) & (tx < bb[rep])
    reached = tile_reached(sl, pr, v, g, tx, yy)
    assert not np.any(reached & ~in_fp), int((reached & ~in_fp).sum())
    dropped = int((~in_fp).sum())
    report(f"footprint_{case}", box_tiles=len(g), dropped=dropped, unreached=int((~reached).sum()))
    assert dropped > 0 or len(g) < 2000


@pytest.mark.parametrize("case", list(CASES))
def test_bin_bitexact_on_gpu_keys(R, case):
    """X15: the GPU's order, pairs and ranges equal a CPU re-execution of the
    integer stage on the GPU's own depth keys and tile boxes, bit for bit."""
    scene, views = CASES[case]()
    v = views[0]
    b = _render(R, scene, v)
    counts = b.counts().cpu().numpy()
    dk = b.depth_key().cpu().numpy().view(np.uint32)
    rect = b.rect().cpu().numpy().view(np.uint32)
    tiles_x, tiles_y = (v.W + 15) // 16, (v.H + 15) // 16
    order, tile, g, ranges = cpu_bin(dk, rect, tiles_x, tiles_x * tiles_y)
    kept = int(counts[0, 0])
    assert kept == len(order)
    assert np.array_equal(b.order().cpu().numpy()[:kept], order)
    t_gpu, g_gpu, base = b.pairs(0, counts)
    assert int(counts[0, 1]) == len(tile)
    assert np.array_equal(t_gpu.cpu().numpy(), tile)
    assert np.array_equal(g_gpu.cpu().numpy(), g)
    rg = b.ranges(0).cpu().numpy().astype(np.int64)
    nonempty = ranges[:, 1] > ranges[:, 0]
    assert np.array_equal(rg[nonempty] - base, ranges[nonempty])
    assert np.all(rg[~nonempty, 0] == rg[~nonempty, 1])


@pytest.mark.parametrize("case", list(CASES))
def test_tile_lists_match_oracle(R, case):
    """X16: per-tile lists against the FP64 oracle's (every Gaussian whose tile
    box covers the tile), except Gaussians flagged as within rounding of a
    visibility or tile-edge decision: the GPU list holds every Gaussian of the
    oracle's list that reaches alpha >= 1/255 in the tile and nothing outside
    the oracle's list (the footprint drops only tiles a splat cannot reach);
    order compared on Gaussians with distinct FP32 depths."""
    scene, views = CASES[case]()
    v = views[0]
    b = _render(R, scene, v)
    sl = oracle.slice_(scene, v)
    pr = oracle.project(sl, scene.sh, v)
    flag = oracle_rect_flags(sl, pr, v)
    ora_lists = oracle.tile_lists(pr, v)
    counts = b.counts().cpu().numpy()
    t_gpu, g_gpu, _ = b.pairs(0, counts)
    t_gpu, g_gpu = t_gpu.cpu().numpy(), g_gpu.cpu().numpy()
    z32 = pr.depth.astype(np.float32)
    ntiles = ((v.W + 15) // 16) * ((v.H + 15) // 16)
    tx_ = (v.W + 15) // 16
    for t in range(ntiles):
        gl = [x for x in g_gpu[t_gpu == t] if not flag[x]]
        ol = [x for x in ora_lists.get(t, []) if not flag[x]]
        assert set(gl) <= set(ol), f"tile {t}"
        oa = np.array(ol, np.int64)
        must = oa[tile_reached(sl, pr, v, oa, np.full(len(oa), t % tx_), np.full(len(oa), t // tx_))]
        assert set(must.tolist()) <= set(gl), f"tile {t}"
        ol = [x for x in ol if x in set(gl)]
        # order: compare after removing Gaussians that tie in FP32 depth with a neighbour
        zs = z32[np.array(ol, dtype=np.int64)] if ol else np.array([], np.float32)
        tie = np.zeros(len(ol), bool)
        if len(ol) > 1:
            close = np.abs(np.diff(zs.astype(np.float64))) <= 8 * np.spacing(np.abs(zs[1:]))
            tie[1:] |= close
            tie[:-1] |= close
        keep = set(np.array(ol)[~tie].tolist())
        assert [x for x in gl if x in keep] == [x for x in ol if x in keep], f"tile {t}"


@pytest.mark.parametrize("case", list(CASES))
def test_image_parity(R, case, report):
    """X14: the tiled FP32 image equals the brute-force FP64 image within 1e-4
    on every unflagged pixel."""
    scene, views = CASES[case]()
    v = views[0]
    print(f"[render] n={scene.n} {v.W}x{v.H} with contributor counts", flush=True)
    b = R.render(_gs(scene), v, count=True)
    torch.cuda.synchronize()
    ora = oracle.render(scene, v)
    img = b.frames[0].image.cpu().numpy()
    err, nflag = image_check(img, ora)
    report("image_parity", case=case, max_err=err, flagged=nflag, pixels=v.W * v.H,
           events=int((ora.fbound > 0).sum()))
    assert err <= 1e-4
    T = b.frames[0].final_T.cpu().numpy().astype(np.float64)
    mask = ora.fbound == 0
    assert np.abs(T - ora.final_T)[mask].max() <= 1e-4
    assert nflag <= flag_cap(v.W * v.H)
    if case.startswith("c0"):
        assert nflag == 0   # the small workload: no decision within FP32 reach
    # the contributor set itself: counts equal wherever no decision is within
    # FP32 rounding of its threshold (no impact filter here)
    strict = oracle.render(scene, v, flags={"impact_min": 0.0})
    m0 = strict.flags == 0
    nc = b.frames[0].ncontrib.cpu().numpy()
    assert np.array_equal(nc[m0], strict.ncontrib[m0])


def test_radix_binner_for_frames_above_32768_tiles(R, report):
    """A 2912x2912 frame has 182 x 182 = 33,124 tiles, beyond the counting
    binner's LDS budget: binning falls back to the radix tile sort, which must
    give the same bit-exact lists and an oracle-matching image."""
    scene = scenegen.make_scene(20000, 17, h=1.0, sigma_off=0.1)
    v = scenegen.make_views(1, 17, r=3.0, W=2912, H=2912)[0]
    b = _render(R, scene, v)
    counts = b.counts().cpu().numpy()
    dk = b.depth_key().cpu().numpy().view(np.uint32)
    rect = b.rect().cpu().numpy().view(np.uint32)
    order, tile, g, ranges = cpu_bin(dk, rect, 182, 182 * 182)
    t_gpu, g_gpu, base = b.pairs(0, counts)
    assert np.array_equal(t_gpu.cpu().numpy(), tile)
    assert np.array_equal(g_gpu.cpu().numpy(), g)
    img = b.frames[0].image.cpu().numpy()
    crop = (1440, 1440, 32, 32)
    ora = oracle.render(scene, v, crop=crop)
    err, nflag = image_check(img[:, 1440:1472, 1440:1472], ora)
    report("radix_fallback", pairs=int(counts[0, 1]), max_err=err, flagged=nflag)
    assert err <= 1e-4
    assert nflag <= flag_cap(32 * 32)


def test_empty_and_transparent_scenes(R):
    from paper_2503_07946_amd.render import GaussianScene
    v = scenegen.make_views(1, 3, r=3.0, W=40, H=24, bg=(0.25, 0.5, 0.75))[0]
    empty = GaussianScene(*(torch.zeros((k, 0), device="cuda").reshape(-1) if k == 1 else
                            torch.zeros((k, 0), device="cuda") for k in (3, 1, 3, 28, 1, 48)))
    b = R.render(empty, v)
    torch.cuda.synchronize()
    img = b.frames[0].image.cpu().numpy()
    bg = np.array([0.25, 0.5, 0.75], np.float32)
    assert np.array_equal(img, np.broadcast_to(bg[:, None, None], img.shape))
    assert np.all(b.frames[0].final_T.cpu().numpy() == 1.0)
    assert np.all(b.frames[0].last.cpu().numpy() == 0)
    sc = scenegen.make_scene(500, 4)
    sc.alpha[:] = 1e-4
    b = _render(R, sc, v)
    img = b.frames[0].image.cpu().numpy()
    assert np.array_equal(img, np.broadcast_to(bg[:, None, None], img.shape))
    assert int(b.counts().cpu().numpy()[0, 0]) == 0


def test_one_pixel_image(R):
    scene, _ = scenegen.config0()
    v = scenegen.make_view([0.1, -3.0, 0.2], 1, 1, 0.5)
    b = _render(R, scene, v)
    ora = oracle.render(scene, v)
    err, nflag = image_check(b.frames[0].image.cpu().numpy(), ora)
    assert err <= 1e-4 or nflag == 1


def test_pair_overflow_flag_and_recovery(R):
    from paper_2503_07946_amd import _lib as L
    from paper_2503_07946_amd.render import GaussianScene
    scene, views = scenegen.config0()
    v = views[0]
    gs = GaussianScene.from_host(scene)
    fr = R.make_frames([(gs, v)])
    b = R.render_frames(fr, capacity=16, exact=False)
    c = R.read_counts(b)
    assert c[0, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW
    assert c[0, L.SD7_CNT_PAIRS] == 0 and c[0, L.SD7_CNT_NEEDED] > 16
    img = b.frames[0].image.cpu().numpy()
    assert np.all(img == 0.0)   # black background, nothing rasterized
    b2 = R.render_frames(R.make_frames([(gs, v)]), capacity=16, exact=True)
    c2 = R.read_counts(b2)
    assert not (c2[0, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW)
    ora = oracle.render(scene, v)
    err, _ = image_check(b2.frames[0].image.cpu().numpy(), ora)
    assert err <= 1e-4


def test_nonpositive_diagonal_is_flagged_and_culled(R):
    from paper_2503_07946_amd import _lib as L
    scene, views = scenegen.config0()
    bad = scene.subset(np.arange(scene.n))
    bad.L[scenegen.tri_index(4, 4), 10] = -0.05
    b = _render(R, bad, views[0])
    c = R.read_counts(b)
    assert c[0, L.SD7_CNT_FLAGS] & L.SD7_FLAG_NONPOS_DIAG
    assert b.depth_key().cpu().numpy().view(np.uint32)[10] == CULLED
    keep = np.r_[0:10, 11:scene.n]
    ora = oracle.render(scene.subset(keep), views[0])
    err, _ = image_check(b.frames[0].image.cpu().numpy(), ora)
    assert err <= 1e-4


def test_invalid_arguments_raise(R):
    from paper_2503_07946_amd import _lib as L
    scene, views = scenegen.config0()
    v = views[0].replace(W=0)
    with pytest.raises(L.Sd7Error):
        R.render(_gs(scene), v)
