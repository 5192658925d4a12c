"""The paths of calls with few Gaussians or few tiles.

* Frames of at most 2,048 Gaussians take a one-block depth sort: its order,
  pairs and ranges equal a CPU re-execution of the integer stage on the GPU's
  own keys (Sec. 4.4 sorting; ties to the smaller index), on both sides of
  the 2,048 boundary and in calls of several such frames.
* Calls of at most 256 tiles composite each band of a tile in a wave of its
  own: the image, final T and last equal, bit for bit, those of the
  four-band kernel (the contributor-count pass runs it on the same pairs),
  and the image equals the FP64 oracle's within the image bar.
GPU only."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_helpers import cpu_bin, flag_cap, image_check

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


SORT_CASES = {  # (Gaussians, W, H, views): one block per frame up to 2,048
    "n2048_128x96": (2048, 128, 96, 1),
    "n2049_128x96": (2049, 128, 96, 1),
    "n1000_64x64_x3": (1000, 64, 64, 3),
    "n2048_288x256": (2048, 288, 256, 1),  # 288 tiles: the four-band kernel
}


@pytest.mark.parametrize("case", list(SORT_CASES))
def test_small_sort_is_bitexact(R, case):
    n, W, H, nv = SORT_CASES[case]
    seed = 500 + list(SORT_CASES).index(case)
    scene = scenegen.make_scene(n, seed, sigma_off=0.15)
    views = scenegen.make_views(nv, seed, r=3.0, W=W, H=H, bg=(0.2, 0.5, 1.0))
    print(f"[small_sort] {case}", flush=True)
    gs = _gs(scene)
    b = R.render_frames(R.make_frames([(gs, v) for v in views]))
    torch.cuda.synchronize()
    counts = b.counts().cpu().numpy()
    tiles_x, tiles_y = (W + 15) // 16, (H + 15) // 16
    for f in range(nv):
        dk = b.depth_key(f).cpu().numpy().view(np.uint32)
        rect = b.rect(f).cpu().numpy().view(np.uint32)
        order, tile, g, ranges = cpu_bin(dk, rect, tiles_x, tiles_x * tiles_y)
        kept = int(counts[f, 0])
        assert kept == len(order) and kept > 0
        assert np.array_equal(b.order(f).cpu().numpy()[:kept], order), f
        t_gpu, g_gpu, base = b.pairs(f, counts)
        assert np.array_equal(t_gpu.cpu().numpy(), tile), f
        assert np.array_equal(g_gpu.cpu().numpy(), g), f
        rg = b.ranges(f).cpu().numpy().astype(np.int64)
        nonempty = ranges[:, 1] > ranges[:, 0]
        assert np.array_equal(rg[nonempty] - base, ranges[nonempty]), f


BAND_CASES = {  # calls of at most 256 tiles
    "c0": lambda: scenegen.config0(0.05),
    "ragged_37x23": lambda: (scenegen.make_scene(3000, 7, h=1.0, sigma_off=0.1),
                             scenegen.make_views(1, 7, r=3.0, W=37, H=23)),
    "corr015_128x72": lambda: (scenegen.make_scene(5000, 9, sigma_off=0.15),
                               scenegen.make_views(1, 9, r=3.0, W=128, H=72)),
    "x3_64x64": lambda: (scenegen.make_scene(1500, 12, sigma_off=0.1),
                         scenegen.make_views(3, 12, r=3.0, W=64, H=64, bg=(0.1, 0.2, 0.3))),
    "256_tiles": lambda: (scenegen.make_scene(6000, 13, sigma_off=0.1),
                          scenegen.make_views(1, 13, r=3.0, W=256, H=256)),
}


@pytest.mark.parametrize("case", list(BAND_CASES))
def test_band_waves_match_four_band_waves_and_oracle(R, case, report):
    scene, views = BAND_CASES[case]()
    print(f"[band_waves] {case}", flush=True)
    gs = _gs(scene)
    items = [(gs, v) for v in views]
    a = R.render_frames(R.make_frames(items))                # a wave per band
    c = R.render_frames(R.make_frames(items, count=True))    # the four-band kernel
    torch.cuda.synchronize()
    for fa, fc in zip(a.frames, c.frames):
        for k in ("image", "final_T", "last"):
            assert torch.equal(getattr(fa, k), getattr(fc, k)), (case, k)
    v = views[0]
    ora = oracle.render(scene, v)
    err, nflag = image_check(a.frames[0].image.cpu().numpy(), ora)
    report("band_waves", case=case, max_err=err, flagged=nflag, pixels=v.W * v.H)
    assert err <= 1e-4
    assert nflag <= flag_cap(v.W * v.H)
