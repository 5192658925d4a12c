"""The counting binner on frames of several tile groups, ragged at both edges,
with footprint boxes on both sides of the 8 x 8-tile limit of the coverage-mask
form and tiles whose lists overflow a placement wave's 16-entry LDS stage: the
integer stage (depth order, tile lists, ranges) against the
reference integer stage re-run on the CPU from the GPU's own depth keys and
footprints, bit for bit."""
import dataclasses

import numpy as np
import pytest

import scenegen
from tests.gpu_helpers import cpu_bin

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 256              # one chunk of the depth order (a chunk per 256 Gaussians at most)
N_BIG = 128          # Gaussians enlarged and gathered near the origin
W, H = 472, 344      # 30 x 22 tiles: tile groups of 8 x 8 with a ragged last column and row


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


def mixed_scene():
    """scenegen.make_scene(N, 41) with, for the first N_BIG Gaussians, rows
    0..2 of L (the spatial block of the Cholesky factor) scaled by 6 (their
    conditional spatial covariance by 36), positions scaled by 0.2 towards the
    origin and opacity 0.9, so that their footprints overlap in the middle of
    the frame."""
    s = scenegen.make_scene(N, 41)
    L, mu, al = s.L.copy(), s.mu_p.copy(), s.alpha.copy()
    for i in range(3):
        for j in range(i + 1):
            L[scenegen.tri_index(i, j), :N_BIG] *= 6.0
    mu[:, :N_BIG] *= 0.2
    al[:N_BIG] = 0.9
    return dataclasses.replace(s, L=np.ascontiguousarray(L), mu_p=np.ascontiguousarray(mu), alpha=al)


def test_counting_binner_mask_and_trim_boxes_and_stage_flushes(R, report):
    from paper_2503_07946_amd.render import GaussianScene
    scene = mixed_scene()
    views = scenegen.make_views(3, 42, r=3.0, W=W, H=H)
    gs = GaussianScene.from_host(scene)
    print(f"[binner] {N} Gaussians ({N_BIG} enlarged), 3 views {W}x{H}", flush=True)
    b = R.render_frames(R.make_frames([(gs, v) for v in views]))
    torch.cuda.synchronize()
    counts = b.counts().cpu().numpy()
    tx, ty = (W + 15) // 16, (H + 15) // 16
    for f in range(len(views)):
        dk = b.depth_key(f).cpu().numpy().view(np.uint32)
        rect = b.rect(f).cpu().numpy().view(np.uint32)
        order, tile, g, ranges = cpu_bin(dk, rect, tx, tx * ty)
        kept = int(counts[f, 0])
        assert kept == len(order)
        # the case is what it claims to be: boxes of both forms among the kept ...
        r = rect[order].astype(np.int64)
        bw = (r[:, 1] & 0xFFFF) - (r[:, 0] & 0xFFFF)
        bh = (r[:, 1] >> 16) - (r[:, 0] >> 16)
        big = (bw > 8) | (bh > 8)
        assert big.any() and (~big & (bw > 0)).any()
        # ... and a tile list longer than the 16-entry stage (one chunk here)
        per_tile = np.bincount(tile, minlength=tx * ty)
        assert per_tile.max() >= 17 * -(-N // 256)
        assert np.array_equal(b.order(f).cpu().numpy()[:kept], order)
        t_gpu, g_gpu, base = b.pairs(f, counts)
        assert np.array_equal(t_gpu.cpu().numpy(), tile)
        assert np.array_equal(g_gpu.cpu().numpy(), g)
        rg = b.ranges(f).cpu().numpy().astype(np.int64)
        ne = ranges[:, 1] > ranges[:, 0]
        assert np.array_equal(rg[ne] - base, ranges[ne])
        assert np.all(rg[~ne, 0] == rg[~ne, 1])
        report("binner_paths", frame=f, kept=kept, pairs=len(tile), big_boxes=int(big.sum()),
               longest_list=int(per_tile.max()))
