"""The compositing kernel reads splat records at 32-bit byte offsets unless a
frame of the call has so many Gaussians that its records span 4 GiB or more
(more than 89,478,485); then every frame of the call is composited with
64-bit addressing.  A frame renders bitwise the same in such a call as alone
(X17's batch invariance, here across the two addressing forms)."""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIDE_N = 0xFFFFFFFF // 48 + 1  # the fewest Gaussians whose 48-byte records pass 4 GiB
DIAGONAL = (0, 2, 5, 9, 14, 20, 27)  # rows of L's diagonal in the packed lower triangle


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


def big_culled_scene(n):
    """n valid Gaussians of zero opacity (every one culled by the slice's
    opacity test), built on the device: 84 floats each, about 30 GB."""
    from paper_2503_07946_amd.render import GaussianScene
    dev = "cuda"
    mu_p = torch.zeros(3 * n, dtype=torch.float32, device=dev)
    mu_t = torch.zeros(n, dtype=torch.float32, device=dev)
    mu_d = torch.zeros(3 * n, dtype=torch.float32, device=dev)
    mu_d[2 * n:].fill_(1.0)
    L_ = torch.zeros(28 * n, dtype=torch.float32, device=dev)
    for r in DIAGONAL:
        L_[r * n:(r + 1) * n].fill_(0.1)
    alpha = torch.zeros(n, dtype=torch.float32, device=dev)
    sh = torch.zeros(48 * n, dtype=torch.float32, device=dev)
    return GaussianScene(mu_p, mu_t, mu_d, L_, alpha, sh)


def test_frame_renders_the_same_beside_a_frame_past_4gib_of_records(R):
    from paper_2503_07946_amd.render import GaussianScene
    free, _ = torch.cuda.mem_get_info()
    if free < 60 * (1 << 30):
        pytest.skip(f"needs about 45 GiB of free device memory, {free >> 30} GiB free")
    s = scenegen.make_scene(20000, 41, sigma_off=0.15)
    v = scenegen.make_views(1, 41, r=3.0, W=200, H=120, bg=(0.2, 0.5, 1.0))[0]
    g = GaussianScene.from_host(s)
    print("[wide] small frame alone (32-bit offsets)", flush=True)
    alone = R.render_frames(R.make_frames([(g, v)]))
    a = {k: getattr(alone.frames[0], k).cpu().numpy() for k in ("image", "final_T", "last")}
    ca = R.read_counts(alone)
    assert ca[0, 1] > 0  # the frame has pairs to composite
    del alone
    print(f"[wide] building a culled scene of {WIDE_N} Gaussians on the device", flush=True)
    big = big_culled_scene(WIDE_N)
    print("[wide] small frame beside it (64-bit addressing)", flush=True)
    mix = R.render_frames(R.make_frames([(g, v), (big, v)]))
    cm = R.read_counts(mix)
    for k in ("image", "final_T", "last"):
        assert np.array_equal(a[k], getattr(mix.frames[0], k).cpu().numpy()), k
    assert cm[0, 1] == ca[0, 1] and cm[1, 1] == 0  # same pairs; the big frame keeps none
    del mix, big
    torch.cuda.empty_cache()
