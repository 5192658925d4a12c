"""Served frames of the serving configuration's sizes against the FP64
oracle: the four resident scenes (100k, 300k, 1M and 2M Gaussians, the
ill-conditioned sigma_off = 0.15 set) and the request stream's resolutions
(512^2, 800^2, 1280x720, 1920x1080) go through the scheduler's continuous
batching; the 32x32 centre crop of every completed frame is compared pixel by
pixel with the oracle (|gpu - oracle| <= 1e-4 + fbound).  The oracle takes the
Gaussians whose FP64 opacity box comes within a pixel of the crop; every
other Gaussian is below 1/255 on the crop.  GPU only."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_helpers import image_check

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# This set's correlated (t, d) blocks make the FP32 slice's error, and with it
# the oracle's opacity bands, several times wider than the other
# configurations': measured 0.2-2.6 % of crop pixels hold an in-band decision.
C3_FLAG_CAP = 0.03


def test_served_c3_frames_match_the_oracle_on_centre_crops(report):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd import serve
    from paper_2503_07946_amd.render import GaussianScene, get_renderer
    R = get_renderer(0)
    print("[serve-c3] scenes of 100k, 300k, 1M and 2M Gaussians", flush=True)
    host = scenegen.config3_scenes()
    sizes = [s.n for s in host]
    scenes = [GaussianScene.from_host(s) for s in host]
    ex = serve.GpuExecutor(R, scenes, nstreams=2, keep_images=True)
    reqs = serve.default_requests(16, 200.0, sizes, seed=305, resolutions=scenegen.SERVE_RES)
    print("[serve-c3] 16 requests through the scheduler", flush=True)
    st = serve.Scheduler(ex, hbm_budget=16 << 30, max_slots=8, max_inflight=2).run(reqs)
    assert sorted(r.rid for r in st.completed) == list(range(16))
    seen = set()
    for r in sorted(st.completed, key=lambda q: q.rid):
        v = r.view
        img = r.result[0].numpy()
        assert img.shape == (3, v.H, v.W)
        x0, y0, cw, ch = v.W // 2 - 16, v.H // 2 - 16, 32, 32
        scene = host[r.scene]
        print(f"[serve-c3] request {r.rid}: {scene.n} Gaussians at {v.W}x{v.H}, oracle crop", flush=True)
        sl = oracle.slice_(scene, v)
        pr = oracle.project(sl, scene.sh, v)
        near = pr.visible & (pr.box[2] >= x0 - 1) & (pr.box[0] <= x0 + cw + 1) & \
            (pr.box[3] >= y0 - 1) & (pr.box[1] <= y0 + ch + 1)
        o = oracle.render(scene.subset(np.nonzero(near)[0]), v, crop=(x0, y0, cw, ch))
        err, nflag = image_check(img[:, y0:y0 + ch, x0:x0 + cw], o)
        report("serve_c3_crop", rid=r.rid, gaussians=scene.n, res=[v.W, v.H], near=int(near.sum()),
               max_err=err, flagged=nflag)
        assert err <= 1e-4, (r.rid, err)
        assert nflag <= C3_FLAG_CAP * cw * ch, (r.rid, nflag)
        seen.add((scene.n, (v.W, v.H)))
    # the stream (seed 305) covers every scene, every resolution and the
    # largest frame, 2M Gaussians at 1920x1080
    assert {n for n, _ in seen} == set(sizes) and (2_000_000, (1920, 1080)) in seen, seen
