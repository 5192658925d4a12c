"""SD7_PROFILE: a context created with the variable set times each stage it
runs between two HIP events (sd7_profile_read); one created without it
records nothing, and timing changes no output.  GPU only."""
import time

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_profile_times_each_stage_and_changes_no_output(monkeypatch, report):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import GaussianScene, Renderer
    monkeypatch.setenv("SD7_PROFILE", "1")
    Rp = Renderer(0)
    monkeypatch.delenv("SD7_PROFILE")
    R0 = Renderer(0)
    s = scenegen.make_scene(20000, 61, sigma_off=0.1)
    views = scenegen.make_views(4, 61, r=3.0, W=256, H=192)
    g = GaussianScene.from_host(s)
    items = [(g, views[0]), (g, views[1])]
    print("[profile] three two-frame renders with SD7_PROFILE=1", flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        bp = Rp.render_frames(Rp.make_frames(items))
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    st = Rp.profile()
    assert set(st) == {"slice_project", "bin", "rasterize"}, st
    for name, (calls, total, mx) in st.items():
        assert calls == 3 and 0.0 < mx <= total, (name, st[name])
    assert sum(t for _, t, _ in st.values()) <= wall_ms
    report("profile", stages={k: v[1] for k, v in st.items()}, wall_ms=wall_ms)
    # the no-allocation entry point times its three stages too
    fr = Rp.make_frames([(g, views[2])])
    Rp.render_static(fr, 1 << 18)
    st2 = Rp.profile(reset=True)
    assert all(st2[k][0] == 4 for k in ("slice_project", "bin", "rasterize")), st2
    assert Rp.profile() == {}
    print("[profile] the same renders without the variable", flush=True)
    b0 = R0.render_frames(R0.make_frames(items))
    torch.cuda.synchronize()
    assert R0.profile() == {}
    for fp, f0 in zip(bp.frames, b0.frames):
        assert np.array_equal(fp.image.cpu().numpy(), f0.image.cpu().numpy())
        assert np.array_equal(fp.last.cpu().numpy(), f0.last.cpu().numpy())
    Rp.close()
    R0.close()
