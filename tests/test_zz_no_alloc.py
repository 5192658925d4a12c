"""sd7_render_static, the render entry point for callers that cannot allocate
device memory, against sd7_render with a caller workspace on the same frames:
bitwise equal images, transmittance, consumed-entry counts and counters, on
consecutive calls whose inputs shrink (the static workspace keeps the previous
call's contents); and the refusal of frames that need more workspace than the
static one holds.  GPU only."""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_07946_amd.render import get_renderer
    return get_renderer(0)


def _frames(R, gs, views):
    fr = R.make_frames([(gs, v) for v in views])
    for f in fr:  # outputs the render must overwrite
        f.image.fill_(float("nan"))
        f.final_T.fill_(float("nan"))
        f.last.fill_(-1)
    return fr


CALLS = {
    "3x160x120_6k": lambda: (scenegen.make_scene(6000, 41, sigma_off=0.1),
                             scenegen.make_views(3, 41, r=3.0, W=160, H=120, bg=(0.2, 0.1, 0.3))),
    "2x37x23_2k": lambda: (scenegen.make_scene(2000, 42, sigma_off=0.15),
                           scenegen.make_views(2, 42, r=3.0, W=37, H=23)),
    "1x64x64_1k": lambda: scenegen.config0(),
}


def test_static_render_equals_workspace_render(R, report):
    from paper_2503_07946_amd import _lib as L
    from paper_2503_07946_amd.render import GaussianScene
    cap = 1 << 18
    sizes = []
    for name, make in CALLS.items():   # each call's input is smaller than the one before
        scene, views = make()
        gs = GaussianScene.from_host(scene)
        print(f"[no_alloc] {name}: workspace render", flush=True)
        ref = _frames(R, gs, views)
        b = R.batch(ref, cap)
        sizes.append(int(b.layout.bytes))
        assert b.layout.bytes <= L.SD7_STATIC_WS_BYTES
        R.stage("sd7_render", b)
        torch.cuda.synchronize()
        print(f"[no_alloc] {name}: static render", flush=True)
        got = _frames(R, gs, views)
        counts = torch.full((len(views), L.SD7_CNT_WORDS), -1, dtype=torch.int32, device="cuda")
        R.render_static(got, cap, counts)
        torch.cuda.synchronize()
        for f, (a, g) in enumerate(zip(ref, got)):
            assert torch.equal(a.image, g.image), (name, f)
            assert torch.equal(a.final_T, g.final_T), (name, f)
            assert torch.equal(a.last, g.last), (name, f)
            assert not torch.isnan(g.image).any()
        c_ref = b.counts()[:, :L.SD7_CNT_NEEDED + 1]
        assert torch.equal(counts[:, :L.SD7_CNT_NEEDED + 1], c_ref), name
        assert int(c_ref[:, L.SD7_CNT_PAIRS].min()) > 0
        report("no_alloc", call=name, frames=len(views), workspace_bytes=int(b.layout.bytes),
               pairs=c_ref[:, L.SD7_CNT_PAIRS].tolist())
    assert sizes[0] > sizes[1] and sizes[1] > sizes[2]


def test_static_render_refuses_frames_beyond_its_workspace(R):
    """300,000 Gaussians at 1920x1080 with an 8M-pair arena need about 140 MB
    of workspace: refused synchronously with SD7_EWORKSPACE, nothing written."""
    from paper_2503_07946_amd import _lib as L
    from paper_2503_07946_amd.render import GaussianScene
    n = 300_000
    dev = torch.device("cuda")
    z = lambda k: torch.zeros((k, n) if k > 1 else (n,), dtype=torch.float32, device=dev)
    gs = GaussianScene(z(3), z(1), z(3), z(28), z(1), z(48))
    v = scenegen.make_views(1, 5, r=3.0, W=1920, H=1080)[0]
    fr = _frames(R, gs, [v])
    cap = 8 << 20
    assert R.plan(fr, cap).bytes > L.SD7_STATIC_WS_BYTES
    with pytest.raises(L.Sd7Error) as e:
        R.render_static(fr, cap)
    assert e.value.code == L.SD7_EWORKSPACE
    assert "static" in str(e.value)
    torch.cuda.synchronize()
    assert torch.isnan(fr[0].image).all() and bool((fr[0].last == -1).all())
