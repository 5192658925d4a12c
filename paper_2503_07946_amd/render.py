"""PyTorch-facing wrapper of lib7dgs.  PyTorch provides device memory and
streams; every step of the render path runs in the HIP library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

PARAMS = ("mu_p", "mu_t", "mu_d", "L", "alpha", "sh")
SHAPES = {"mu_p": 3, "mu_t": 1, "mu_d": 3, "L": 28, "alpha": 1, "sh": 48}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class GaussianScene:
    """A scene of 7D Gaussians resident in device memory (FP32 planes)."""

    def __init__(self, mu_p, mu_t, mu_d, L_, alpha, sh, agr=None):
        self.mu_p, self.mu_t, self.mu_d, self.L, self.alpha, self.sh = mu_p, mu_t, mu_d, L_, alpha, sh
        self.agr = agr  # optional AGR weights (Sec. 4.3), SD7_AGR_WEIGHTS floats
        if agr is not None and (agr.dtype != torch.float32 or not agr.is_contiguous()
                                or agr.device.type != "cuda" or agr.numel() != L.SD7_AGR_WEIGHTS):
            raise ValueError(f"agr: need a contiguous float32 device tensor of {L.SD7_AGR_WEIGHTS} values")
        n = int(mu_t.shape[0])
        for k in PARAMS:
            t = getattr(self, k)
            if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError(f"{k}: need a contiguous float32 device tensor")
            if t.numel() != SHAPES[k] * n:
                raise ValueError(f"{k}: expected {SHAPES[k]} x {n} values, got {tuple(t.shape)}")

    @classmethod
    def from_host(cls, scene, device="cuda", agr=None):
        arrs = scene.arrays() if hasattr(scene, "arrays") else scene
        w = None if agr is None else torch.as_tensor(np.ascontiguousarray(agr, np.float32)).to(device)
        return cls(*(torch.as_tensor(np.ascontiguousarray(arrs[k], np.float32)).to(device)
                     for k in PARAMS), agr=w)

    @property
    def n(self) -> int:
        return int(self.mu_t.shape[0])

    @property
    def device(self):
        return self.mu_t.device

    def nbytes(self) -> int:
        return 84 * 4 * self.n

    def sd7(self) -> L.Sd7Scene:
        return L.Sd7Scene(*(_ptr(getattr(self, k)) for k in PARAMS), self.n, _ptr(self.agr))


def view_struct(v) -> L.Sd7View:
    s = L.Sd7View()
    s.R_wc[:] = [float(x) for x in np.asarray(v.R_wc, np.float32).reshape(9)]
    s.c[:] = [float(x) for x in np.asarray(v.c, np.float32).reshape(3)]
    s.fx, s.fy, s.cx, s.cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
    s.W, s.H = int(v.W), int(v.H)
    s.t = float(v.t)
    s.d[:] = [float(x) for x in np.asarray(v.d, np.float32).reshape(3)]
    s.lambda_t, s.lambda_d = float(v.lambda_t), float(v.lambda_d)
    s.bg[:] = [float(x) for x in np.asarray(v.bg, np.float32).reshape(3)]
    s.d_per_gaussian = 1 if getattr(v, "d_per_gaussian", False) else 0
    return s


@dataclass
class FrameIO:
    scene: GaussianScene
    view: object
    image: torch.Tensor
    final_T: torch.Tensor
    last: torch.Tensor
    dL_dimage: torch.Tensor | None = None
    grads: dict | None = None
    ncontrib: torch.Tensor | None = None
    keep_sliced: bool = False   # keep the sliced statistics in the workspace


@dataclass
class Batch:
    """One call's frames, their outputs and the workspace."""
    frames: list
    cstruct: object
    nf: int
    capacity: int
    layout: L.Sd7Layout
    ws: torch.Tensor
    counts_host: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    # ---- typed views of workspace arrays (frame f) -------------------------
    def _arr(self, off, dtype, count, offset_elems=0):
        itemsize = torch.tensor([], dtype=dtype).element_size()
        start = int(off) + itemsize * int(offset_elems)
        return self.ws[start:start + itemsize * int(count)].view(dtype)

    def g0(self, f):
        return int(self.layout.g0[f])

    def planes(self, name, k, f):
        n = self.frames[f].scene.n
        return self._arr(getattr(self.layout, name), torch.float32, k * n, k * self.g0(f)).view(k, n)

    def mu_c(self, f=0):
        return self.planes("off_mu_c", 3, f)

    def cov_c(self, f=0):
        return self.planes("off_cov_c", 6, f)

    def alpha_c(self, f=0):
        return self.planes("off_alpha_c", 1, f)[0]

    def splat(self, f=0):
        n = self.frames[f].scene.n
        return self._arr(self.layout.off_splat, torch.float32, 12 * n, 12 * self.g0(f)).view(n, 12)

    def rect(self, f=0):
        n = self.frames[f].scene.n
        return self._arr(self.layout.off_rect, torch.int32, 4 * n, 4 * self.g0(f)).view(n, 4)

    def depth_key(self, f=0):
        n = self.frames[f].scene.n
        return self._arr(self.layout.off_depth_key, torch.int32, n, self.g0(f))

    def order(self, f=0):
        n = self.frames[f].scene.n
        return self._arr(self.layout.off_order, torch.int32, n, self.g0(f))

    def counts(self):
        return self._arr(self.layout.off_counts, torch.int32, self.nf * L.SD7_CNT_WORDS).view(
            self.nf, L.SD7_CNT_WORDS)

    def pairs(self, f=0, counts=None):
        """(tile id, Gaussian index) of every pair of frame f, in arena order,
        and the frame's first arena slot.  Tile ids come from the ranges."""
        c = self.counts().cpu().numpy() if counts is None else counts
        base, P = int(c[f, L.SD7_CNT_PAIR_BASE]), int(c[f, L.SD7_CNT_PAIRS])
        g = self._arr(self.layout.off_pair_g, torch.int32, P, base)
        rg = self.ranges(f).to(torch.int64)
        lens = (rg[:, 1] - rg[:, 0]).clamp(min=0)
        t = torch.repeat_interleave(torch.arange(rg.shape[0], device=rg.device, dtype=torch.int32), lens)
        return t, g, base

    def ranges(self, f=0):
        v = self.frames[f].view
        T = ((v.W + 15) // 16) * ((v.H + 15) // 16)
        return self._arr(self.layout.off_ranges, torch.int32, 2 * T, 2 * int(self.layout.tile0[f])).view(T, 2)

    def d_splat(self, f=0):
        return self.planes("off_d_splat", 9, f)


class Renderer:
    """Owns an sd7 context on one device."""

    def __init__(self, device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the 7DGS render path needs a GPU (no CPU fallback)")
        self.lib = L.load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.sd7_create(self.device, ctypes.byref(h)))
        self.ctx = h
        self.default_capacity = 1 << 20

    def profile(self, reset: bool = False) -> dict:
        """Per-stage GPU times of this renderer's context (sd7_profile_read):
        {stage: (calls, total_ms, max_ms)}; empty unless SD7_PROFILE was set
        when the renderer was created.  Waits for the timed stages."""
        out = (L.Sd7StageTime * 16)()
        n = ctypes.c_int(0)
        L.check(self.lib.sd7_profile_read(self.ctx, out, 16, ctypes.byref(n), int(reset)))
        return {out[i].name.decode(): (int(out[i].calls), float(out[i].total_ms), float(out[i].max_ms))
                for i in range(n.value)}

    def close(self):
        if self.ctx:
            self.lib.sd7_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- batch construction ------------------------------------------------
    def make_frames(self, items, outputs=None, need_grad=False, count=False, keep_sliced=False) -> list:
        frames = []
        dev = torch.device("cuda", self.device)
        for k, (scene, view) in enumerate(items):
            H, W = int(view.H), int(view.W)
            if outputs is not None:
                img, T, last = outputs[k]
            else:
                img = torch.empty((3, H, W), dtype=torch.float32, device=dev)
                T = torch.empty((H, W), dtype=torch.float32, device=dev)
                last = torch.empty((H, W), dtype=torch.int32, device=dev)
            fr = FrameIO(scene, view, img, T, last, keep_sliced=keep_sliced)
            if count:
                fr.ncontrib = torch.empty((H, W), dtype=torch.int32, device=dev)
            if need_grad:
                fr.grads = {k2: torch.empty_like(getattr(scene, k2)) for k2 in PARAMS}
            frames.append(fr)
        return frames

    @staticmethod
    def cstruct(frames):
        arr = (L.Sd7Frame * len(frames))()
        for i, fr in enumerate(frames):
            if getattr(fr, "sliced_in_ws", None) is None:
                # whether a render with these descriptors keeps the sliced
                # statistics the reverse pass reads
                fr.sliced_in_ws = fr.keep_sliced or fr.grads is not None
            c = arr[i]
            c.scene = fr.scene.sd7()
            c.view = view_struct(fr.view)
            c.image, c.final_T, c.last = _ptr(fr.image), _ptr(fr.final_T), _ptr(fr.last)
            c.dL_dimage = _ptr(fr.dL_dimage)
            c.ncontrib = _ptr(fr.ncontrib)
            c.outputs = L.SD7_OUT_SLICED if fr.keep_sliced else 0
            if fr.grads is not None:
                c.grad = L.Sd7SceneGrad(*(_ptr(fr.grads[k]) for k in PARAMS), _ptr(fr.grads.get("lambda")))
        return arr

    def plan(self, frames, capacity: int) -> L.Sd7Layout:
        cs = self.cstruct(frames)
        lay = L.Sd7Layout()
        L.check(self.lib.sd7_plan(cs, len(frames), int(capacity), ctypes.byref(lay)))
        return lay

    def batch(self, frames, capacity: int, ws: torch.Tensor | None = None) -> Batch:
        cs = self.cstruct(frames)
        lay = L.Sd7Layout()
        L.check(self.lib.sd7_plan(cs, len(frames), int(capacity), ctypes.byref(lay)))
        if ws is None or ws.numel() < lay.bytes:
            ws = torch.empty(int(lay.bytes), dtype=torch.uint8, device=torch.device("cuda", self.device))
        return Batch(frames, cs, len(frames), int(capacity), lay, ws)

    def stage(self, name: str, b: Batch, stream=None):
        st = torch.cuda.current_stream(self.device) if stream is None else stream
        fn = getattr(self.lib, name)
        L.check(fn(self.ctx, b.cstruct, b.nf, b.capacity, ctypes.c_void_p(b.ws.data_ptr()),
                   b.ws.numel(), ctypes.c_void_p(st.cuda_stream)))

    def read_counts(self, b: Batch, stream=None) -> np.ndarray:
        st = torch.cuda.current_stream(self.device) if stream is None else stream
        out = (ctypes.c_uint32 * (b.nf * L.SD7_CNT_WORDS))()
        L.check(self.lib.sd7_read_counts(self.ctx, b.nf, ctypes.c_void_p(b.ws.data_ptr()), out,
                                         ctypes.c_void_p(st.cuda_stream)))
        b.counts_host = np.frombuffer(out, dtype=np.uint32).reshape(b.nf, L.SD7_CNT_WORDS).copy()
        return b.counts_host

    # ---- whole renders -------------------------------------------------------
    def render_frames(self, frames, capacity: int | None = None, stream=None,
                      exact: bool = True) -> Batch:
        """slice, project, bin, rasterize.  With exact=True the pair counts are
        read back after binning (one host sync) and binning is redone with a
        larger arena if a frame overflowed."""
        cap = self.default_capacity if capacity is None else int(capacity)
        b = self.batch(frames, cap)
        for s in ("sd7_slice_project", "sd7_bin"):
            self.stage(s, b, stream)
        if exact:
            c = self.read_counts(b, stream)
            if np.any(c[:, L.SD7_CNT_FLAGS] & L.SD7_FLAG_SORT_STALL):
                raise L.Sd7Error(L.SD7_EHIP, "depth sort stalled (SD7_FLAG_SORT_STALL)")
            if np.any(c[:, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW):
                need = int(sum(-(-int(x) // L.SD7_PAIR_ROUND) * L.SD7_PAIR_ROUND for x in c[:, L.SD7_CNT_NEEDED]))
                b2 = self.batch(frames, need)
                prefix = int(b.layout.off_pair_g)
                b2.ws[:prefix].copy_(b.ws[:prefix])
                b = b2
                self.stage("sd7_bin", b, stream)
                self.default_capacity = max(self.default_capacity, need)
        self.stage("sd7_rasterize", b, stream)
        return b

    def graph(self, frames, capacity: int) -> "RenderGraph":
        """sd7_render of frames of these sizes captured as one HIP graph
        (sd7_graph_create), with its own workspace."""
        return RenderGraph(self, frames, capacity)

    def render_static(self, frames, capacity: int, counts_out: torch.Tensor | None = None, stream=None):
        """sd7_render over the library's own per-device workspace (no workspace
        argument; nothing is allocated).  counts_out: optional int32 device
        tensor of len(frames) x SD7_CNT_WORDS words for the frames' counters."""
        st = torch.cuda.current_stream(self.device) if stream is None else stream
        cs = self.cstruct(frames)
        if counts_out is not None:
            assert counts_out.is_cuda and counts_out.numel() >= len(frames) * L.SD7_CNT_WORDS
        L.check(self.lib.sd7_render_static(self.ctx, cs, len(frames), int(capacity), _ptr(counts_out),
                                           ctypes.c_void_p(st.cuda_stream)))

    def render(self, scene: GaussianScene, view, capacity=None, stream=None, count=False,
               keep_sliced=True) -> Batch:
        return self.render_frames(self.make_frames([(scene, view)], count=count, keep_sliced=keep_sliced),
                                  capacity, stream)

    def backward(self, b: Batch, dL_dimages, stream=None):
        """Reverse pass of a rendered batch: returns per-frame gradient dicts."""
        for fr in b.frames:
            if not fr.sliced_in_ws:
                raise RuntimeError("the batch was rendered without its sliced statistics: render with "
                                   "keep_sliced=True (or gradient buffers) before the reverse pass")
        for fr, g in zip(b.frames, dL_dimages):
            fr.dL_dimage = g.contiguous()
            if fr.grads is None:
                fr.grads = {k: torch.empty_like(getattr(fr.scene, k)) for k in PARAMS}
                fr.grads["lambda"] = torch.empty(2, dtype=torch.float32, device=fr.scene.device)
            fr.grads["lambda"].zero_()  # dL/dlambda_t, dL/dlambda_d (accumulated)
        b.cstruct = self.cstruct(b.frames)
        for s in ("sd7_rasterize_backward", "sd7_project_backward", "sd7_slice_backward"):
            self.stage(s, b, stream)
        return [fr.grads for fr in b.frames]


class RenderGraph:
    """A captured sd7_render (include/sd7.h, sd7_graph_*): launch() replays it
    for frames of the captured sizes (other views, scenes of the same size,
    other outputs).  Owns the workspace the graph uses."""

    def __init__(self, renderer: Renderer, frames, capacity: int):
        self.R = renderer
        self.b = renderer.batch(frames, capacity)
        h = ctypes.c_void_p()
        L.check(renderer.lib.sd7_graph_create(renderer.ctx, self.b.cstruct, self.b.nf, int(capacity),
                                              ctypes.c_void_p(self.b.ws.data_ptr()), self.b.ws.numel(),
                                              ctypes.byref(h)))
        self.handle = h

    def launch(self, frames=None, stream=None) -> Batch:
        """Replay for `frames` (default: the captured ones); returns the batch
        view of the workspace with these frames."""
        st = torch.cuda.current_stream(self.R.device) if stream is None else stream
        cs, nf = self.b.cstruct, self.b.nf
        if frames is not None:
            cs, nf = self.R.cstruct(frames), len(frames)
        L.check(self.R.lib.sd7_graph_launch(self.handle, cs, nf, ctypes.c_void_p(st.cuda_stream)))
        if frames is not None:
            self.b.frames, self.b.cstruct = frames, cs
        return self.b

    def close(self):
        if self.handle:
            self.R.lib.sd7_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_RENDERERS: dict = {}


def cov_decompose(cov: torch.Tensor, renderer=None):
    """Densification helper: cov [6, n] (packed symmetric, float32, device) ->
    (scale [3, n] descending, rot [9, n] row-major R with det R = +1)."""
    r = renderer or get_renderer(cov.device.index)
    if cov.dtype != torch.float32 or not cov.is_contiguous() or cov.dim() != 2 or cov.shape[0] != 6:
        raise ValueError("cov: need a contiguous float32 [6, n] device tensor")
    n = int(cov.shape[1])
    scale = torch.empty((3, n), dtype=torch.float32, device=cov.device)
    rot = torch.empty((9, n), dtype=torch.float32, device=cov.device)
    st = torch.cuda.current_stream(cov.device)
    L.check(r.lib.sd7_cov_decompose(r.ctx, n, _ptr(cov), _ptr(scale), _ptr(rot), ctypes.c_void_p(st.cuda_stream)))
    return scale, rot


def split_mask(scene: GaussianScene, extent: float, time_span: float = 1.0, renderer=None) -> torch.Tensor:
    """Densification helper: bool [n], the Gaussians the temporal split test selects."""
    r = renderer or get_renderer(scene.device.index)
    out = torch.empty(scene.n, dtype=torch.uint8, device=scene.device)
    st = torch.cuda.current_stream(scene.device)
    s = scene.sd7()
    L.check(r.lib.sd7_split_test(r.ctx, ctypes.byref(s), float(extent), float(time_span), _ptr(out),
                                 ctypes.c_void_p(st.cuda_stream)))
    return out.bool()


class Adam:
    """Fused Adam over a scene's six parameter arrays (sd7_adam_step) and
    pruning at an opacity floor (sd7_prune_count / sd7_prune_apply).

    The learning rates are per group; the defaults follow 3DGS's schedule at
    its start where a group has a counterpart (position 1.6e-4 for the three
    means, SH 2.5e-3) and are readings for the others: the paper keeps the
    3DGS settings and names none for mu_t, mu_d or the factor L, and this
    library renders the activated opacity instead of a logit."""

    DEFAULT_LR = {"mu_p": 1.6e-4, "mu_t": 1.6e-4, "mu_d": 1.6e-4, "L": 1e-3, "alpha": 1e-2, "sh": 2.5e-3}

    def __init__(self, scene: GaussianScene, lr=None, betas=(0.9, 0.999), eps=1e-15,
                 alpha_bounds=(1e-4, 0.9999), diag_min=1e-4, renderer=None):
        self.r = renderer or get_renderer(scene.device.index)
        self.lr = dict(self.DEFAULT_LR, **(lr or {}))
        self.betas, self.eps, self.alpha_bounds, self.diag_min = betas, eps, alpha_bounds, diag_min
        self.m = {k: torch.zeros_like(getattr(scene, k)) for k in PARAMS}
        self.v = {k: torch.zeros_like(getattr(scene, k)) for k in PARAMS}
        self.t = 0

    @staticmethod
    def _arrays(d) -> L.Sd7Arrays:
        return L.Sd7Arrays(*(_ptr(d[k]) for k in PARAMS))

    def step(self, scene: GaussianScene, grads: dict):
        self.t += 1
        cfg = L.Sd7Adam()
        cfg.lr[:] = [float(self.lr[k]) for k in PARAMS]
        cfg.beta1, cfg.beta2 = float(self.betas[0]), float(self.betas[1])
        cfg.eps, cfg.step = float(self.eps), self.t
        cfg.alpha_lo, cfg.alpha_hi = float(self.alpha_bounds[0]), float(self.alpha_bounds[1])
        cfg.diag_min = float(self.diag_min)
        p = self._arrays({k: getattr(scene, k) for k in PARAMS})
        g = L.Sd7SceneGrad(*(_ptr(grads[k]) for k in PARAMS), None)
        st = torch.cuda.current_stream(scene.device)
        L.check(self.r.lib.sd7_adam_step(self.r.ctx, scene.n, ctypes.byref(p), ctypes.byref(g),
                                         ctypes.byref(self._arrays(self.m)), ctypes.byref(self._arrays(self.v)),
                                         ctypes.byref(cfg), ctypes.c_void_p(st.cuda_stream)))

    def prune(self, scene: GaussianScene, tau: float = 0.01) -> GaussianScene:
        """The Gaussians with opacity >= tau (the paper's tau_min = 0.01), with
        their moments; one host read of the kept count."""
        n, dev = scene.n, scene.device
        lib = self.r.lib
        ws = torch.empty(max(int(lib.sd7_prune_workspace_size(n)), 256), dtype=torch.uint8, device=dev)
        cnt = torch.zeros(1, dtype=torch.int32, device=dev)
        st = torch.cuda.current_stream(dev)
        L.check(lib.sd7_prune_count(self.r.ctx, n, _ptr(scene.alpha), float(tau), _ptr(ws), ws.numel(),
                                    _ptr(cnt), ctypes.c_void_p(st.cuda_stream)))
        k = int(cnt.item())
        srcs = [getattr(scene, p) for p in PARAMS] + [self.m[p] for p in PARAMS] + [self.v[p] for p in PARAMS]
        dsts = [torch.empty(SHAPES[p] * k, dtype=torch.float32, device=dev).view(*(
                (SHAPES[p], k) if getattr(scene, p).dim() == 2 else (k,))) for p in PARAMS] * 3
        dsts = [torch.empty_like(d) for d in dsts]
        planes = (ctypes.c_int32 * len(srcs))(*[SHAPES[p] for p in PARAMS] * 3)
        sp = (ctypes.c_void_p * len(srcs))(*[t.data_ptr() for t in srcs])
        dp = (ctypes.c_void_p * len(dsts))(*[t.data_ptr() for t in dsts])
        L.check(lib.sd7_prune_apply(self.r.ctx, n, k, sp, dp, planes, len(srcs), _ptr(ws), ws.numel(),
                                    ctypes.c_void_p(st.cuda_stream)))
        self.m = dict(zip(PARAMS, dsts[6:12]))
        self.v = dict(zip(PARAMS, dsts[12:18]))
        return GaussianScene(*dsts[:6], agr=scene.agr)


def get_renderer(device=None) -> Renderer:
    dev = torch.cuda.current_device() if device is None else int(device)
    r = _RENDERERS.get(dev)
    if r is None:
        r = _RENDERERS[dev] = Renderer(dev)
    return r


class Render7DGS(torch.autograd.Function):
    """image = render(mu_p, mu_t, mu_d, L, alpha, sh; view).  The backward runs
    the library's reverse kernels (compositing recomputed back to front from
    each pixel's final transmittance, no per-pixel list state saved)."""

    @staticmethod
    def forward(ctx, mu_p, mu_t, mu_d, L_, alpha, sh, view):
        r = get_renderer(mu_p.device.index)
        scene = GaussianScene(*(t.detach().contiguous() for t in (mu_p, mu_t, mu_d, L_, alpha, sh)))
        b = r.render_frames(r.make_frames([(scene, view)], keep_sliced=True))
        ctx.batch = b
        ctx.renderer = r
        return b.frames[0].image

    @staticmethod
    def backward(ctx, dimage):
        g = ctx.renderer.backward(ctx.batch, [dimage.contiguous()])[0]
        ctx.batch = None
        return g["mu_p"], g["mu_t"], g["mu_d"], g["L"], g["alpha"], g["sh"], None


def render_image(params: dict, view) -> torch.Tensor:
    return Render7DGS.apply(params["mu_p"], params["mu_t"], params["mu_d"], params["L"],
                            params["alpha"], params["sh"], view)
