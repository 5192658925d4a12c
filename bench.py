#!/usr/bin/env python3
"""7DGS render-path benchmark on one MI355X.

Workload: 200,000 7D Gaussians (positions in [-2,2]^3, Cholesky covariance
factors with log-uniform diagonal and N(0, 0.05) off-diagonals), 50 pinhole
views of 800x800 on a sphere of radius 4 looking at the origin, t ~ U[0,1],
FP32, white background.  One step renders all 50 views through the whole
forward path (slice, project, bin, rasterize), frames batched B at a time
into one set of launches, inputs resident in HBM.

Prints one JSON line: throughput (FPS, Mpixel/s), per-stage times measured
with HIP events on the launch stream over the timed region, p50/p99 frame
latency of batched vs plain (one frame per call, pair count read back)
rendering, the roofline of the dominant kernel, and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (it counts packed FP32 FMAs: two per lane
# per clock), and the peak without packed math, which this library is built
# without: 256 CUs x 64 lanes x one FMA (2 operations) per clock x 2.4 GHz.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12

# Rasterizer roofline, in algorithmic FP32 operations of the compositing as the
# method defines it.  Per (pixel, splat) test -- every list entry a pixel
# consumes -- 12: the offsets (2), the exponent A dx^2 + B dx dy + C dy^2 + lo
# (3 squares/products, 3 coefficient products, 3 adds) and the opacity
# threshold test (1).  Per contribution -- a test that passes and does not stop
# the pixel -- 12 more: 2^p and the 0.99 clamp (2), T' = T (1 - alpha) (2),
# the stop test (1), w = T alpha (1) and three colour FMAs (6).  Traffic:
# FETCH_SIZE x 2 + WRITE_SIZE (KiB x 1024) per launch, scaling factors from a
# 1 GiB device copy, with the VALU instruction count of the same runs.  They
# hold for the library source whose digest is RASTER_SRC_SHA256 -- every
# kernel source, since the splat records and tile lists the rasterizer walks
# come from the other stages -- and are dropped (null) once it differs.
RASTER_OPS_PER_TEST = 12
RASTER_OPS_PER_CONTRIBUTION = 12
RASTER_SRC_DIR = "paper_2503_07946_amd/csrc"
RASTER_SRC_SHA256 = "289ae38be2ab3ce0cd9b13878f1b4f351d350560c7ad0e128520ee2a7b567e3f"
RASTER_TRAFFIC_BYTES = 2398679040       # (1014980 KiB x 2 + 312500 KiB) x 1024
RASTER_VALU_INSTRUCTIONS = 1040066229   # SQ_INSTS_VALU per launch (wave64 instructions)


def raster_src_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, RASTER_SRC_DIR)
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def wave_evaluations(last, ranges, W: int, H: int) -> int:
    """256 x the list entries each tile's wave traversed: up to the check
    (every 8 entries) after the last of its pixels stopped, or the whole list."""
    import torch
    th, tw = (H + 15) // 16, (W + 15) // 16
    x = torch.zeros((th * 16, tw * 16), dtype=torch.int64, device=last.device)
    x[:H, :W] = last.to(torch.int64)
    mx = x.view(th, 16, tw, 16).amax(dim=(1, 3)).reshape(-1)
    r = ranges.to(torch.int64)
    ln = r[:, 1] - r[:, 0]
    trav = torch.where(mx >= ln, ln, torch.minimum(ln, (mx + 1 + 7) // 8 * 8))
    return 256 * int(trav.sum())


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--views", type=int, default=50)
    ap.add_argument("--batch", type=int, default=25, help="frames per set of launches")
    ap.add_argument("--streams", type=int, default=2, help="HIP streams the batches of a step alternate over")
    ap.add_argument("--gaussians", type=int, default=200_000)
    ap.add_argument("--plain-frames", type=int, default=20, help="frames timed one per call")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-crop", type=int, default=128, help="side of the centre crop timed with all threads")
    ap.add_argument("--small", type=int, default=1,
                    help="also time the small workload (1,000 Gaussians, one 64x64 frame per call)")
    ap.add_argument("--stress", type=int, default=1,
                    help="also time the stress workload (4M Gaussians, 64 views of 1920x1080, forward + backward)")
    ap.add_argument("--stress-inflight", type=int, default=8)
    ap.add_argument("--serve", type=int, default=1, help="also run the serving comparison")
    ap.add_argument("--agr", type=int, default=1,
                    help="also time the full variant with adaptive Gaussian refinement (seeded weights)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests per offered load")
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-loads", type=str, default="0.5,0.9,1.25,2,4",
                    help="offered loads as multiples of the plain path's capacity")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-sizes", type=str, default="100000,300000,1000000,2000000")
    ap.add_argument("--train", type=int, default=1,
                    help="also time the training step (forward, L1 gradient, reverse pass, Adam) on 500k Gaussians at 1352x1014")
    ap.add_argument("--train-steps", type=int, default=10)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def copy_probe(mib: int):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 3}))
    return 0


def serve_bench(a, R, L):
    """Serving: four resident scenes, Poisson streams of (scene, camera, t)
    requests at mixed resolutions offered at several loads around the plain
    path's capacity; continuous batching vs one request per call.  Per load:
    `serve_warmup` + `serve_requests` requests (the first `serve_warmup` not
    counted), p50/p99 latency (arrival to completion) and the throughput each
    path sustains; the highest is each path's ceiling."""
    import numpy as np
    import torch

    import scenegen
    from paper_2503_07946_amd import serve
    from paper_2503_07946_amd.render import GaussianScene

    sizes = [int(x) for x in a.serve_sizes.split(",")]
    scenes = [GaussianScene.from_host(s) for s in scenegen.config3_scenes(sizes)]
    torch.cuda.synchronize()
    ex = serve.GpuExecutor(R, scenes, nstreams=2)
    # learn the pair counts (scene, resolution) and the plain path's service
    # time on a calibration stream
    cal = serve.default_requests(64, 1000.0, sizes, seed=301)
    for r in cal:
        ex.render_one(r)
    for r in cal:
        ex.render_one(r)
    t0 = time.perf_counter()
    for r in cal:
        ex.render_one(r)
    plain_service = (time.perf_counter() - t0) / len(cal)
    cap_plain = 1.0 / plain_service
    n = a.serve_requests + a.serve_warmup
    points = []
    for load in [float(x) for x in a.serve_loads.split(",")]:
        qps = load * cap_plain
        print(f"[bench] serving: {n} requests at {qps:.0f} QPS ({load}x the plain capacity)",
              file=sys.stderr, flush=True)
        st_p = serve.run_plain(ex, serve.default_requests(n, qps, sizes, seed=300))
        sch = serve.Scheduler(ex, serve.budget_from_gb(a.serve_budget_gb), max_slots=16, max_inflight=2)
        st_b = sch.run(serve.default_requests(n, qps, sizes, seed=300))
        points.append({"load": load, "offered_qps": round(qps, 1),
                       "plain": st_p.summary(skip=a.serve_warmup), "batched": st_b.summary(skip=a.serve_warmup)})
    ceil_p = max(p["plain"]["throughput_fps"] or 0 for p in points)
    ceil_b = max(p["batched"]["throughput_fps"] or 0 for p in points)
    return {"scenes": sizes, "resolutions": [list(r) for r in scenegen.SERVE_RES],
            "hbm_budget_gb": a.serve_budget_gb, "requests_per_load": a.serve_requests,
            "warmup_per_load": a.serve_warmup, "plain_service_ms": round(1e3 * plain_service, 3),
            "plain_path": "one request per call: one sd7_render with the pair count learned for its "
                          "(scene, resolution), then one wait for it (a re-render if the arena overflowed)",
            "throughput_ceiling_fps": {"plain": round(ceil_p, 1), "batched": round(ceil_b, 1),
                                       "batched_over_plain": round(ceil_b / ceil_p, 3) if ceil_p else None},
            "loads": points}


def run_steps(R, batches, steps, streams, record_stage=None):
    """`steps` passes over the batches, batch i on streams[i % len(streams)]
    (a batch's stages stay ordered on its stream; the batches of a step are
    independent, so one batch's slicing and binning overlap another's
    compositing).  With record_stage, HIP events on the batch's stream bracket
    that stage of every batch; returns (seconds, [ms per launch])."""
    import torch
    names = ("sd7_slice_project", "sd7_bin", "sd7_rasterize")
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for i, b in enumerate(batches):
            st = streams[i % len(streams)]
            if record_stage is None:
                R.stage("sd7_render", b, stream=st)
                continue
            for s in names:
                if s == record_stage:
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(st)
                    R.stage(s, b, stream=st)
                    e1.record(st)
                    ev.append((e0, e1))
                else:
                    R.stage(s, b, stream=st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, [e0.elapsed_time(e1) for e0, e1 in ev]


def copy_bandwidth(mib: int = 1024, reps: int = 10):
    """HBM bandwidth a plain device-to-device copy reaches (bytes read +
    written per second, the mean of `reps` timed copies of `mib` MiB after one
    untimed one): the practical ceiling beside the 8 TB/s peak."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return {"gb_s": round(2 * n * 4 / t / 1e9, 1), "bytes_per_copy": 2 * n * 4,
            "kind": f"device copy of {mib} MiB (torch copy_), mean of {reps}"}


def stage_hbm_fracs(stage_ms, n, views, batch, kept, pairs, tiles, copy_gb_s=None):
    """Algorithmic HBM bytes of a step's slice + project and binning stages and
    the fraction of the 8 TB/s peak their serial times reach (and of the
    measured copy bandwidth when given).  Slice + project: the 336 B of scene
    parameters read once per launch (the frames of a launch share the scene;
    144 B of the slice's inputs, 192 B of SH coefficients), and per frame the
    68 B a kept Gaussian's splat needs (48 B record, 16 B tile footprint, 4 B
    depth key) and the 4 B key that marks a culled one.  Binning: the depth
    keys read (4 B per Gaussian), the depth sort's 64 B per kept Gaussian (four
    passes, each reading and writing a key and a value), the footprints read
    in depth order (16 B per kept Gaussian), 4 B per pair of the tile lists
    and 8 B per tile range."""
    launches = -(-views // batch)
    out = {}
    sp = 336 * n * launches + 68 * kept + 4 * (n * views - kept)
    bn = 4 * n * views + 64 * kept + 16 * kept + 4 * pairs + 8 * tiles
    for name, b in (("sd7_slice_project", sp), ("sd7_bin", bn)):
        t = stage_ms[name] * 1e-3
        out[name] = {"algorithmic_bytes": int(b), "gb_s": round(b / t / 1e9, 1),
                     "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
        if copy_gb_s:
            out[name]["frac_of_copy"] = round(b / t / 1e9 / copy_gb_s, 4)
    return out


def serial_stage_ms(R, batches, reps):
    """Per-step milliseconds of each stage, one stream, no overlap."""
    import numpy as np
    import torch
    names = ("sd7_slice_project", "sd7_bin", "sd7_rasterize")
    stream = torch.cuda.current_stream()
    ms = {s: [] for s in names}
    torch.cuda.synchronize()
    for _ in range(reps):
        for b in batches:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
            e[0].record(stream)
            for k, s in enumerate(names):
                R.stage(s, b, stream=stream)
                e[k + 1].record(stream)
            torch.cuda.synchronize()
            for k, s in enumerate(names):
                ms[s].append(e[k].elapsed_time(e[k + 1]))
    return {s: round(float(np.mean(v)) * len(batches), 4) for s, v in ms.items()}


def train_bench(a, R, L):
    """The reverse pass in a training step (scenegen.config2: 500,000 Gaussians,
    one 1352x1014 view and its seeded target): per step the forward stages, the
    L1 loss gradient image, the three reverse stages and the Adam update, on one
    stream, each bracketed by HIP events; `train_steps` timed steps after two
    untimed ones."""
    import numpy as np
    import torch

    import scenegen
    from paper_2503_07946_amd.render import Adam, GaussianScene

    scene, views, target = scenegen.config2()
    v = views[0]
    gs = GaussianScene.from_host(scene)
    tgt = torch.as_tensor(target, device="cuda")
    c0 = R.read_counts(R.render(gs, v))
    cap = int(int(c0[0, L.SD7_CNT_NEEDED]) * 1.5) + L.SD7_PAIR_ROUND  # room for the pairs to grow as it trains
    frames = R.make_frames([(gs, v)], need_grad=True)
    fr = frames[0]
    fr.dL_dimage = torch.empty_like(fr.image)
    fr.grads["lambda"] = torch.zeros(2, dtype=torch.float32, device="cuda")
    b = R.batch(frames, cap)
    opt = Adam(gs)
    st = torch.cuda.current_stream()
    tmp = torch.empty_like(fr.image)
    names = ("sd7_slice_project", "sd7_bin", "sd7_rasterize", "loss_gradient",
             "sd7_rasterize_backward", "sd7_project_backward", "sd7_slice_backward", "adam")
    inv = 1.0 / tgt.numel()

    def step(ev):
        k = 0
        for name in names:
            if name == "loss_gradient":  # d(mean |image - target|) / d image
                torch.sub(fr.image, tgt, out=tmp)
                torch.sign(tmp, out=fr.dL_dimage)
                fr.dL_dimage.mul_(inv)
                fr.grads["lambda"].zero_()
            elif name == "adam":
                opt.step(gs, fr.grads)
            else:
                R.stage(name, b, stream=st)
            if ev is not None:
                ev[k].record(st)
            k += 1

    for _ in range(2):
        step(None)
    runs = []
    torch.cuda.synchronize()
    for _ in range(a.train_steps):
        e0 = torch.cuda.Event(enable_timing=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in names]
        e0.record(st)
        step(ev)
        runs.append((e0, ev))
    torch.cuda.synchronize()
    per = {n: [] for n in names}
    total = []
    for e0, ev in runs:
        prev = e0
        for n, e in zip(names, ev):
            per[n].append(prev.elapsed_time(e))
            prev = e
        total.append(e0.elapsed_time(ev[-1]))
    c = R.read_counts(b)
    loss = float((fr.image - tgt).abs().mean())
    stage_ms = {n: round(float(np.mean(x)), 4) for n, x in per.items()}
    return {"workload": "500k 7D Gaussians, one 1352x1014 view, L1 loss against a seeded target, "
                        "forward + reverse pass + Adam per step",
            "ms_per_step": round(float(np.mean(total)), 4), "steps": a.train_steps,
            "stage_ms": stage_ms,
            "pairs": int(c[0, L.SD7_CNT_PAIRS]),
            "overflowed": bool(c[0, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW),
            "l1_loss_after": round(loss, 6)}


def agr_bench(a, R, L, scene, views, streams):
    """The full 7DGS variant: the same scenes and views with adaptive Gaussian
    refinement (Sec. 4.3) before the slice, weights from scenegen.agr_weights(1)."""
    import numpy as np
    import torch

    import scenegen
    from paper_2503_07946_amd.render import GaussianScene

    gs = GaussianScene.from_host(scene, agr=scenegen.agr_weights(1))
    groups = [views[i:i + a.batch] for i in range(0, len(views), a.batch)]
    batches = []
    for gv in groups:
        frames = R.make_frames([(gs, v) for v in gv])
        c = R.read_counts(R.render_frames(frames, exact=True))
        need = int(sum(-(-int(p) // L.SD7_PAIR_ROUND) * L.SD7_PAIR_ROUND for p in c[:, L.SD7_CNT_NEEDED]))
        batches.append(R.batch(frames, int(need * 1.05) + L.SD7_PAIR_ROUND))
    run_steps(R, batches, a.warmup, streams)
    dt, _ = run_steps(R, batches, a.steps, streams)
    over = sum(int(np.sum(R.read_counts(b)[:, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW != 0)) for b in batches)
    return {"value": round(len(views) * a.steps / dt, 2), "unit": "FPS",
            "ms_per_step": round(1e3 * dt / a.steps, 3),
            "stage_ms_per_step": serial_stage_ms(R, batches, 2),
            "overflowed_frames": over, "weights": "scenegen.agr_weights(1)"}


def stress_bench(a, R, L, scene, views, target):
    """The stress workload: 4,000,000 Gaussians with ill-conditioned (t, d)
    blocks, 64 views of 1920x1080, `stress_inflight` views resident at once
    (one set of launches), each followed by the full reverse pass of an L1
    loss against the seeded target.  One untimed pass sizes each group's pair
    arena; the timed pass brackets every stage of every group with HIP events
    on one stream."""
    import numpy as np
    import torch

    from paper_2503_07946_amd.render import GaussianScene, PARAMS

    gs = GaussianScene.from_host(scene)
    tgt = torch.as_tensor(target, device="cuda")
    V = a.stress_inflight
    groups = [views[i:i + V] for i in range(0, len(views), V)]
    grads = [{k: torch.empty_like(getattr(gs, k)) for k in PARAMS} for _ in range(V)]
    for g in grads:
        g["lambda"] = torch.zeros(2, dtype=torch.float32, device="cuda")
    outs = [(torch.empty((3, views[0].H, views[0].W), device="cuda"),
             torch.empty((views[0].H, views[0].W), device="cuda"),
             torch.empty((views[0].H, views[0].W), dtype=torch.int32, device="cuda")) for _ in range(V)]
    # the loss gradient's buffers, one per resident view, made before the timed pass
    dls = [torch.empty((3, views[0].H, views[0].W), device="cuda") for _ in range(V)]
    tmps = [torch.empty((3, views[0].H, views[0].W), device="cuda") for _ in range(V)]
    caps = []
    for gv in groups:   # untimed: exact pair counts per group
        fr = R.make_frames([(gs, v) for v in gv], outputs=outs[:len(gv)])
        c = R.read_counts(R.render_frames(fr, exact=True))
        caps.append(int(sum(-(-int(p) // L.SD7_PAIR_ROUND) * L.SD7_PAIR_ROUND for p in c[:, L.SD7_CNT_NEEDED])))
        torch.cuda.empty_cache()
    cap = int(max(caps) * 1.02) + L.SD7_PAIR_ROUND * V
    # the loss gradient's elementwise kernels load on their first launch (about
    # 0.15 s): launch them once before the timed pass
    torch.sub(outs[0][0], tgt, out=tmps[0])
    torch.sign(tmps[0], out=dls[0])
    dls[0].mul_(1.0 / tgt.numel())
    ws = None
    names = ("sd7_slice_project", "sd7_bin", "sd7_rasterize", "loss_gradient",
             "sd7_rasterize_backward", "sd7_project_backward", "sd7_slice_backward")
    st = torch.cuda.current_stream()
    per = {n: 0.0 for n in names}
    pairs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gv in groups:
        fr = R.make_frames([(gs, v) for v in gv], outputs=outs[:len(gv)])
        for k, f in enumerate(fr):
            f.grads = grads[k]
            f.dL_dimage = dls[k]
        b = R.batch(fr, cap, ws)
        ws = b.ws
        b.cstruct = R.cstruct(fr)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record(st)
        for k, name in enumerate(names):
            if name == "loss_gradient":  # d(mean |image - target|) / d image
                for j, f in enumerate(fr):
                    torch.sub(f.image, tgt, out=tmps[j])
                    torch.sign(tmps[j], out=f.dL_dimage)
                    f.dL_dimage.mul_(1.0 / tgt.numel())
                    f.grads["lambda"].zero_()
            else:
                R.stage(name, b, stream=st)
            ev[k + 1].record(st)
        torch.cuda.synchronize()
        for k, name in enumerate(names):
            per[name] += ev[k].elapsed_time(ev[k + 1])
        c = R.read_counts(b)
        assert not np.any(c[:, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW)
        pairs += c[:, L.SD7_CNT_PAIRS].tolist()
    dt = time.perf_counter() - t0
    nv = len(views)
    stage = {n: round(per[n] / nv, 4) for n in names}
    return {"workload": f"{scene.n // 1000000}M 7D Gaussians (condition number of the (t, d) block up to 1e4), "
                        f"{nv} views {views[0].W}x{views[0].H}, {V} in flight, forward + reverse pass per view",
            "ms_per_view": round(1e3 * dt / nv, 3), "views": nv, "inflight": V,
            "stage_ms_per_view": stage, "largest_stage": max(stage, key=stage.get),
            "pairs_per_view_mean": int(np.mean(pairs))}


def small_bench(R, L, reps: int = 300):
    """The small workload (1,000 Gaussians, one 64x64 view): launch-bound, so
    reported as microseconds per frame: one sd7_render call waited for each
    time (latency), and back-to-back calls (throughput)."""
    import numpy as np
    import torch

    import scenegen
    from paper_2503_07946_amd.render import GaussianScene

    scene, views = scenegen.config0()
    gs = GaussianScene.from_host(scene)
    c = R.read_counts(R.render(gs, views[0]))
    cap = int(c[0, L.SD7_CNT_NEEDED]) + L.SD7_PAIR_ROUND
    frames = R.make_frames([(gs, views[0])])
    b = R.batch(frames, cap)
    G = R.graph(frames, cap)
    out = {"workload": "1,000 7D Gaussians, one 64x64 view per call"}
    for name, call in (("graph", lambda: G.launch()), ("eager", lambda: R.stage("sd7_render", b))):
        for _ in range(20):
            call()
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            call()
            torch.cuda.synchronize()
            lat.append(1e6 * (time.perf_counter() - t0))
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        out[name] = {"latency_us_p50": round(float(np.percentile(lat, 50)), 1),
                     "latency_us_p99": round(float(np.percentile(lat, 99)), 1),
                     "back_to_back_us_per_frame": round(1e6 * (time.perf_counter() - t0) / reps, 1)}
    G.close()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_bench(a, scene1, views1, stress=None):
    """The FP64 CPU oracle (brute force: every visible Gaussian tested at each
    pixel until it stops) on bounded samples of the workloads, with all host
    threads and with one: the throughput workload's centre crops (FPS
    extrapolated to the 800x800 frame, labelled so), the small workload's full
    frame, and 64x64 centre crops of the training and stress workloads,
    forward (C oracle) and reverse (PyTorch FP64 autograd, on the Gaussians
    whose opacity box reaches the crop; the others add nothing there)."""
    import numpy as np
    import torch

    import oracle
    import oracle.grad as og
    import scenegen

    nall = oracle.num_threads()
    W, H = views1[0].W, views1[0].H

    def crop_render(scene, view, crop, nt):
        oracle.set_threads(nt)
        t0 = time.perf_counter()
        o = oracle.render(scene, view, crop=crop, banded=False)
        dt = time.perf_counter() - t0
        tests = int(o.ntest.sum())
        return o, dt, tests

    out = {"cpu_model": cpu_model(), "threads": nall}
    c1 = {}
    for nt, cs in ((nall, a.cpu_crop), (1, 64)):
        crop = ((W - cs) // 2, (H - cs) // 2, cs, cs)
        _, dt, tests = crop_render(scene1, views1[0], crop, nt)
        c1[nt] = {"threads": nt, "crop": [cs, cs], "seconds": round(dt, 3), "pair_tests": tests,
                  "pair_tests_per_s": round(tests / dt, 1),
                  "fps_extrapolated": round(cs * cs / (W * H) / dt, 6)}
    out["throughput_workload"] = c1
    sc0, v0 = scenegen.config0()
    c0 = {}
    for nt in (1, nall):
        crop_render(sc0, v0[0], None, nt)
        _, dt, tests = crop_render(sc0, v0[0], None, nt)
        c0[nt] = {"threads": nt, "ms_per_frame": round(1e3 * dt, 3), "pair_tests_per_s": round(tests / dt, 1)}
    out["small_workload_full_frame"] = c0

    def crop_fwd_bwd(scene, view, target, nt):
        oracle.set_threads(nt)
        torch.set_num_threads(nt)
        crop = ((view.W - 64) // 2, (view.H - 64) // 2, 64, 64)
        t0 = time.perf_counter()
        sl = oracle.slice_(scene, view)
        pr = oracle.project(sl, scene.sh, view)
        x0, y0 = crop[0], crop[1]
        near = np.nonzero(pr.visible & (pr.box[2] >= x0 - 1) & (pr.box[0] <= x0 + 65) &
                          (pr.box[3] >= y0 - 1) & (pr.box[1] <= y0 + 65))[0]
        sub = scene.subset(near)
        o = oracle.render(sub, view, crop=crop, banded=False)
        t1 = time.perf_counter()
        dL = og.l1_grad_image(o.image, target[:, y0:y0 + 64, x0:x0 + 64].astype(np.float64))
        og.grad(sub, view, dL, crop=crop)
        t2 = time.perf_counter()
        return {"threads": nt, "crop": [64, 64], "gaussians_reaching_crop": int(len(near)),
                "forward_s": round(t1 - t0, 3), "reverse_s": round(t2 - t1, 3),
                "pair_tests_per_s": round(int(o.ntest.sum()) / (t1 - t0), 1)}

    sc2, v2, t2 = scenegen.config2()
    out["training_workload_crop"] = crop_fwd_bwd(sc2, v2[0], t2, nall)
    if stress is not None:
        s4, v4, t4 = stress
        out["stress_workload_crop"] = crop_fwd_bwd(s4, v4[0], t4, nall)
    oracle.set_threads(nall)
    torch.set_num_threads(nall)
    return {"value": c1[nall]["fps_extrapolated"], "unit": "FPS", "cores": nall, "kind": "oracle",
            "sample": f"throughput workload: {a.cpu_crop}x{a.cpu_crop} centre crop of view 0 with all {nall} "
                      f"threads (all 200k Gaussians sliced and projected, brute-force compositing), "
                      f"{c1[nall]['seconds']} s; FPS extrapolated to the full 800x800 frame",
            "one_thread": c1[1], **out}


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is described, not built)"}))
        return 2
    if a.copy_probe:
        return copy_probe(a.copy_probe)
    import numpy as np
    import torch

    import scenegen
    from paper_2503_07946_amd import _lib as L
    from paper_2503_07946_amd.render import GaussianScene, get_renderer

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    scene, views = scenegen.config1(a.views, n=a.gaussians)
    W, H = views[0].W, views[0].H
    gs = GaussianScene.from_host(scene, dev)
    R = get_renderer(0)
    stream = torch.cuda.current_stream()
    print(f"[bench] {scene.n} Gaussians, {len(views)} views {W}x{H}, batch {a.batch}", file=sys.stderr, flush=True)

    # -- batches, each with its outputs and a pair arena sized by one exact render
    groups = [views[i:i + a.batch] for i in range(0, len(views), a.batch)]
    batches = []
    for gv in groups:
        frames = R.make_frames([(gs, v) for v in gv])
        b0 = R.render_frames(frames, exact=True)
        c = R.read_counts(b0)
        need = int(sum(-(-int(p) // L.SD7_PAIR_ROUND) * L.SD7_PAIR_ROUND for p in c[:, L.SD7_CNT_NEEDED]))
        cap = int(need * 1.05) + L.SD7_PAIR_ROUND
        batches.append(R.batch(frames, cap))
    torch.cuda.synchronize()

    # default-priority streams the batches of a step alternate over
    streams = [stream] + [torch.cuda.Stream() for _ in range(max(1, a.streams) - 1)]
    run_steps(R, batches, a.warmup, streams)
    dt, raster_ms = run_steps(R, batches, a.steps, streams, record_stage="sd7_rasterize")
    nframes = len(views) * a.steps
    fps = nframes / dt
    # correctness of the timed run: no frame overflowed its arena
    overflow = 0
    pairs = []
    kept = []
    tests = contribs = 0
    evals = 0
    for b in batches:
        c = R.read_counts(b)
        overflow += int(np.sum(c[:, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW != 0))
        pairs += [int(x) for x in c[:, L.SD7_CNT_PAIRS]]
        kept += [int(x) for x in c[:, L.SD7_CNT_KEPT]]
        for f, fr in enumerate(b.frames):
            tests += int(fr.last.to(torch.int64).sum())
            evals += wave_evaluations(fr.last, b.ranges(f), fr.view.W, fr.view.H)
    # contributing (pixel, splat) pairs: one untimed pass with per-pixel counts
    for b in batches:
        fc = R.make_frames([(fr.scene, fr.view) for fr in b.frames], count=True)
        bc = R.batch(fc, b.capacity)
        R.stage("sd7_render", bc)
        contribs += sum(int(fr.ncontrib.to(torch.int64).sum()) for fr in fc)
    per_step_stage = serial_stage_ms(R, batches, 2)
    hbm_copy = copy_bandwidth()
    stage_hbm = stage_hbm_fracs(per_step_stage, scene.n, len(views), a.batch, sum(kept), sum(pairs),
                                len(views) * ((W + 15) // 16) * ((H + 15) // 16), hbm_copy["gb_s"])

    # -- roofline of the dominant kernel (the rasterizer): its launches in the
    # timed region, HIP events on their own stream (other batches' stages run
    # alongside)
    raster_launch_ms = float(np.mean(raster_ms))
    t_r = raster_launch_ms * 1e-3                                  # per batch launch, s
    evals_l = evals / len(batches)
    current = RASTER_SRC_SHA256 is not None and raster_src_digest() == RASTER_SRC_SHA256
    tests_l, contribs_l = tests / len(batches), contribs / len(batches)
    flops_l = RASTER_OPS_PER_TEST * tests_l + RASTER_OPS_PER_CONTRIBUTION * contribs_l
    achieved = flops_l / t_r / 1e12
    roofline = {"bound": "alu", "kernel": "k_raster", "achieved": round(achieved, 3),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "peak_without_packed_fp32": round(FP32_NONPACKED_PEAK_TFLOPS, 2),
                "frac_without_packed_fp32": round(achieved / FP32_NONPACKED_PEAK_TFLOPS, 4),
                "traffic": RASTER_TRAFFIC_BYTES if current else None,
                "algorithmic_units": {"pixel_tests_per_launch": int(tests_l),
                                      "contributions_per_launch": int(contribs_l),
                                      "ops_per_test": RASTER_OPS_PER_TEST,
                                      "ops_per_contribution": RASTER_OPS_PER_CONTRIBUTION,
                                      "fp32_ops_per_launch": int(flops_l),
                                      "wave_evaluations_per_launch": int(evals_l)},
                "counters_current": current,
                "valu_instructions_per_launch": RASTER_VALU_INSTRUCTIONS if current else None,
                "avg_launch_ms": round(raster_launch_ms, 4)}

    # -- latency: batched (frames of a batch finish with their batch) vs plain
    lat_batched = []
    torch.cuda.synchronize()
    for _ in range(2):
        for b in batches:
            s0 = time.perf_counter()
            R.stage("sd7_render", b)
            torch.cuda.synchronize()
            lat_batched += [1e3 * (time.perf_counter() - s0)] * b.nf
    # plain: one frame per call with the pair count learned for this scene and
    # resolution (no read-back inside the frame), waited for; replayed as a
    # captured HIP graph (sd7_graph_launch), and as eager sd7_render calls
    lat_plain, lat_plain_eager = [], []
    cap1 = int(max(pairs) * 1.05) + L.SD7_PAIR_ROUND
    G = R.graph(R.make_frames([(gs, views[0])]), cap1)
    for v in views[:a.plain_frames]:
        s0 = time.perf_counter()
        G.launch(R.make_frames([(gs, v)]))
        torch.cuda.synchronize()
        lat_plain.append(1e3 * (time.perf_counter() - s0))
        s0 = time.perf_counter()
        bp = R.batch(R.make_frames([(gs, v)]), cap1)
        R.stage("sd7_render", bp)
        torch.cuda.synchronize()
        lat_plain_eager.append(1e3 * (time.perf_counter() - s0))
    G.close()
    plain_fps = len(lat_plain) / (sum(lat_plain) / 1e3) if lat_plain else None

    small = small_bench(R, L) if a.small else None
    stress_in = scenegen.config4() if (a.stress or a.cpu_baseline) else None
    stress = stress_bench(a, R, L, *stress_in) if a.stress else None
    torch.cuda.empty_cache()
    # -- FP64 CPU oracle on bounded samples
    cpu = cpu_baseline_bench(a, scene, views, stress_in) if a.cpu_baseline else None
    del stress_in
    serving = serve_bench(a, R, L) if a.serve else None
    agr = agr_bench(a, R, L, scene, views, streams) if a.agr else None
    training = train_bench(a, R, L) if a.train else None

    out = {
        "metric": "rendered FPS and Mpixel/s at 1 GPU; p50/p99 frame latency, batched vs plain",
        "value": round(fps, 2), "unit": "FPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * dt / a.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "200k 7D Gaussians, 50 views 800x800, forward (slice, project, bin, raster)",
                   "gaussians": scene.n, "views": len(views), "resolution": [W, H],
                   "batch": a.batch, "streams": a.streams, "parallelism": "single GPU"},
        "mpixel_per_s": round(fps * W * H / 1e6, 1),
        "latency_ms": {"batched_p50": pct(lat_batched, 50), "batched_p99": pct(lat_batched, 99),
                       "plain_p50": pct(lat_plain, 50), "plain_p99": pct(lat_plain, 99),
                       "plain_eager_p50": pct(lat_plain_eager, 50), "plain_eager_p99": pct(lat_plain_eager, 99),
                       "plain": "one frame per call, waited for: a replayed HIP graph of the render "
                                "(eager: one sd7_render call)"},
        "plain_fps": round(plain_fps, 2) if plain_fps else None,
        "stage_ms_per_step": per_step_stage,
        "pairs_per_view_mean": int(np.mean(pairs)), "kept_per_view_mean": int(np.mean(kept)),
        "overflowed_frames": overflow,
        "stage_hbm": stage_hbm,
        "hbm_copy": hbm_copy,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "agr": agr,
        "training": training,
        "small": small,
        "stress": stress,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
