"""Helpers of the GPU parity tests: a CPU re-execution of the integer stage
(depth sort, pair emission, tile sort, ranges) on the GPU's own FP32 outputs,
and oracle-side flags for decisions that FP32 may legitimately take
differently from FP64."""
import numpy as np

import oracle

CULLED = 0xFFFFFFFF


def cpu_bin(depth_key: np.ndarray, rect: np.ndarray, tiles_x: int, tiles: int):
    """Reference integer stage: kept Gaussians ordered by (key, index); pairs
    emitted row-major over each rect in that order; stable sort by tile."""
    dk = depth_key.astype(np.uint32)
    kept = np.nonzero(dk != CULLED)[0]
    order = kept[np.lexsort((kept, dk[kept]))]
    r = rect.astype(np.uint32)
    x0 = (r[order, 0] & 0xFFFF).astype(np.int64)
    y0 = (r[order, 0] >> 16).astype(np.int64)
    x1 = (r[order, 1] & 0xFFFF).astype(np.int64)
    y1 = (r[order, 1] >> 16).astype(np.int64)
    w = x1 - x0
    cnt = w * (y1 - y0)
    off = np.concatenate([[0], np.cumsum(cnt)])
    P = int(off[-1])
    rep = np.repeat(np.arange(len(order)), cnt)
    loc = np.arange(P) - off[rep]
    tile = (y0[rep] + loc // w[rep]) * tiles_x + x0[rep] + loc % w[rep]
    g = order[rep]
    idx = np.argsort(tile, kind="stable")
    tile, g = tile[idx], g[idx]
    ranges = np.zeros((tiles, 2), np.int64)
    if P:
        starts = np.nonzero(np.r_[True, tile[1:] != tile[:-1]])[0]
        ends = np.r_[starts[1:], P]
        ranges[tile[starts], 0] = starts
        ranges[tile[starts], 1] = ends
    return order, tile, g, ranges


def slice_tolerance(ora: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """4 FP32 ulp of the oracle value, or 2e-7 of the per-Gaussian scale."""
    ulp = np.spacing(np.abs(ora).astype(np.float32)).astype(np.float64)
    return np.maximum(4 * ulp, 2e-7 * scale)


def oracle_rect_flags(sl, pr, view, eps=1e-4):
    """Gaussians whose visibility or tile box may differ in FP32: alpha_c or z
    near a threshold, or a footprint edge within eps tiles of a boundary."""
    ac = sl.alpha_c
    flag = np.abs(ac - oracle.ALPHA_MIN) < 1e-5 * oracle.ALPHA_MIN
    a, b, c = pr.conic
    det = a * c - b * b
    with np.errstate(all="ignore"):
        s00 = c / det
        s11 = a / det
        k = 2 * np.log(np.maximum(ac, 1e-300) / oracle.ALPHA_MIN)
        hx = np.sqrt(np.maximum(k * s00, 0))
        hy = np.sqrt(np.maximum(k * s11, 0))
        u, v = pr.mean2d
        for e in ((u - hx) / 16, (u + hx) / 16, (v - hy) / 16, (v + hy) / 16):
            flag |= pr.visible & (np.abs(e - np.round(e)) < eps)
    return flag


def image_check(gpu_img, ora, tol=1e-4):
    """max |gpu - oracle| over unflagged pixels; returns (err, n_flagged)."""
    mask = ora.flags == 0
    err = np.abs(gpu_img.astype(np.float64) - ora.image)
    return float(err[:, mask].max()) if mask.any() else 0.0, int((~mask).sum())
