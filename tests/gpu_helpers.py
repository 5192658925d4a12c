"""Helpers of the GPU parity tests: a CPU re-execution of the integer stage
(depth sort, pair emission, tile sort, ranges) on the GPU's own FP32 outputs,
and oracle-side flags for decisions that FP32 may legitimately take
differently from FP64."""
import numpy as np

import oracle

CULLED = 0xFFFFFFFF


def footprint_rows(rect: np.ndarray):
    """Rows of tile footprints [n, 4] (box, then row trims: word 2 for box rows
    0..3, word 3 for rows m..m+3 with m = h - 4 when h > 8 else 4; byte = left
    | right << 4).  Returns, per (footprint, box row) in footprint-major,
    row-major order: footprint index, tile row y, first tile a, end tile b
    (a >= b: empty row)."""
    r = rect.astype(np.uint32).astype(np.int64)
    x0, y0 = r[:, 0] & 0xFFFF, r[:, 0] >> 16
    x1, y1 = r[:, 1] & 0xFFFF, r[:, 1] >> 16
    h = np.maximum(y1 - y0, 0)
    gi = np.repeat(np.arange(len(r)), h)
    rr = np.arange(int(h.sum())) - np.repeat(np.cumsum(h) - h, h)
    hh = h[gi]
    m = np.where(hh > 8, hh - 4, 4)
    top = (r[gi, 2] >> (8 * np.clip(rr, 0, 3))) & 0xFF
    bot = (r[gi, 3] >> (8 * np.clip(rr - m, 0, 3))) & 0xFF
    byte = np.where(rr < 4, top, np.where(rr >= m, bot, 0))
    return gi, y0[gi] + rr, x0[gi] + (byte & 15), x1[gi] - (byte >> 4)


def cpu_bin(depth_key: np.ndarray, rect: np.ndarray, tiles_x: int, tiles: int):
    """Reference integer stage: kept Gaussians ordered by (key, index); pairs
    emitted over each footprint's tiles in that order; stable sort by tile."""
    dk = depth_key.astype(np.uint32)
    kept = np.nonzero(dk != CULLED)[0]
    order = kept[np.lexsort((kept, dk[kept]))]
    gi, y, a, b = footprint_rows(rect[order])
    w = np.maximum(b - a, 0)
    P = int(w.sum())
    rep = np.repeat(np.arange(len(w)), w)
    loc = np.arange(P) - np.repeat(np.cumsum(w) - w, w)
    tile = y[rep] * tiles_x + a[rep] + loc
    g = order[gi[rep]]
    idx = np.argsort(tile, kind="stable")
    tile, g = tile[idx], g[idx]
    ranges = np.zeros((tiles, 2), np.int64)
    if P:
        starts = np.nonzero(np.r_[True, tile[1:] != tile[:-1]])[0]
        ends = np.r_[starts[1:], P]
        ranges[tile[starts], 0] = starts
        ranges[tile[starts], 1] = ends
    return order, tile, g, ranges


def tile_reached(sl, pr, view, g, tx, ty, chunk=4096):
    """Per (Gaussian g, tile (tx, ty)): whether the oracle's opacity
    alpha_c exp(-q/2) reaches 1/255 at a pixel centre of the tile inside the
    image (FP64)."""
    g, tx, ty = (np.asarray(x, np.int64) for x in (g, tx, ty))
    off = np.arange(16) + 0.5
    out = np.zeros(len(g), bool)
    for s0 in range(0, len(g), chunk):
        sl_ = slice(s0, s0 + chunk)
        px = tx[sl_, None] * 16 + off[None, :]
        py = ty[sl_, None] * 16 + off[None, :]
        dx = (px - pr.mean2d[0][g[sl_], None])[:, None, :]
        dy = (py - pr.mean2d[1][g[sl_], None])[:, :, None]
        ca, cb, cc = (pr.conic[i][g[sl_], None, None] for i in range(3))
        q = ca * dx * dx + 2 * cb * dx * dy + cc * dy * dy
        al = sl.alpha_c[g[sl_], None, None] * np.exp(-0.5 * q)
        inside = (px[:, None, :] < view.W) & (py[:, :, None] < view.H)
        out[sl_] = ((al >= oracle.ALPHA_MIN) & inside).any(axis=(1, 2))
    return out


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
