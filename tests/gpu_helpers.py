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
    """Every pixel is compared: |gpu - oracle| <= tol + fbound + vbound, where
    fbound is the oracle's bound on the first-order change of the pixel should
    an FP32 evaluation take one of its in-band decisions (opacity test, stop,
    depth order) the other way (0 on pixels without such a decision), and
    vbound its bound on the first-order change when every contributor's
    opacity moves within its FP32 band (decisions kept).  Returns (max over
    all pixels of |gpu - oracle| - fbound - vbound, number of flagged
    pixels)."""
    err = np.abs(gpu_img.astype(np.float64) - ora.image).max(0)
    return float((err - ora.fbound - ora.vbound).max()), int((ora.flags != 0).sum())


def grad_entry_error(gpu: np.ndarray, ora: np.ndarray) -> np.ndarray:
    """Per-entry gradient error |g_gpu - g_ora| / max(|g_ora|, 1e-2 max|g_ora|)
    (the bar is 1e-3)."""
    scale = np.maximum(np.abs(ora), 1e-2 * np.abs(ora).max())
    return np.abs(gpu - ora) / np.maximum(scale, 1e-300)


SPLAT_GROUPS = ((0, 2), (2, 5), (5, 6), (6, 9))   # mean2d, conic, opacity, colour
SPLAT_GROUP_NAMES = ("d_mean2d", "d_conic", "d_opacity", "d_rgb")


def splat_grads(b, f):
    """The GPU's gradients with respect to frame f's splats, [9][n] (the
    reverse compositing's output: u, v, a, b, c, opacity, r, g, b)."""
    return b.planes("off_d_splat", 9, f).cpu().numpy().astype(np.float64)


def check_gradients(g_gpu: dict, d_gpu: np.ndarray, g_ora: dict, d_ora: np.ndarray, J: dict, bar=1e-3) -> dict:
    """The gradient parity bar (Sec. 4.4 reverse pass).

    * Splat gradients (the sums over pixels the reverse compositing
      accumulates in FP32): per entry |d_gpu - d_ora| <= bar max(|d_ora|,
      1e-2 max of its group).
    * Parameter gradients: per group relative L2 <= bar; per entry
      |g_gpu - g_ora| <= max(bar max(|g_ora|, 1e-2 max|g_ora|), prop), where
      prop = bar (|J|^T s)_entry propagates the splat bar s through the
      magnitudes of the Jacobian J of projection and slice (both reverses are
      linear in the splat gradients and run in FP64, so an error within the
      bar there moves a parameter gradient by at most prop; prop exceeds the
      plain bar only where the 2D covariance or the (t, d) block is
      ill-conditioned).
    Returns the measured figures."""
    rep = {}
    sd = np.abs(d_ora).copy()
    for a, c in SPLAT_GROUPS:
        sd[a:c] = np.maximum(sd[a:c], 1e-2 * np.abs(d_ora[a:c]).max())
    e_d = np.abs(d_gpu - d_ora) / np.maximum(sd, 1e-300)
    for name, (a, c) in zip(SPLAT_GROUP_NAMES, SPLAT_GROUPS):
        rep[name] = float(e_d[a:c].max())
    for k, go in g_ora.items():
        if k == "lambda":
            continue
        a = np.asarray(g_gpu[k], np.float64).reshape(go.shape)
        err = np.abs(a - go)
        plain = bar * np.maximum(np.abs(go), 1e-2 * np.abs(go).max())
        prop = bar * np.einsum("jpn,jn->pn", np.abs(J[k]), sd).reshape(go.shape)
        tol = np.maximum(plain, prop)
        rep[k] = {"rel_l2": float(np.linalg.norm(a - go) / max(np.linalg.norm(go), 1e-30)),
                  "worst_entry": float((err / np.maximum(plain, 1e-300) * bar).max()),
                  "of_bound": float((err / np.maximum(tol, 1e-300)).max()),
                  "entries_over_plain_bar": int((err > plain).sum())}
    assert max(rep[x] for x in SPLAT_GROUP_NAMES) <= bar, rep
    for k, r in rep.items():
        if isinstance(r, dict):
            assert r["rel_l2"] <= bar and r["of_bound"] <= 1.0, (k, rep)
    return rep


def flag_cap(npx: int) -> float:
    """Largest accepted number of flagged pixels: 0.5 % (at least 2)."""
    return max(2.0, 0.005 * npx)


# The FP32 error scales of the refined (AGR) path, for the oracle's decision
# bands: twice the largest relative errors measured against the oracle, in
# units of 2^-24 (mu_cond 2.4e-6 of its scale through mean2d, x sqrt 3;
# Sigma_cond 1.5e-6; alpha_cond 1.9e-5: FP32 sums of up to 64 products in the
# refinement's MLPs).
AGR_FLAGS = dict(k_mu=2 * 1.7321 * 2.4e-6 * 2 ** 24, k_s=2 * 1.5e-6 * 2 ** 24, k_ac=2 * 1.9e-5 * 2 ** 24)
