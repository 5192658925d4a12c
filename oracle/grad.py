"""Gradient reference of the 7DGS render path -- TEST INFRASTRUCTURE.

The forward is written a second time with plain PyTorch CPU FP64 ops so that
autograd yields the exact derivative of the plain definition.  It shares no
code with ``oracle7d.c`` (the two forwards are checked against each other) and
none with the HIP library.

Steps, in the paper's order:
  Sec. 4.1  Sigma = L L^T from the packed lower-triangular L.
  Sec. 4.2  mu_cond = mu_p + Sigma_PQ Sigma_QQ^{-1} r           (eq. cond_mean)
            Sigma_cond = Sigma_PP - Sigma_PQ Sigma_QQ^{-1} Sigma_QP (eq. cond_cov)
            f_temp, f_dir (eq. temp_mod, eq. dir_mod), alpha_cond = alpha f_temp f_dir
  Sec. 4.4  perspective (EWA) projection, SH colour (Sec. 3, eq. 2),
            depth-ordered front-to-back alpha compositing.
Discrete decisions (culling, the alpha and transmittance thresholds, clamps,
order) are taken on detached values; gradients flow through the values of the
branch that was taken (a clamped branch has zero gradient).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import ALPHA_MAX, ALPHA_MIN, DILATION, JCLAMP, T_MIN, TILE, Z_NEAR

PARAMS = ("mu_p", "mu_t", "mu_d", "L", "alpha", "sh")


def _tri(i, j):
    return i * (i + 1) // 2 + j


_SEL = torch.zeros(28, 49, dtype=torch.float64)
for _i in range(7):
    for _j in range(_i + 1):
        _SEL[_tri(_i, _j), _i * 7 + _j] = 1.0


def scene_tensors(scene, requires_grad=True) -> dict:
    out = {}
    for k in PARAMS:
        t = torch.tensor(np.asarray(getattr(scene, k), np.float32), dtype=torch.float64)
        out[k] = t.requires_grad_(requires_grad)
    return out


def sh_basis(x, y, z):
    """Real degree-3 SH basis (k = l*l + l + m, (-1)^|m| signs), closed forms."""
    pi = math.pi
    c1 = math.sqrt(3 / (4 * pi))
    return torch.stack([
        torch.full_like(x, 0.5 / math.sqrt(pi)),
        -c1 * y, c1 * z, -c1 * x,
        0.5 * math.sqrt(15 / pi) * x * y,
        -0.5 * math.sqrt(15 / pi) * y * z,
        0.25 * math.sqrt(5 / pi) * (2 * z * z - x * x - y * y),
        -0.5 * math.sqrt(15 / pi) * x * z,
        0.25 * math.sqrt(15 / pi) * (x * x - y * y),
        -0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y),
        0.5 * math.sqrt(105 / pi) * x * y * z,
        -0.25 * math.sqrt(21 / (2 * pi)) * y * (4 * z * z - x * x - y * y),
        0.25 * math.sqrt(7 / pi) * z * (2 * z * z - 3 * x * x - 3 * y * y),
        -0.25 * math.sqrt(21 / (2 * pi)) * x * (4 * z * z - x * x - y * y),
        0.25 * math.sqrt(105 / pi) * z * (x * x - y * y),
        -0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),
    ], dim=0)


def slice_t(P: dict, view):
    """Conditional mean, covariance (full 3x3) and opacity, Sec. 4.2.  The
    modulation strengths are P["lambda_t"], P["lambda_d"] when present (so
    that they can be differentiated), else the view's."""
    n = P["mu_t"].shape[0]
    Ld = (P["L"].T @ _SEL).reshape(n, 7, 7)
    S = Ld @ Ld.transpose(1, 2)
    SPP, SPQ, SQQ = S[:, :3, :3], S[:, :3, 3:], S[:, 3:, 3:]
    if getattr(view, "d_per_gaussian", False):
        c = torch.tensor(np.asarray(view.c, np.float32), dtype=torch.float64)
        e = P["mu_p"].T - c[None, :]
        d = e / torch.sqrt((e * e).sum(1, keepdim=True))              # [n,3]
    else:
        d = torch.tensor(np.asarray(view.d, np.float32), dtype=torch.float64)[None, :]
    r = torch.cat([(float(view.t) - P["mu_t"])[:, None], d - P["mu_d"].T], dim=1)  # [n,4]
    lam_t = P.get("lambda_t", float(view.lambda_t))
    lam_d = P.get("lambda_d", float(view.lambda_d))
    Kt = torch.linalg.solve(SQQ, SPQ.transpose(1, 2))          # Sigma_QQ^{-1} Sigma_QP
    mu_c = P["mu_p"].T + (SPQ @ torch.linalg.solve(SQQ, r[:, :, None]))[:, :, 0]
    Sc = SPP - SPQ @ Kt
    Sc = 0.5 * (Sc + Sc.transpose(1, 2))
    f_t = torch.exp(-0.5 * lam_t * r[:, 0] ** 2 / S[:, 3, 3])
    dl = r[:, 1:]
    SDD = S[:, 4:, 4:]
    qd = (dl[:, None, :] @ torch.linalg.solve(SDD, dl[:, :, None]))[:, 0, 0]
    f_d = torch.exp(-0.5 * lam_d * qd)
    alpha_c = P["alpha"] * f_t * f_d
    return mu_c, Sc, alpha_c


def project_t(mu_c, Sc, alpha_c, sh, view):
    """Perspective/EWA projection + SH colour, Sec. 4.4.  Returns differentiable
    mean2d [n,2], conic [n,3], depth [n], rgb [n,3] and a detached visibility
    mask plus the footprint boxes (pixel units) used for crop pre-filtering."""
    f64 = torch.float64
    R = torch.tensor(np.asarray(view.R_wc, np.float32), dtype=f64).reshape(3, 3)
    c = torch.tensor(np.asarray(view.c, np.float32), dtype=f64)
    fx, fy, cx, cy = (float(view.fx), float(view.fy), float(view.cx), float(view.cy))
    limx = JCLAMP * (0.5 * view.W) / fx
    limy = JCLAMP * (0.5 * view.H) / fy
    dm = mu_c - c[None, :]
    x = dm @ R.T
    z = x[:, 2]
    zs = torch.where(z > Z_NEAR, z, torch.ones_like(z))   # avoid 0-division on culled
    u = fx * x[:, 0] / zs + cx
    v = fy * x[:, 1] / zs + cy
    rx = x[:, 0] / zs
    ry = x[:, 1] / zs
    rx = torch.where(rx >= limx, torch.full_like(rx, limx), torch.where(rx <= -limx, torch.full_like(rx, -limx), rx))
    ry = torch.where(ry >= limy, torch.full_like(ry, limy), torch.where(ry <= -limy, torch.full_like(ry, -limy), ry))
    zero = torch.zeros_like(zs)
    J = torch.stack([torch.stack([fx / zs, zero, -fx * rx / zs], 1),
                     torch.stack([zero, fy / zs, -fy * ry / zs], 1)], 1)   # [n,2,3]
    M = J @ R[None]
    S2 = M @ Sc @ M.transpose(1, 2)
    s00 = S2[:, 0, 0] + DILATION
    s11 = S2[:, 1, 1] + DILATION
    s01 = 0.5 * (S2[:, 0, 1] + S2[:, 1, 0])
    det = s00 * s11 - s01 * s01
    dets = torch.where(det > 0, det, torch.ones_like(det))
    conic = torch.stack([s11 / dets, -s01 / dets, s00 / dets], 1)
    ln = torch.sqrt((dm * dm).sum(1))
    dirn = dm / ln[:, None]
    Y = sh_basis(dirn[:, 0], dirn[:, 1], dirn[:, 2])            # [16,n]
    shv = sh.reshape(16, 3, -1)                                   # [k][ch][n]
    raw = (shv * Y[:, None, :]).sum(0) + 0.5                      # [3,n]
    rgb = torch.where(raw > 0, raw, torch.zeros_like(raw)).T      # [n,3]
    with torch.no_grad():
        ac = alpha_c.detach()
        vis = (ac >= ALPHA_MIN) & (z.detach() > Z_NEAR) & (det.detach() > 0)
        k = 2.0 * torch.log(torch.clamp(ac, min=1e-300) / ALPHA_MIN)
        hx = torch.sqrt(torch.clamp(k * s00.detach(), min=0))
        hy = torch.sqrt(torch.clamp(k * s11.detach(), min=0))
        tiles_x = (view.W + TILE - 1) // TILE
        tiles_y = (view.H + TILE - 1) // TILE
        ud, vd = u.detach(), v.detach()
        tx0 = torch.clamp(torch.floor((ud - hx) / TILE), min=0)
        tx1 = torch.clamp(torch.floor((ud + hx) / TILE), max=tiles_x - 1)
        ty0 = torch.clamp(torch.floor((vd - hy) / TILE), min=0)
        ty1 = torch.clamp(torch.floor((vd + hy) / TILE), max=tiles_y - 1)
        vis &= (tx0 <= tx1) & (ty0 <= ty1)
        box = torch.stack([ud - hx, vd - hy, ud + hx, vd + hy], 1)
    return torch.stack([u, v], 1), conic, z, rgb, vis, box


def render_t(P: dict, view, crop=None, chunk_rows: int = 16):
    """Differentiable FP64 render of the crop (x0, y0, w, h): image [3,h,w]."""
    mu_c, Sc, alpha_c = slice_t(P, view)
    return render_sliced_t(mu_c, Sc, alpha_c, P["sh"], view, crop, chunk_rows)


def render_sliced_t(mu_c, Sc, alpha_c, sh, view, crop=None, chunk_rows: int = 16):
    """Projection and compositing (Sec. 4.4) of sliced Gaussians: image [3,h,w]
    of the crop (x0, y0, w, h)."""
    mean2d, conic, depth, rgb, vis, box = project_t(mu_c, Sc, alpha_c, sh, view)
    return render_splats_t(mean2d, conic, alpha_c, rgb, depth, vis, box, view, crop, chunk_rows)


def render_splats_t(mean2d, conic, alpha_c, rgb, depth, vis, box, view, crop=None, chunk_rows: int = 16):
    """Front-to-back compositing (Sec. 4.4) of projected splats: image [3,h,w]
    of the crop (x0, y0, w, h)."""
    x0, y0, w, h = crop if crop is not None else (0, 0, view.W, view.H)
    with torch.no_grad():
        # Gaussians whose footprint box holds no pixel centre of the crop have
        # alpha < ALPHA_MIN at every crop pixel and contribute nothing.
        inside = (box[:, 2] >= x0 - 1) & (box[:, 0] <= x0 + w + 1) & \
                 (box[:, 3] >= y0 - 1) & (box[:, 1] <= y0 + h + 1)
        sel = torch.nonzero(vis & inside)[:, 0].numpy()
        zs = depth.detach().numpy()[sel]
        sel = sel[np.lexsort((sel, zs))]            # (depth, index) order
    idx = torch.as_tensor(sel, dtype=torch.long)
    m2, cn, ac, col = mean2d[idx], conic[idx], alpha_c[idx], rgb[idx]
    bg = torch.tensor(np.asarray(view.bg, np.float32), dtype=torch.float64)
    rows = []
    for r0 in range(0, h, chunk_rows):
        r1 = min(h, r0 + chunk_rows)
        py, px = torch.meshgrid(torch.arange(y0 + r0, y0 + r1, dtype=torch.float64) + 0.5,
                                torch.arange(x0, x0 + w, dtype=torch.float64) + 0.5, indexing="ij")
        px, py = px.reshape(-1, 1), py.reshape(-1, 1)
        dx = m2[None, :, 0] - px
        dy = m2[None, :, 1] - py
        q = cn[None, :, 0] * dx * dx + 2 * cn[None, :, 1] * dx * dy + cn[None, :, 2] * dy * dy
        araw = ac[None, :] * torch.exp(-0.5 * q)
        a = torch.where(araw >= ALPHA_MAX, torch.full_like(araw, ALPHA_MAX), araw)
        with torch.no_grad():
            pas = a >= ALPHA_MIN
            ap = torch.where(pas, a, torch.zeros_like(a))
            Tn = torch.cumprod(1 - ap, dim=1)
            stop = pas & (Tn < T_MIN)
            incl = pas & (torch.cumsum(stop.to(torch.int64), dim=1) == 0)
        ai = torch.where(incl, a, torch.zeros_like(a))
        one_m = 1 - ai
        Tinc = torch.cumprod(one_m, dim=1)
        Texc = torch.cat([torch.ones_like(Tinc[:, :1]), Tinc[:, :-1]], dim=1)
        wgt = ai * Texc
        C = wgt @ col                                  # [npx,3]
        Tf = Tinc[:, -1] if Tinc.shape[1] else torch.ones(px.shape[0], dtype=torch.float64)
        img = C + Tf[:, None] * bg[None, :]
        rows.append(img.T.reshape(3, r1 - r0, w))
    return torch.cat(rows, dim=1)


def grad(scene, view, dL_dimage: np.ndarray, crop=None):
    """Vector-Jacobian product of the render with dL_dimage [3,h,w]:
    returns ({param: FP64 gradient array of the parameter's shape, plus
    "lambda": [dL/dlambda_t, dL/dlambda_d]}, image)."""
    P = scene_tensors(scene)
    for k in ("lambda_t", "lambda_d"):
        P[k] = torch.tensor(float(getattr(view, k)), dtype=torch.float64, requires_grad=True)
    img = render_t(P, view, crop)
    g = torch.tensor(np.asarray(dL_dimage), dtype=torch.float64)
    (img * g).sum().backward()
    out = {k: P[k].grad.numpy().copy() for k in PARAMS}
    out["lambda"] = np.array([float(P["lambda_t"].grad), float(P["lambda_d"].grad)])
    return out, img.detach().numpy()


def l1_grad_image(image: np.ndarray, target: np.ndarray) -> np.ndarray:
    """d/dC of mean |C - target| over all 3HW entries, with sign(0) = 0."""
    return np.sign(image - target) / image.size


SPLAT = ("u", "v", "a", "b", "c", "alpha_c", "r", "g", "b_")   # splat parameters, in d_splat order
SPLAT_GROUPS = ((0, 2), (2, 5), (5, 6), (6, 9))   # mean2d, conic, opacity, colour


def grad_splats(scene, view, dL_dimage: np.ndarray, crop=None) -> np.ndarray:
    """Gradient of <dL, image> with respect to each Gaussian's splat (Sec. 4.4),
    [9][n]: mean2d (u, v), conic (a, b, c) of q = a dx^2 + 2 b dx dy + c dy^2,
    the conditional opacity, and the (clamped) colour."""
    P = scene_tensors(scene, requires_grad=False)
    mu_c, Sc, alpha_c = slice_t(P, view)
    mean2d, conic, depth, rgb, vis, box = project_t(mu_c, Sc, alpha_c, P["sh"], view)
    leaves = [x.detach().requires_grad_(True) for x in (mean2d, conic, alpha_c, rgb)]
    img = render_splats_t(*leaves[:2], leaves[2], leaves[3], depth.detach(), vis, box, view, crop)
    (img * torch.tensor(np.asarray(dL_dimage), dtype=torch.float64)).sum().backward()
    m, c, a, r = (x.grad for x in leaves)
    return np.concatenate([m.numpy().T, c.numpy().T, a.numpy()[None], r.numpy().T], 0)


def splat_jacobian(scene, view) -> dict:
    """Jacobian of each Gaussian's splat (the 9 values of grad_splats, through
    the slice and the projection) with respect to its own parameters, by one
    reverse pass per splat value (the splat of Gaussian i depends only on the
    parameters of Gaussian i): {param: [9][planes][n]}.  Zero for culled
    Gaussians' clamped branches as in the forward."""
    P = scene_tensors(scene)
    mu_c, Sc, alpha_c = slice_t(P, view)
    mean2d, conic, depth, rgb, vis, box = project_t(mu_c, Sc, alpha_c, P["sh"], view)
    outs = [mean2d[:, 0], mean2d[:, 1], conic[:, 0], conic[:, 1], conic[:, 2], alpha_c,
            rgb[:, 0], rgb[:, 1], rgb[:, 2]]
    n = scene.n
    J = {k: np.zeros((len(SPLAT), 1 if P[k].dim() == 1 else P[k].shape[0], n)) for k in PARAMS}
    for j, y in enumerate(outs):
        gs = torch.autograd.grad(y.sum(), [P[k] for k in PARAMS], retain_graph=True, allow_unused=True)
        for k, gk in zip(PARAMS, gs):
            if gk is not None:
                J[k][j] = gk.numpy().reshape(J[k].shape[1], n)
    return J
