"""FP64 reference ("oracle") of the 7DGS render path -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library and must never be
used as a fallback for it.

Two independent implementations live here:
  * ``oracle7d.c`` (loaded through ctypes): slice (Sec. 4.2, Schur complement),
    EWA projection and brute-force compositing (Sec. 4.4), FP64.
  * ``oracle.grad``: the same forward written with plain PyTorch CPU FP64 ops,
    differentiated by autograd; it is the gradient reference.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle7d.so")
SRC = os.path.join(HERE, "oracle7d.c")

ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))
Z_NEAR = float(np.float32(0.2))
DILATION = float(np.float32(0.3))
JCLAMP = float(np.float32(1.3))
TILE = 16


def build(force: bool = True) -> str:
    """Compile oracle7d.c with gcc (-O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", "-Wall", "-o", tmp, SRC,
                               "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OraView(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("c", ctypes.c_float * 3),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("W", ctypes.c_int32), ("H", ctypes.c_int32),
                ("t", ctypes.c_float), ("d", ctypes.c_float * 3),
                ("lambda_t", ctypes.c_float), ("lambda_d", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("d_mode", ctypes.c_int32)]


class OraFlagCfg(ctypes.Structure):
    _fields_ = [("k_mu", ctypes.c_double), ("k_uv", ctypes.c_double), ("k_s", ctypes.c_double),
                ("k_eval", ctypes.c_double), ("k_ac", ctypes.c_double), ("k_T", ctypes.c_double),
                ("k_z", ctypes.c_double),
                ("impact_min", ctypes.c_double)]


# The parity protocol's model of an FP32 evaluation of the path (oracle7d.h,
# ora_flagcfg): coefficients, in units of 2^-24, of the error terms that set
# each decision's band.  The opacity-test coefficients are the smallest (on a
# grid of powers of two) under which every exponent error measured on the
# MI355X path near the threshold stays below half its band (small, correlated,
# 200k-, 500k- and 4M-Gaussian workloads, 175k samples); k_ac is one rounding
# of alpha_cond, twice; k_T one fused multiply-add per step, four times;
# k_z = 2 bounds the depth error of FP32-rounded conditional means,
# 2^-24 (sqrt(3) max|mu_c| + z), outright.
DEFAULT_FLAGS = dict(k_mu=1.0, k_uv=2.0, k_s=1.0, k_eval=2.0, k_ac=2.0, k_T=4.0, k_z=2.0, impact_min=1e-5)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.ora_slice.argtypes = [i64, P, P, P, P, P, ctypes.POINTER(OraView), P, P, P, P, P, P]
        L.ora_slice.restype = ctypes.c_int
        L.ora_project.argtypes = [i64, P, P, P, P, ctypes.POINTER(OraView), P, P, P, P, P, P, P]
        L.ora_project.restype = i64
        L.ora_order.argtypes = [i64, P, P, P]
        L.ora_order.restype = i64
        L.ora_fp32_model.argtypes = [i64, P, P, ctypes.POINTER(OraView), P]
        L.ora_fp32_model.restype = None
        L.ora_composite.argtypes = [i64, P, P, P, P, P, P, i64, P, ctypes.POINTER(OraView),
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(OraFlagCfg), P, P, P, P, P, P, P, P]
        L.ora_composite.restype = ctypes.c_int
        L.ora_render.argtypes = [i64, P, P, P, P, P, P, ctypes.POINTER(OraView),
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(OraFlagCfg), P, P, P, P, P, P, P, P]
        L.ora_render.restype = ctypes.c_int
        L.ora_sh_basis.argtypes = [ctypes.c_double] * 3 + [P]
        L.ora_agr_encoding.argtypes = [ctypes.c_double, P]
        L.ora_agr.argtypes = [i64, P, P, P, P, ctypes.c_double, P, P, P, P, P]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    """Exact promotion of the FP32 scene planes (FP64 input passes through)."""
    a = np.asarray(a)
    if a.dtype != np.float64:
        a = np.asarray(a, np.float32).astype(np.float64)
    return np.ascontiguousarray(a)


def ora_view(v) -> OraView:
    o = OraView()
    o.R[:] = [float(x) for x in np.asarray(v.R_wc, np.float32).reshape(9)]
    o.c[:] = [float(x) for x in np.asarray(v.c, np.float32)]
    o.fx, o.fy, o.cx, o.cy = v.fx, v.fy, v.cx, v.cy
    o.W, o.H = v.W, v.H
    o.t = v.t
    o.d[:] = [float(x) for x in np.asarray(v.d, np.float32)]
    o.lambda_t, o.lambda_d = v.lambda_t, v.lambda_d
    o.bg[:] = [float(x) for x in np.asarray(v.bg, np.float32)]
    o.d_mode = 1 if getattr(v, "d_per_gaussian", False) else 0
    return o


def flagcfg(**kw) -> OraFlagCfg:
    d = dict(DEFAULT_FLAGS)
    d.update(kw)
    return OraFlagCfg(**d)


def set_threads(n: int) -> None:
    lib().ora_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().ora_num_threads())


@dataclass
class Sliced:
    mu_c: np.ndarray      # [3][n]
    cov_c: np.ndarray     # [6][n]
    alpha_c: np.ndarray   # [n]
    f_temp: np.ndarray
    f_dir: np.ndarray
    status: np.ndarray


# ---- adaptive Gaussian refinement (Sec. 4.3) --------------------------------
AGR_K = 10
AGR_IN = 27
AGR_HIDDEN = 64
AGR_OUT = (3, 1, 3, 28)          # MLPs for mu_p, mu_t, mu_d, the packed L
AGR_WEIGHTS = sum(AGR_HIDDEN * AGR_IN + AGR_HIDDEN + c * AGR_HIDDEN + c for c in AGR_OUT)


def agr_encoding(t: float) -> np.ndarray:
    """gamma(t): sin(2^k pi t), cos(2^k pi t) for k = 0 .. 9, interleaved."""
    g = np.zeros(2 * AGR_K)
    lib().ora_agr_encoding(float(t), _p(g))
    return g


@dataclass
class Refined:
    """A scene with AGR-refined means and factor (FP64), other fields as given."""
    n: int
    mu_p: np.ndarray
    mu_t: np.ndarray
    mu_d: np.ndarray
    L: np.ndarray
    alpha: np.ndarray
    sh: np.ndarray


def agr(scene, t: float, weights) -> Refined:
    """mu_p + phi_p(f), mu_t + phi_t(f), mu_d + phi_d(f), l + phi_l(f) with
    f = mu_p (+) mu_t (+) mu_d (+) gamma(t) (Sec. 4.3; Algorithm 1 steps 1-2).
    weights: AGR_WEIGHTS values, MLPs p, t, d, l, each W1[64][27], b1[64],
    W2[C_out][64], b2[C_out]."""
    n = scene.n
    w = _f64(np.asarray(weights).reshape(-1))
    assert w.size == AGR_WEIGHTS
    arrs = [_f64(scene.mu_p), _f64(scene.mu_t), _f64(scene.mu_d), _f64(scene.L)]
    out = [np.zeros((3, n)), np.zeros(n), np.zeros((3, n)), np.zeros((28, n))]
    lib().ora_agr(n, *[_p(a) for a in arrs], float(t), _p(w), *[_p(o) for o in out])
    return Refined(n, out[0], out[1], out[2], out[3], scene.alpha, scene.sh)


def slice_(scene, view, agr_weights=None) -> Sliced:
    if agr_weights is not None:
        scene = agr(scene, view.t, agr_weights)
    n = scene.n
    mu_c = np.zeros((3, n)); cov_c = np.zeros((6, n)); ac = np.zeros(n)
    ft = np.zeros(n); fd = np.zeros(n); st = np.zeros(n, np.int32)
    arrs = [_f64(scene.mu_p), _f64(scene.mu_t), _f64(scene.mu_d), _f64(scene.L), _f64(scene.alpha)]
    ov = ora_view(view)
    lib().ora_slice(n, *[_p(a) for a in arrs], ctypes.byref(ov), _p(mu_c), _p(cov_c), _p(ac),
                    _p(ft), _p(fd), _p(st))
    return Sliced(mu_c, cov_c, ac, ft, fd, st)


@dataclass
class Projected:
    mean2d: np.ndarray   # [2][n]
    conic: np.ndarray    # [3][n]
    depth: np.ndarray    # [n]
    rgb: np.ndarray      # [3][n]
    rect: np.ndarray     # [4][n] int32 tile range x0, y0, x1, y1 (x1, y1 exclusive)
    visible: np.ndarray  # [n] bool
    box: np.ndarray      # [4][n] opacity footprint in pixels (x0, y0, x1, y1)


def project(sliced: Sliced, sh, view) -> Projected:
    n = sliced.alpha_c.shape[0]
    mean2d = np.zeros((2, n)); conic = np.zeros((3, n)); depth = np.zeros(n)
    rgb = np.zeros((3, n)); rect = np.zeros((4, n), np.int32); vis = np.zeros(n, np.uint8)
    box = np.zeros((4, n))
    sh = _f64(sh)
    ov = ora_view(view)
    lib().ora_project(n, _p(np.ascontiguousarray(sliced.mu_c)), _p(np.ascontiguousarray(sliced.cov_c)),
                      _p(np.ascontiguousarray(sliced.alpha_c)), _p(sh), ctypes.byref(ov),
                      _p(mean2d), _p(conic), _p(depth), _p(rgb), _p(rect), _p(vis), _p(box))
    return Projected(mean2d, conic, depth, rgb, rect, vis.astype(bool), box)


def order(proj: Projected) -> np.ndarray:
    n = proj.depth.shape[0]
    out = np.zeros(n, np.int64)
    vis = proj.visible.astype(np.uint8)
    m = lib().ora_order(n, _p(proj.depth), _p(vis), _p(out))
    return out[:m]


@dataclass
class Image:
    image: np.ndarray     # [3][h][w]
    final_T: np.ndarray   # [h][w]
    ncontrib: np.ndarray  # [h][w]
    chash: np.ndarray     # [h][w] uint64 hash of the contributor set
    flags: np.ndarray     # [h][w] uint32 ORA_FLAG_* bits
    fbound: np.ndarray    # [h][w] bound on the pixel's change from in-band decisions
    ntest: np.ndarray     # [h][w] Gaussians tested by the pixel's brute-force loop
    vbound: np.ndarray    # [h][w] bound on its change from opacities moving within their bands


FLAG_ALPHA, FLAG_T, FLAG_DEPTH = 1, 2, 4


def fp32_model(sliced: Sliced, view) -> np.ndarray:
    """Per-Gaussian scales of the FP32 error model [5][n] (ora_fp32_model)."""
    n = sliced.alpha_c.shape[0]
    out = np.zeros((5, n))
    ov = ora_view(view)
    lib().ora_fp32_model(n, _p(np.ascontiguousarray(sliced.mu_c)), _p(np.ascontiguousarray(sliced.cov_c)),
                         ctypes.byref(ov), _p(out))
    return out


def composite(sliced: Sliced, proj: Projected, view, crop=None, flags=None, banded=True) -> Image:
    x0, y0, w, h = crop if crop is not None else (0, 0, view.W, view.H)
    n = proj.depth.shape[0]
    ordv = np.ascontiguousarray(order(proj))
    img = np.zeros((3, h, w)); T = np.zeros((h, w)); nc = np.zeros((h, w), np.int32)
    ch = np.zeros((h, w), np.uint64); fl = np.zeros((h, w), np.uint32); fb = np.zeros((h, w))
    nt = np.zeros((h, w), np.int64); vb = np.zeros((h, w))
    fc = flagcfg(**(flags or {}))
    ep = fp32_model(sliced, view) if banded else None
    ov = ora_view(view)
    lib().ora_composite(n, _p(proj.mean2d), _p(proj.conic), _p(np.ascontiguousarray(sliced.alpha_c)),
                        _p(proj.depth), _p(proj.rgb), _p(ep) if ep is not None else None, len(ordv),
                        _p(ordv), ctypes.byref(ov), x0, y0, w, h, ctypes.byref(fc) if banded else None,
                        _p(img), _p(T), _p(nc), _p(ch), _p(fl), _p(fb), _p(nt), _p(vb))
    return Image(img, T, nc, ch, fl, fb, nt, vb)


def render(scene, view, crop=None, flags=None, agr_weights=None, banded=True) -> Image:
    """Full FP64 forward of one view (optionally a pixel crop x0, y0, w, h),
    with the scene first refined by AGR when weights are given.  banded:
    also flag in-band decisions and bound their effect (flags, fbound), and
    bound the effect of every contributor's opacity moving within its band
    (vbound)."""
    if agr_weights is not None:
        scene = agr(scene, view.t, agr_weights)
    x0, y0, w, h = crop if crop is not None else (0, 0, view.W, view.H)
    n = scene.n
    img = np.zeros((3, h, w)); T = np.zeros((h, w)); nc = np.zeros((h, w), np.int32)
    ch = np.zeros((h, w), np.uint64); fl = np.zeros((h, w), np.uint32); fb = np.zeros((h, w))
    nt = np.zeros((h, w), np.int64); vb = np.zeros((h, w))
    fc = flagcfg(**(flags or {}))
    arrs = [_f64(scene.mu_p), _f64(scene.mu_t), _f64(scene.mu_d), _f64(scene.L),
            _f64(scene.alpha), _f64(scene.sh)]
    ov = ora_view(view)
    rc = lib().ora_render(n, *[_p(a) for a in arrs], ctypes.byref(ov), x0, y0, w, h,
                          ctypes.byref(fc) if banded else None, _p(img), _p(T), _p(nc), _p(ch), _p(fl), _p(fb),
                          _p(nt), _p(vb))
    if rc != 0:
        raise MemoryError("oracle render failed to allocate")
    return Image(img, T, nc, ch, fl, fb, nt, vb)


def sh_basis(x: float, y: float, z: float) -> np.ndarray:
    Y = np.zeros(16)
    lib().ora_sh_basis(float(x), float(y), float(z), _p(Y))
    return Y


def tile_lists(proj: Projected, view) -> dict:
    """Per-tile lists of visible Gaussians in (depth, index) order, from the
    FP64 footprints: {tile_id: [g, ...]} with tile_id = ty * tiles_x + tx."""
    tiles_x = (view.W + TILE - 1) // TILE
    out: dict[int, list[int]] = {}
    for g in order(proj):
        x0, y0, x1, y1 = proj.rect[:, g]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                out.setdefault(int(ty * tiles_x + tx), []).append(int(g))
    return out
