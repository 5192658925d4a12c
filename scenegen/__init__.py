"""Seeded synthetic inputs for the 7DGS render path.

This module only draws inputs: scene parameters of 7D Gaussians, pinhole views,
target images and request streams.  It computes none of the method's outputs
(no conditioning, projection or compositing), so both the FP64 oracle and the
HIP path can take their inputs from here without sharing any arithmetic.

Layouts (FP32, structure of arrays, one plane per component):
  mu_p  [3][N]   spatial mean (x, y, z)
  mu_t  [N]      temporal mean
  mu_d  [3][N]   directional mean
  L     [28][N]  lower-triangular Cholesky factor of the 7x7 covariance, packed
                 row-major: entry (i, j), i >= j, sits at plane i*(i+1)/2 + j;
                 dimension order (x, y, z, t, dx, dy, dz)
  alpha [N]      base opacity in (0, 1)
  sh    [48][N]  degree-3 spherical-harmonic colour coefficients; plane 3*k+ch
                 holds coefficient k (k = l*l + l + m) of channel ch

The parameter distributions follow the 7D representation of Sec. 4.1 (a 7D
Gaussian with a Cholesky-factored covariance and SH colour); the values are
random because trained scenes are not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_L = 28
N_SH = 48
TAN_HALF_FOV = math.tan(math.radians(30.0))  # 60 degree horizontal field of view


def tri_index(i: int, j: int) -> int:
    """Packed position of lower-triangular entry (i, j), i >= j."""
    return i * (i + 1) // 2 + j


# Off-diagonal entries in the draw order: row-major over the strict lower triangle.
OFFDIAG = [(i, j) for i in range(1, 7) for j in range(i)]


@dataclass
class Scene:
    mu_p: np.ndarray
    mu_t: np.ndarray
    mu_d: np.ndarray
    L: np.ndarray
    alpha: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.mu_t.shape[0])

    def arrays(self):
        return dict(mu_p=self.mu_p, mu_t=self.mu_t, mu_d=self.mu_d, L=self.L,
                    alpha=self.alpha, sh=self.sh)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(*(np.ascontiguousarray(a[..., idx]) for a in
                       (self.mu_p, self.mu_t, self.mu_d, self.L, self.alpha, self.sh)))

    def save(self, path: str) -> None:
        np.savez(path, version=np.int32(1), **self.arrays())

    @staticmethod
    def load(path: str) -> "Scene":
        z = np.load(path, allow_pickle=False)
        if int(z["version"]) != 1:
            raise ValueError(f"unsupported scene file version {int(z['version'])}")
        return Scene(*(np.ascontiguousarray(z[k], dtype=np.float32) for k in
                       ("mu_p", "mu_t", "mu_d", "L", "alpha", "sh")))


@dataclass
class View:
    """A pinhole view at time t.  R_wc maps world vectors to camera axes
    (x right, y down, z forward); c is the camera centre; d is the view
    direction the Gaussians are conditioned on; bg is the background colour."""
    R_wc: np.ndarray
    c: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    W: int
    H: int
    t: float
    d: np.ndarray
    lambda_t: float = 0.05
    lambda_d: float = 0.05
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    d_per_gaussian: bool = False   # condition each Gaussian on unit(mu_p - c) instead of d

    def replace(self, **kw) -> "View":
        d = dict(self.__dict__)
        d.update(kw)
        v = View(**d)
        v._cast()
        return v

    def _cast(self):
        f32 = np.float32
        self.R_wc = np.asarray(self.R_wc, f32).reshape(3, 3)
        self.c = np.asarray(self.c, f32).reshape(3)
        self.d = np.asarray(self.d, f32).reshape(3)
        self.bg = np.asarray(self.bg, f32).reshape(3)
        for k in ("fx", "fy", "cx", "cy", "t", "lambda_t", "lambda_d"):
            setattr(self, k, float(f32(getattr(self, k))))
        self.W, self.H = int(self.W), int(self.H)
        self.d_per_gaussian = bool(self.d_per_gaussian)


def look_at(c, target=(0.0, 0.0, 0.0)) -> np.ndarray:
    """World-to-camera rotation for a camera at c looking at target; world +z is
    up (world +y when the view is within ~2.6 degrees of vertical)."""
    c = np.asarray(c, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) <= 0.999 else np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return np.stack([right, down, f]).astype(np.float32)


def make_view(c, W, H, t, *, d=None, lambda_t=0.05, lambda_d=0.05, bg=(0, 0, 0)) -> View:
    c = np.asarray(c, np.float64)
    R = look_at(c)
    f = (W / 2.0) / TAN_HALF_FOV
    if d is None:
        d = R[2]  # the camera's forward axis
    v = View(R_wc=R, c=c, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0, W=W, H=H, t=t,
             d=np.asarray(d), lambda_t=lambda_t, lambda_d=lambda_d, bg=np.asarray(bg))
    v._cast()
    return v


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def make_scene(n: int, seed: int, *, h: float = 1.0, sigma_off: float = 0.05,
               recondition: bool = False, kappa_max: float = 1e4) -> Scene:
    """Draw n 7D Gaussians.  Draw order (PCG64, FP64 draws cast to FP32):
    mu_p ~ U[-h,h]^3; mu_t ~ U[0,1]; mu_d = unit(N(0,I3)); L off-diagonals ~
    N(0, sigma_off) (standard deviation); L diagonal = exp(U[ln .01, ln .3]);
    alpha ~ U(.05,.95); sh ~ N(0, .2)."""
    rng = np.random.default_rng(seed)
    mu_p = rng.uniform(-h, h, size=(n, 3))
    mu_t = rng.uniform(0.0, 1.0, size=n)
    mu_d = _unit(rng.normal(0.0, 1.0, size=(n, 3)))
    off = rng.normal(0.0, sigma_off, size=(n, 21))
    diag = np.exp(rng.uniform(math.log(0.01), math.log(0.3), size=(n, 7)))
    alpha = rng.uniform(0.05, 0.95, size=n)
    sh = rng.normal(0.0, 0.2, size=(n, 16, 3))

    L = np.zeros((n, N_L))
    for k, (i, j) in enumerate(OFFDIAG):
        L[:, tri_index(i, j)] = off[:, k]
    for i in range(7):
        L[:, tri_index(i, i)] = diag[:, i]
    if recondition:
        L = _recondition(L, np.random.default_rng(seed + 7), kappa_max)

    f32 = np.float32
    return Scene(mu_p=np.ascontiguousarray(mu_p.T, f32), mu_t=mu_t.astype(f32),
                 mu_d=np.ascontiguousarray(mu_d.T, f32), L=np.ascontiguousarray(L.T, f32),
                 alpha=alpha.astype(f32),
                 sh=np.ascontiguousarray(sh.reshape(n, 48).T, f32))


def unpack_L(Lp: np.ndarray) -> np.ndarray:
    """[N][28] packed -> [N][7][7] dense lower-triangular (input bookkeeping)."""
    n = Lp.shape[0]
    out = np.zeros((n, 7, 7), Lp.dtype)
    for i in range(7):
        for j in range(i + 1):
            out[:, i, j] = Lp[:, tri_index(i, j)]
    return out


def _recondition(Lp: np.ndarray, rng, kappa_max: float) -> np.ndarray:
    """Ill-conditioned (t, d) blocks with an unchanged spatial slice.

    The (t, d) block of each covariance gets eigenvalues e0 * kappa^(-j/3),
    j = 0..3 (kappa ~ logU[1, kappa_max]) in its own eigenbasis, and the
    position-(t, d) cross block is rescaled so that the regression of x_p on
    x_(t,d) explains the same spatial covariance as before.  Hence the
    conditional covariance is unchanged and only the conditioning of the
    (t, d) block varies.  Works in FP64; the caller stores FP32."""
    n = Lp.shape[0]
    Ld = unpack_L(Lp)
    S = Ld @ np.transpose(Ld, (0, 2, 1))
    kappa = np.exp(rng.uniform(0.0, math.log(kappa_max), size=n))
    SQQ = S[:, 3:, 3:]
    e, V = np.linalg.eigh(SQQ)           # ascending
    e, V = e[:, ::-1], V[:, :, ::-1]     # descending
    j = np.arange(4)
    e_new = e[:, :1] * kappa[:, None] ** (-j[None, :] / 3.0)
    inv_sqrt_old = V @ (np.reciprocal(np.sqrt(e))[:, :, None] * np.transpose(V, (0, 2, 1)))
    sqrt_new = V @ (np.sqrt(e_new)[:, :, None] * np.transpose(V, (0, 2, 1)))
    SPQ_new = S[:, :3, 3:] @ inv_sqrt_old @ sqrt_new
    S2 = S.copy()
    S2[:, 3:, 3:] = V @ (e_new[:, :, None] * np.transpose(V, (0, 2, 1)))
    S2[:, :3, 3:] = SPQ_new
    S2[:, 3:, :3] = np.transpose(SPQ_new, (0, 2, 1))
    C = np.linalg.cholesky(S2)
    out = np.zeros_like(Lp)
    for i in range(7):
        for jj in range(i + 1):
            out[:, tri_index(i, jj)] = C[:, i, jj]
    return out


def make_views(nview: int, seed: int, *, r: float, W: int, H: int, lam: float = 0.05,
               bg=(0, 0, 0), t=None) -> list[View]:
    """Views from stream default_rng(seed + 1000): per view u = unit(N(0, I3)),
    then t ~ U[0,1]; camera at r*u looking at the origin, d = -u."""
    rng = np.random.default_rng(seed + 1000)
    out = []
    for _ in range(nview):
        u = _unit(rng.normal(0.0, 1.0, size=3))
        tt = rng.uniform(0.0, 1.0)
        if t is not None:
            tt = t
        out.append(make_view(r * u, W, H, tt, d=-u, lambda_t=lam, lambda_d=lam, bg=bg))
    return out


def target_image(seed: int, W: int, H: int) -> np.ndarray:
    """Seeded target image U[0,1]^(3 x H x W), FP32."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(3, H, W)).astype(np.float32)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

AGR_OUT = (3, 1, 3, 28)      # outputs of the MLPs for mu_p, mu_t, mu_d, the packed L
AGR_IN, AGR_HIDDEN = 27, 64


def agr_weights(seed: int, out_scale=(0.03, 0.03, 0.03, 0.003)) -> np.ndarray:
    """Random AGR weights (FP32, the packed layout: per MLP p, t, d, l the
    arrays W1[64][27], b1[64], W2[C_out][64], b2[C_out]).  Drawn in that order
    from default_rng(seed): W1 ~ N(0, 1/27), b1 ~ N(0, 0.1), W2 ~ N(0, 1/64)
    and b2 ~ N(0, 0.1), W2 and b2 then scaled by the MLP's out_scale so that
    the residuals stay small next to the parameters they refine (an untrained
    network; no trained weights are available)."""
    rng = np.random.default_rng(seed)
    parts = []
    for c, sc in zip(AGR_OUT, out_scale):
        parts.append(rng.normal(0.0, np.sqrt(1.0 / AGR_IN), size=AGR_HIDDEN * AGR_IN))
        parts.append(rng.normal(0.0, 0.1, size=AGR_HIDDEN))
        parts.append(sc * rng.normal(0.0, np.sqrt(1.0 / AGR_HIDDEN), size=c * AGR_HIDDEN))
        parts.append(sc * rng.normal(0.0, 0.1, size=c))
    return np.concatenate(parts).astype(np.float32)


def config0(lam: float = 0.05):
    """1,000 Gaussians, one 64x64 view: random unit view direction d, camera at
    -3d looking at the origin, t = 0.5, black background."""
    scene = make_scene(1000, 0, h=1.0, sigma_off=0.05)
    rng = np.random.default_rng(1000)
    d = _unit(rng.normal(0.0, 1.0, size=3))
    view = make_view(-3.0 * d, 64, 64, 0.5, d=d, lambda_t=lam, lambda_d=lam)
    return scene, [view]


def config1(nview: int = 50, n: int = 200_000):
    """200,000 Gaussians in [-2,2]^3, 800x800, views on a sphere of radius 4,
    t ~ U[0,1], white background."""
    scene = make_scene(n, 1, h=2.0, sigma_off=0.05)
    views = make_views(nview, 1, r=4.0, W=800, H=800, bg=(1, 1, 1))
    return scene, views


def config2(n: int = 500_000):
    """Training step: 500,000 Gaussians, one 1352x1014 view at radius 3 and
    its seeded random target image."""
    scene = make_scene(n, 2, h=1.0, sigma_off=0.05)
    views = make_views(1, 2, r=3.0, W=1352, H=1014)
    return scene, views, target_image(2002, 1352, 1014)


SERVE_RES = [(512, 512), (800, 800), (1280, 720), (1920, 1080)]
SERVE_SIZES = [100_000, 300_000, 1_000_000, 2_000_000]


def config3_scenes(sizes=SERVE_SIZES):
    """Four resident scenes with strong time/direction-position correlation."""
    return [make_scene(n, 30 + i, h=1.0, sigma_off=0.15) for i, n in enumerate(sizes)]


@dataclass
class Request:
    arrival: float       # seconds since stream start
    scene: int
    view: View


def request_stream(nreq: int, qps: float, *, nscenes: int = 4, seed: int = 300,
                   resolutions=SERVE_RES, r: float = 3.0, lam: float = 0.05) -> list[Request]:
    """Poisson stream: per request, exponential inter-arrival (mean 1/qps), scene
    uniform, resolution uniform, camera direction unit(N(0,I3)) at radius r,
    t ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    tnow = 0.0
    out = []
    for _ in range(nreq):
        tnow += rng.exponential(1.0 / qps)
        s = int(rng.integers(nscenes))
        W, H = resolutions[int(rng.integers(len(resolutions)))]
        u = _unit(rng.normal(0.0, 1.0, size=3))
        t = rng.uniform(0.0, 1.0)
        out.append(Request(tnow, s, make_view(r * u, W, H, t, d=-u, lambda_t=lam, lambda_d=lam)))
    return out


def config4(n: int = 4_000_000, nview: int = 64):
    """Stress: 4M Gaussians with ill-conditioned (t, d) blocks, 1920x1080."""
    scene = make_scene(n, 4, h=1.0, sigma_off=0.05, recondition=True)
    views = make_views(nview, 4, r=3.0, W=1920, H=1080)
    return scene, views, target_image(4004, 1920, 1080)
