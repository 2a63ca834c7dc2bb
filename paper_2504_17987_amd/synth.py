"""Seeded synthetic particle-image pairs and analytic flows.

This module only *produces inputs*: particle images rendered from known
displacement fields, and the fields themselves (for truth at the vector
nodes).  It holds none of the PIV method's arithmetic (no pyramid, no block
matching, no correlation, no validation, no derivative stencils), so both
the GPU path and the CPU oracle may be fed from it.

Recipe (the paper measures on laboratory sequences that are not available;
these seeded images stand in for them):

* particles: Gaussian spots I0 * exp(-8 r^2 / d_p^2), integrated over each
  pixel's unit square with erf, diameter d_p = 2.5 px unless stated;
* positions uniform over the image plus a 16 px margin, count = ppp * area;
* frame A shows a particle at x - u(x)/2, frame B at x + u(x)/2 (u evaluated
  at the mid position), so the truth at a node is u at the node centre;
* independent Gaussian noise per frame, then rint and clipping to the
  dtype's range;
* optional dropout: a fraction of the particles is absent from frame B
  (out-of-plane loss of pairs).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Sequence, Tuple

import numpy as np
from scipy.special import erf

# ----------------------------------------------------------------------------
# flows: callables (x, y) -> (u, v), displacement in px per frame pair
# ----------------------------------------------------------------------------


@dataclass
class Uniform:
    u: float
    v: float

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        return np.full_like(x, self.u), np.full_like(x, self.v)


@dataclass
class SolidBody:
    """u = -omega (y - yc), v = omega (x - xc); vorticity dv/dx - du/dy = 2 omega."""
    xc: float
    yc: float
    omega: float

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return -self.omega * (y - self.yc), self.omega * (x - self.xc)

    def vorticity(self, x, y):
        return np.full_like(np.asarray(x, dtype=np.float64), 2.0 * self.omega)


@dataclass
class LambOseen:
    """Lamb-Oseen vortex: u_theta(r) = G/(2 pi r) (1 - exp(-r^2/rc^2)).

    Vorticity (dv/dx - du/dy) = G/(pi rc^2) exp(-r^2/rc^2).  The peak
    azimuthal speed 0.638161 * G/(2 pi rc) occurs at r = 1.12091 rc.
    """
    xc: float
    yc: float
    rc: float
    gamma: float

    PEAK_FACTOR = 0.638161  # max over r of (1 - exp(-s^2))/s, s = r/rc

    @classmethod
    def with_peak(cls, xc, yc, rc, peak, sign=1.0):
        gamma = sign * 2.0 * math.pi * rc * peak / cls.PEAK_FACTOR
        return cls(xc, yc, rc, gamma)

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        dx, dy = x - self.xc, y - self.yc
        r2 = dx * dx + dy * dy
        with np.errstate(invalid="ignore", divide="ignore"):
            # u_theta / r, with its r -> 0 limit G/(2 pi rc^2)
            k = np.where(r2 > 1e-24,
                         self.gamma / (2 * math.pi * r2) * (-np.expm1(-r2 / self.rc ** 2)),
                         self.gamma / (2 * math.pi * self.rc ** 2))
        return -k * dy, k * dx

    def vorticity(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        r2 = (x - self.xc) ** 2 + (y - self.yc) ** 2
        return self.gamma / (math.pi * self.rc ** 2) * np.exp(-r2 / self.rc ** 2)


@dataclass
class Shear:
    """u = U tanh((y - yc)/delta), v = 0."""
    U: float
    yc: float
    delta: float

    def __call__(self, x, y):
        y = np.asarray(y, dtype=np.float64)
        return self.U * np.tanh((y - self.yc) / self.delta), np.zeros_like(y)


@dataclass
class Sum:
    parts: List[Callable]

    def __call__(self, x, y):
        u = np.zeros(np.shape(x))
        v = np.zeros(np.shape(x))
        for p in self.parts:
            a, b = p(x, y)
            u = u + a
            v = v + b
        return u, v


@dataclass
class Gridded:
    """A displacement field sampled on the pixel grid, read with bilinear
    lookup (edge values held).  Used for the smooth random flows."""
    u: np.ndarray
    v: np.ndarray

    def __call__(self, x, y):
        from scipy.ndimage import map_coordinates
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        c = np.stack([y.ravel(), x.ravel()])
        uu = map_coordinates(self.u, c, order=1, mode="nearest").reshape(x.shape)
        vv = map_coordinates(self.v, c, order=1, mode="nearest").reshape(x.shape)
        return uu, vv


def smooth_random_flow(W, H, sigma=16.0, amplitude=6.0, seed=0) -> Gridded:
    """White noise per component, Gaussian-filtered (periodic), scaled so the
    largest |u| component magnitude over the image equals `amplitude`."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    u = gaussian_filter(rng.standard_normal((H, W)), sigma, mode="wrap")
    v = gaussian_filter(rng.standard_normal((H, W)), sigma, mode="wrap")
    mag = np.sqrt(u * u + v * v).max()
    return Gridded(u * (amplitude / mag), v * (amplitude / mag))


# ----------------------------------------------------------------------------
# rendering
# ----------------------------------------------------------------------------

def render(W: int, H: int, xs: np.ndarray, ys: np.ndarray, I0: np.ndarray,
           d_p: float = 2.5, radius: int = 3) -> np.ndarray:
    """Sum of pixel-integrated Gaussian particles (float64 image [H][W])."""
    img = np.zeros(H * W, dtype=np.float64)
    if len(xs) == 0:
        return img.reshape(H, W)
    k = math.sqrt(8.0) / d_p
    c = math.sqrt(math.pi) / (2.0 * k)
    off = np.arange(-radius, radius + 1)
    ix = np.floor(xs).astype(np.int64)[:, None] + off[None, :]
    iy = np.floor(ys).astype(np.int64)[:, None] + off[None, :]
    ex = c * (erf(k * (ix + 0.5 - xs[:, None])) - erf(k * (ix - 0.5 - xs[:, None])))
    ey = c * (erf(k * (iy + 0.5 - ys[:, None])) - erf(k * (iy - 0.5 - ys[:, None])))
    val = I0[:, None, None] * ey[:, :, None] * ex[:, None, :]
    yy = np.broadcast_to(iy[:, :, None], val.shape)
    xx = np.broadcast_to(ix[:, None, :], val.shape)
    ok = (xx >= 0) & (xx < W) & (yy >= 0) & (yy < H)
    np.add.at(img, (yy[ok] * W + xx[ok]), val[ok])
    return img.reshape(H, W)


def _quantize(img, noise, rng, maxval, dtype):
    if noise > 0:
        img = img + rng.normal(0.0, noise, img.shape)
    return np.clip(np.rint(img), 0, maxval).astype(dtype)


def make_pair(W: int, H: int, flow: Callable, ppp: float, *, d_p: float = 2.5,
              I0: Tuple[float, float] = (120.0, 255.0), noise: float = 2.0,
              dropout: float = 0.0, dtype=np.uint8, maxval: int = 255,
              seed: int = 0, margin: int = 16) -> Tuple[np.ndarray, np.ndarray]:
    """Render one seeded image pair [H][W] of `dtype`."""
    rng = np.random.default_rng(seed)
    n = int(round(ppp * (W + 2 * margin) * (H + 2 * margin)))
    x = rng.uniform(-margin, W + margin, n)
    y = rng.uniform(-margin, H + margin, n)
    amp = rng.uniform(I0[0], I0[1], n)
    keep = rng.random(n) >= dropout
    u, v = flow(x, y)
    A = render(W, H, x - u / 2, y - v / 2, amp, d_p)
    B = render(W, H, (x + u / 2)[keep], (y + v / 2)[keep], amp[keep], d_p)
    A = _quantize(A, noise, rng, maxval, dtype)
    B = _quantize(B, noise, rng, maxval, dtype)
    return A, B


def node_centres(W: int, H: int, step: int):
    """Vector-node centres (x, y) of the nx x ny grid, nx = W/step: node (a, b)
    sits at (b*step + (step-1)/2, a*step + (step-1)/2)."""
    nx, ny = W // step, H // step
    xs = np.arange(nx) * step + (step - 1) / 2.0
    ys = np.arange(ny) * step + (step - 1) / 2.0
    return np.meshgrid(xs, ys)


def truth(flow: Callable, W: int, H: int, step: int) -> np.ndarray:
    """[2][ny][nx] displacement of `flow` at the node centres."""
    X, Y = node_centres(W, H, step)
    u, v = flow(X, Y)
    return np.stack([u, v]).astype(np.float64)


# ----------------------------------------------------------------------------
# the five workloads (sizes, seeding and flows of the benchmark configurations)
# ----------------------------------------------------------------------------

def cfg1_pair(seed: int = 1000):
    """256x256 u8, 0.03 ppp, I0~U[120,255], sigma=2, uniform (3.4, -1.7)."""
    flow = Uniform(3.4, -1.7)
    A, B = make_pair(256, 256, flow, 0.03, noise=2.0, seed=seed)
    return A, B, flow


def cfg2_flow(W=1024, H=1024):
    return LambOseen.with_peak((W - 1) / 2.0, (H - 1) / 2.0, 128.0, 20.0)


def cfg2_pair(seed: int = 2000, W: int = 1024, H: int = 1024):
    """1 MP u8, 0.04 ppp, Lamb-Oseen (peak 20 px, rc 128), 10% dropout in B."""
    flow = cfg2_flow(W, H)
    A, B = make_pair(W, H, flow, 0.04, noise=2.0, dropout=0.10, seed=seed)
    return A, B, flow


def cfg3_flow(k: int, W=3840, H=2160):
    """Two counter-rotating Lamb-Oseen vortices (peak 8 px, rc 96) advected
    +0.5 px in x per pair index, plus a tanh shear layer of 15 px."""
    s = 0.5 * k
    return Sum([
        LambOseen.with_peak(0.3 * W + s, 0.4 * H, 96.0, 8.0, +1.0),
        LambOseen.with_peak(0.7 * W + s, 0.6 * H, 96.0, 8.0, -1.0),
        Shear(15.0, H / 2.0, 48.0),
    ])


def cfg3_pair(k: int = 0, seed: int = 3000, W: int = 3840, H: int = 2160):
    """u16 with 12-bit values, 0.02 ppp, I0~U[1920,4095], sigma=32."""
    flow = cfg3_flow(k, W, H)
    A, B = make_pair(W, H, flow, 0.02, I0=(1920.0, 4095.0), noise=32.0,
                     dtype=np.uint16, maxval=4095, seed=seed + k)
    return A, B, flow


def cfg4_pair(k: int = 0, seed: int = 4000, W: int = 512, H: int = 512):
    """512x512 float32 = (u8 render, 0.05 ppp, sigma=2)/255, smooth random
    flow (Gaussian-filtered noise, sigma 16 px, max |u| 6 px)."""
    flow = smooth_random_flow(W, H, 16.0, 6.0, seed=seed + 10000 + k)
    A, B = make_pair(W, H, flow, 0.05, noise=2.0, seed=seed + k)
    return (A.astype(np.float32) / 255.0), (B.astype(np.float32) / 255.0), flow


@dataclass
class Deficit:
    """Wake deficit behind a body: u = -D exp(-((y - yc)/w)^2) for x > x0
    (growing in over `ramp` px), v = 0."""
    D: float
    x0: float
    yc: float
    w: float
    ramp: float

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        on = 0.5 * (1.0 + np.tanh((x - self.x0) / self.ramp))
        return -self.D * on * np.exp(-((y - self.yc) / self.w) ** 2), np.zeros_like(y)


def cylinder_wake(W: int = 1024, H: int = 512, U: float = 6.0, D: float = 3.0, peak: float = 2.5):
    """A cylinder-like wake (a stand-in for the paper's low-seeding cylinder
    experiment, Sec. 3.2): free stream U px/frame in x, a velocity deficit
    of D px behind a body of diameter H/8 at (W/6, H/2), and a staggered
    street of alternating Lamb-Oseen vortices (peak `peak` px, core H/16)
    shed downstream at a spacing of H/4."""
    d = H / 8.0
    xb, yc = W / 6.0, H / 2.0
    parts: List[Callable] = [Uniform(U, 0.0), Deficit(D, xb, yc, 0.7 * d, d)]
    k = 0
    x = xb + 1.5 * d
    while x < W + H / 4:
        side = 1.0 if k % 2 == 0 else -1.0
        parts.append(LambOseen.with_peak(x, yc + side * 0.6 * d, H / 16.0, peak, sign=-side))
        x += H / 4.0
        k += 1
    return Sum(parts)


def cfg5_flow(stream: int, W: int, H: int):
    """Even streams: solid-body rotation with |u| = 8 px at the corners;
    odd streams: shear 8 tanh((y - H/2)/(H/16))."""
    if stream % 2 == 0:
        om = 8.0 / math.hypot(W / 2.0, H / 2.0)
        return SolidBody((W - 1) / 2.0, (H - 1) / 2.0, om)
    return Shear(8.0, H / 2.0, H / 16.0)


CFG5_SIZES = (512, 512, 512, 512, 1024, 1024, 1024, 1024, 2048, 2048, 2048, 2048)


def cfg5_pair(stream: int, k: int, seed: int = 5000):
    W = H = CFG5_SIZES[stream % len(CFG5_SIZES)]
    flow = cfg5_flow(stream, W, H)
    A, B = make_pair(W, H, flow, 0.03, noise=2.0, seed=seed + 100 * stream + k)
    return A, B, flow
