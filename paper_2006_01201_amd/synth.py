"""Seeded synthetic overlap strips (inputs only).

The paper evaluates on twenty photo sets that are not available, so every
input here is synthetic, with the paper's panorama shape (9000 x 4000,
Section IV) and the structure of a coarsely registered overlap strip: an
analytic texture seen through a smooth, bounded disparity field, an
optional occluding band at its own disparity, a residual exposure gain and
sensor noise.

This module holds none of the stitching method's arithmetic (no luma, no
pyramid, no search, no warp-and-blend). It is shared by the tests, the
benchmark and the CPU oracle's test harness purely as input plumbing.

Coordinates: ``x`` is the column, ``y`` the row. A strip is ``H`` rows by
``W`` columns. The ground-truth flow of direction "R to L" satisfies
``R(p) ~ L(p + u_rl(p))`` and the "L to R" flow ``L(q) ~ R(q + u_lr(q))``.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

SEED_ROOT = (2006, 1201)
SIZE_DRAW = 99  # the "strip" slot of the seed used for strip-size draws
_WORKERS = max(1, min(16, os.cpu_count() or 1))


def rng_for(cfg: int, pano: int, strip: int) -> np.random.Generator:
    """The one seeding rule: SeedSequence([2006, 1201, cfg, pano, strip])."""
    return np.random.default_rng(np.random.SeedSequence([*SEED_ROOT, cfg, pano, strip]))


class Texture:
    """Analytic multi-scale RGB texture evaluated at real coordinates.

    128 + 24 oriented sinusoids (per-channel phase) + 60 additive
    axis-aligned rectangles. Sinusoid amplitudes U[6, 14], frequencies
    log-uniform in [1/400, 1/5] cycles/px, orientations U[0, pi), phases
    U[0, 2 pi). Rectangle corners uniform over the ``H x W`` frame, widths
    log-uniform in [0.02, 0.4] W and heights in [0.005, 0.4] H, per-channel
    offsets U[-50, 50]. Content at every scale (as in natural images) keeps
    the coarse pyramid levels textured.
    """

    N_SIN = 24
    N_RECT = 60

    def __init__(self, rng: np.random.Generator, H: int, W: int, periodic: bool = False):
        """``periodic``: the texture repeats along x with period W (a
        360-degree panorama): every sinusoid makes a whole number of cycles
        across W and rectangles wrap."""
        n_sin, n_rect = self.N_SIN, self.N_RECT
        self.amp = rng.uniform(6.0, 14.0, n_sin)
        self.freq = np.exp(rng.uniform(np.log(1.0 / 400.0), np.log(1.0 / 5.0), n_sin))
        self.theta = rng.uniform(0.0, np.pi, n_sin)
        self.phase = rng.uniform(0.0, 2.0 * np.pi, (n_sin, 3))
        rx0 = rng.uniform(0.0, W, n_rect)
        ry0 = rng.uniform(0.0, H, n_rect)
        rw = np.exp(rng.uniform(np.log(0.02), np.log(0.4), n_rect)) * W
        rh = np.exp(rng.uniform(np.log(0.005), np.log(0.4), n_rect)) * H
        self.rects = np.stack([rx0, ry0, rx0 + rw, ry0 + rh], axis=1)
        self.offset = rng.uniform(-50.0, 50.0, (n_rect, 3))
        self.period = float(W) if periodic else None
        if periodic:
            fx = np.rint(self.freq * np.cos(self.theta) * W) / W
            fy = self.freq * np.sin(self.theta)
            self.freq = np.hypot(fx, fy)
            self.theta = np.arctan2(fy, fx)

    def rect_mask(self, r, x, y):
        x0, y0, x1, y1 = self.rects[r]
        if self.period is None:
            return (x >= x0) & (x < x1) & (y >= y0) & (y < y1)
        return (np.mod(x - x0, self.period) < x1 - x0) & (y >= y0) & (y < y1)

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        x, y = np.broadcast_arrays(x, y)
        if x.ndim >= 1 and x.size > (1 << 16):
            parts = parallel_rows(lambda r0, r1: self._eval(x[r0:r1], y[r0:r1]), x.shape[0])
            return np.concatenate(parts, axis=0)
        return self._eval(x, y)

    def _eval(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        out = np.full(x.shape + (3,), 128.0, dtype=np.float32)
        cph = np.cos(self.phase).astype(np.float32)
        sph = np.sin(self.phase).astype(np.float32)
        two_pi = 2.0 * np.pi
        for k in range(len(self.amp)):
            arg = (two_pi * self.freq[k]) * (x * np.cos(self.theta[k]) + y * np.sin(self.theta[k]))
            # range-reduce in double, then evaluate the two transcendental
            # functions once in float32; the angle-sum identity gives every
            # channel's phase from them
            arg = (arg - two_pi * np.rint(arg / two_pi)).astype(np.float32)
            s, c = np.sin(arg), np.cos(arg)
            a = np.float32(self.amp[k])
            for ch in range(3):
                out[..., ch] += a * (s * cph[k, ch] + c * sph[k, ch])
        if x.size:
            xlo, xhi, ylo, yhi = x.min(), x.max(), y.min(), y.max()
            for r in range(len(self.rects)):
                x0, y0, x1, y1 = self.rects[r]
                if y1 <= ylo or y0 > yhi or (self.period is None and (x1 <= xlo or x0 > xhi)):
                    continue
                out[self.rect_mask(r, x, y)] += self.offset[r].astype(np.float32)
        return out


def smooth_field(rng: np.random.Generator, H: int, W: int, sigma: float, max_abs: float) -> np.ndarray:
    """White noise low-passed by a Gaussian of std ``sigma`` px (in the
    Fourier domain, periodic), rescaled so that max |f| = ``max_abs``."""
    noise = rng.standard_normal((H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    g = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * (fx ** 2 + fy ** 2))
    f = np.fft.irfft2(np.fft.rfft2(noise) * g, s=(H, W))
    m = np.abs(f).max()
    return f * (max_abs / m) if m > 0 else f


def bilinear_field(f: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Sample a 2-D field at real coordinates, bilinear, clamp to edge."""
    H, W = f.shape
    xc = np.clip(x, 0.0, W - 1.0)
    yc = np.clip(y, 0.0, H - 1.0)
    return ndimage.map_coordinates(f, [yc.ravel(), xc.ravel()], order=1, mode="nearest").reshape(x.shape)


def _row_blocks(H: int, n: int):
    step = max(16, -(-H // n))
    return [(r, min(H, r + step)) for r in range(0, H, step)]


def parallel_rows(fn, H: int):
    """Run ``fn(r0, r1)`` over row blocks on a thread pool (numpy and
    scipy release the GIL in the bulk work) and return the results in
    block order."""
    blocks = _row_blocks(H, 4 * _WORKERS)
    with ThreadPoolExecutor(_WORKERS) as ex:
        return list(ex.map(lambda b: fn(*b), blocks))


def invert_field(ux: np.ndarray, uy: np.ndarray, iters: int = 20, tol: float = 1e-6):
    """Fixed-point inverse v(q) = -u(q + v(q)) on the pixel grid."""
    H, W = ux.shape

    def block(r0, r1):
        yy, xx = np.mgrid[r0:r1, 0:W].astype(np.float64)
        vx, vy = -ux[r0:r1].copy(), -uy[r0:r1].copy()
        for _ in range(iters):
            nx = -bilinear_field(ux, xx + vx, yy + vy)
            ny = -bilinear_field(uy, xx + vx, yy + vy)
            delta = max(np.abs(nx - vx).max(initial=0.0), np.abs(ny - vy).max(initial=0.0))
            vx, vy = nx, ny
            if delta < tol:
                break
        return vx, vy

    parts = parallel_rows(block, H)
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


@dataclass
class Strip:
    """One overlap strip: L and R images (H x W x 3) plus ground truth."""

    L: np.ndarray
    R: np.ndarray
    axis: int  # 0: Area1 (only L) is left of the strip; 1: Area1 is above
    flow_rl_gt: np.ndarray  # H x W x 2 (x, y), R(p) ~ L(p + u)
    flow_lr_gt: np.ndarray  # H x W x 2 (x, y), L(q) ~ R(q + v)
    valid_rl: np.ndarray  # bool H x W: correspondence visible and inside
    valid_lr: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def H(self) -> int:
        return self.L.shape[0]

    @property
    def W(self) -> int:
        return self.L.shape[1]


def _quantise(v: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(v), 0, 255).astype(np.uint8)


def _inside_mask(x, y, H, W):
    return (x >= 0) & (x <= W - 1) & (y >= 0) & (y <= H - 1)


def _strip_axis0(rng, H, W, *, field_kind, max_ux, max_uy, noise_l, noise_r,
                 gain_range=None, occluder=False, float_out=False,
                 frame=None, x_off=0, field_params=None):
    """Generate one strip whose seam runs vertically (disparity mostly along x).

    Draw order (fixed): background texture, flow field, occluder
    (width, position, disparity, texture), gain, noise on L, noise on R.
    """
    fH, fW = frame if frame is not None else (H, W)
    tex = Texture(rng, fH, fW)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    if field_kind == "sinusoid":
        # (3, 0) + separable sinusoids with amplitude <= 2 px and
        # wavelengths U[96, 256] px
        ax, ay = rng.uniform(1.0, 2.0, 2)
        lam = rng.uniform(96.0, 256.0, 4)
        ph = rng.uniform(0.0, 2.0 * np.pi, 4)
        gx = xx + x_off
        ux = max_ux + ax * np.sin(2 * np.pi * gx / lam[0] + ph[0]) * np.sin(2 * np.pi * yy / lam[1] + ph[1])
        uy = ay * np.sin(2 * np.pi * gx / lam[2] + ph[2]) * np.sin(2 * np.pi * yy / lam[3] + ph[3])
    else:
        sigma = field_params.get("sigma") if field_params else None
        if sigma is None:
            sigma = max(128.0, 0.15 * min(H, W))
        ux = smooth_field(rng, H, W, sigma, max_ux)
        uy = smooth_field(rng, H, W, sigma, max_uy)
    band = None
    if occluder:
        wb = int(rng.integers(64, 129))
        xb = float(rng.uniform(0.25 * W, 0.6 * W))
        dob = float(rng.uniform(30.0, 40.0))
        tex_o = Texture(rng, fH, fW)
        band = (xb, xb + wb, dob, tex_o)
    gain = float(rng.uniform(*gain_range)) if gain_range else 1.0

    # L(p) = T(p); R(p) = g * T(p + u(p))
    Lf = tex(xx + x_off, yy)
    Rf = gain * tex(xx + x_off + ux, yy + uy)
    u_rl = np.stack([ux, uy], axis=-1)
    vx, vy = invert_field(ux, uy)
    u_lr = np.stack([vx, vy], axis=-1)
    valid_rl = _inside_mask(xx + ux, yy + uy, H, W)
    valid_lr = _inside_mask(xx + vx, yy + vy, H, W)
    if band is not None:
        b0, b1, dob, tex_o = band
        in_l = (xx >= b0) & (xx < b1)
        Lf[in_l] = tex_o(xx[in_l] + x_off, yy[in_l])
        in_r = (xx + dob >= b0) & (xx + dob < b1)
        Rf[in_r] = gain * tex_o(xx[in_r] + dob + x_off, yy[in_r])
        # background R pixels whose match falls on L's band are occluded
        mx = xx + ux
        valid_rl &= ~((mx >= b0) & (mx < b1) & ~in_r)
        u_rl[in_r] = (dob, 0.0)
        valid_rl[in_r] = _inside_mask(xx[in_r] + dob, yy[in_r], H, W)
        # background L pixels whose match falls on R's band are occluded
        mx = xx + vx
        valid_lr &= ~((mx + dob >= b0) & (mx + dob < b1) & ~in_l)
        u_lr[in_l] = (-dob, 0.0)
        valid_lr[in_l] = _inside_mask(xx[in_l] - dob, yy[in_l], H, W)
    if noise_l:
        Lf = Lf + rng.normal(0.0, noise_l, Lf.shape)
    if noise_r:
        Rf = Rf + rng.normal(0.0, noise_r, Rf.shape)
    if float_out:
        L = (Lf / 255.0).astype(np.float32)
        R = (Rf / 255.0).astype(np.float32)
    else:
        L, R = _quantise(Lf), _quantise(Rf)
    meta = {"gain": gain}
    if band is not None:
        meta.update(band_x0=band[0], band_x1=band[1], band_disp=band[2])
    return L, R, u_rl, u_lr, valid_rl, valid_lr, meta


def make_strip(rng, H, W, axis=0, **kw) -> Strip:
    """One strip of ``H x W``. For ``axis == 1`` (seam runs horizontally,
    disparity mostly along y) the strip is generated in the transposed
    frame and transposed back, so ``max_ux`` is then the bound across the
    seam (vertical) and ``max_uy`` the bound along it."""
    if axis == 0:
        L, R, u_rl, u_lr, v_rl, v_lr, meta = _strip_axis0(rng, H, W, **kw)
    else:
        L, R, u_rl, u_lr, v_rl, v_lr, meta = _strip_axis0(rng, W, H, **kw)
        L = np.ascontiguousarray(L.transpose(1, 0, 2))
        R = np.ascontiguousarray(R.transpose(1, 0, 2))
        u_rl = np.ascontiguousarray(u_rl.transpose(1, 0, 2)[..., ::-1])
        u_lr = np.ascontiguousarray(u_lr.transpose(1, 0, 2)[..., ::-1])
        v_rl, v_lr = v_rl.T.copy(), v_lr.T.copy()
    return Strip(L=L, R=R, axis=axis, flow_rl_gt=u_rl.astype(np.float32),
                 flow_lr_gt=u_lr.astype(np.float32), valid_rl=v_rl, valid_lr=v_lr, meta=meta)


# ---------------------------------------------------------------------------
# the five workloads

#: pyramid levels per workload (parameters of the flow method, listed here
#: only so that every caller uses the same value for the same workload)
LEVELS = {0: 3, 1: 6, 2: 6, 3: 6, 4: 6}


def strip_shapes(cfg: int, pano: int = 0):
    """List of (H, W, axis) for one panorama of workload ``cfg``."""
    if cfg == 0:
        return [(256, 64, 0)]
    if cfg == 1:
        return [(4000, 768, 0)]
    if cfg == 2:
        r = rng_for(2, pano, SIZE_DRAW)
        ws = r.integers(480, 961, size=6)
        return [(4000, int(w), 0) for w in ws] + [(600, 9000, 1)]
    if cfg == 3:
        return [(2048, 512, 0)]
    if cfg == 4:
        r = rng_for(4, pano, SIZE_DRAW)
        hs = r.integers(2000, 4001, size=6)
        ws = r.integers(480, 961, size=6)
        tw = int(r.integers(4500, 9001))
        th = int(r.integers(300, 601))
        return [(int(h), int(w), 0) for h, w in zip(hs, ws)] + [(th, tw, 1)]
    raise ValueError(f"unknown workload {cfg}")


def make_config_strip(cfg: int, pano: int, strip: int) -> Strip:
    shapes = strip_shapes(cfg, pano)
    H, W, axis = shapes[strip]
    rng = rng_for(cfg, pano, strip)
    if cfg == 0:
        # 256 x 256 images; the strip is columns [96, 160)
        return make_strip(rng, H, W, axis, field_kind="sinusoid", max_ux=3.0, max_uy=0.0,
                          noise_l=0.0, noise_r=2.0, frame=(256, 256), x_off=96)
    if cfg == 1:
        return make_strip(rng, H, W, axis, field_kind="smooth", max_ux=40.0, max_uy=8.0,
                          noise_l=3.0, noise_r=3.0, occluder=True)
    if cfg in (2, 4):
        return make_strip(rng, H, W, axis, field_kind="smooth", max_ux=40.0, max_uy=8.0,
                          noise_l=2.0, noise_r=2.0, occluder=True, gain_range=(0.9, 1.1))
    if cfg == 3:
        return make_strip(rng, H, W, axis, field_kind="smooth", max_ux=40.0, max_uy=8.0,
                          noise_l=2.0, noise_r=2.0, float_out=True)
    raise ValueError(f"unknown workload {cfg}")


def make_config(cfg: int, pano: int = 0):
    """All strips of one panorama of workload ``cfg`` (generated in
    parallel; each strip has its own seed, so the result does not depend
    on the order)."""
    n = len(strip_shapes(cfg, pano))
    with ThreadPoolExecutor(min(n, 4)) as ex:
        return list(ex.map(lambda s: make_config_strip(cfg, pano, s), range(n)))


def make_random(seed: int, H: int, W: int, axis: int = 0, max_ux: float = 6.0, max_uy: float = 2.0,
                noise: float = 2.0, sigma: float | None = None, occluder: bool = False,
                float_out: bool = False) -> Strip:
    """A strip of any size for parity tests (seed slot cfg = 100)."""
    rng = rng_for(100, seed, 0)
    if sigma is None:
        sigma = max(8.0, 0.15 * min(H, W))
    return make_strip(rng, H, W, axis, field_kind="smooth", max_ux=max_ux, max_uy=max_uy,
                      noise_l=noise, noise_r=noise, occluder=occluder, float_out=float_out,
                      field_params={"sigma": sigma})


def random_bytes(seed: int, shape) -> np.ndarray:
    """Uniform random uint8 array (tie-rich when drawn from few levels)."""
    return rng_for(101, seed, 0).integers(0, 256, size=shape, dtype=np.uint8)


def random_levels(seed: int, shape, levels: int) -> np.ndarray:
    """uint8 array drawn from ``levels`` distinct values (many ties)."""
    r = rng_for(102, seed, 0)
    vals = np.linspace(0, 255, levels).round().astype(np.uint8)
    return vals[r.integers(0, levels, size=shape)]


# ---------------------------------------------------------------------------
# Canvases: two photos placed on a common canvas with coverage masks of any
# shape (the inputs of canvas compositing).


@dataclass
class Canvas:
    """A pair canvas: L and R (H x W x 3, zero where the photo does not
    reach) with their coverage masks (uint8, 1 = covered)."""

    L: np.ndarray
    R: np.ndarray
    mask_L: np.ndarray
    mask_R: np.ndarray
    axis: int
    flow_rl_gt: np.ndarray  # R(p) ~ L(p + u) over the whole canvas
    meta: dict = field(default_factory=dict)


def _edge(rng, n, centre, slope, bow):
    """A slanted, slightly bowed photo edge: position along the other axis
    for each of n rows (or columns)."""
    t = np.arange(n, dtype=np.float64)
    return centre + slope * (t - n / 2.0) + bow * np.sin(np.pi * t / max(n - 1, 1))


def canvas_masks(rng, H: int, W: int, overlap: float, holes: int = 0):
    """Coverage of two photos side by side (seam running top to bottom):
    L reaches from the left to a slanted, bowed edge, R from another such
    edge to the right, with overlap ~ ``overlap`` W between them; both have
    slanted top and bottom edges (canvas corners stay uncovered), and
    ``holes`` elliptical gaps are cut out of R's coverage inside the
    overlap (Area1 islands inside Area3)."""
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    ow = overlap * W
    cx = rng.uniform(0.45, 0.55) * W
    right_L = _edge(rng, H, cx + ow / 2, rng.uniform(-0.08, 0.08) * W / max(H, 1), rng.uniform(-0.03, 0.03) * W)
    left_R = _edge(rng, H, cx - ow / 2, rng.uniform(-0.08, 0.08) * W / max(H, 1), rng.uniform(-0.03, 0.03) * W)
    mL = xx <= right_L[:, None]
    mR = xx >= left_R[:, None]
    for m in (mL, mR):
        top = _edge(rng, W, rng.uniform(0.0, 0.04) * H, rng.uniform(-0.04, 0.04) * H / max(W, 1), 0.0)
        bot = _edge(rng, W, rng.uniform(0.96, 1.0) * H, rng.uniform(-0.04, 0.04) * H / max(W, 1), 0.0)
        m &= (yy >= top[None, :]) & (yy <= bot[None, :])
    for _ in range(holes):
        ex, ey = rng.uniform(cx - ow / 3, cx + ow / 3), rng.uniform(0.15, 0.85) * H
        ax, ay = rng.uniform(0.05, 0.2) * ow + 1, rng.uniform(0.02, 0.08) * H + 1
        mR &= ((xx - ex) / ax) ** 2 + ((yy - ey) / ay) ** 2 > 1.0
    return mL.astype(np.uint8), mR.astype(np.uint8)


def make_canvas(seed: int, H: int, W: int, axis: int = 0, overlap: float = 0.3, holes: int = 0,
                max_ux: float = 6.0, max_uy: float = 2.0, noise: float = 2.0) -> Canvas:
    """A pair canvas (seed slot cfg = 110). Draw order: masks, texture,
    flow field, noise on L, noise on R. For axis 1 (seam running left to
    right, Area1 above) the canvas is generated transposed."""
    rng = rng_for(110, seed, axis)
    h, w = (H, W) if axis == 0 else (W, H)
    mL, mR = canvas_masks(rng, h, w, overlap, holes)
    tex = Texture(rng, h, w)
    sigma = max(8.0, 0.05 * min(h, w))
    ux = smooth_field(rng, h, w, sigma, max_ux)
    uy = smooth_field(rng, h, w, sigma, max_uy)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    Lf = tex(xx, yy)
    Rf = tex(xx + ux, yy + uy)
    if noise:
        Lf = Lf + rng.normal(0.0, noise, Lf.shape)
        Rf = Rf + rng.normal(0.0, noise, Rf.shape)
    L = _quantise(Lf) * mL[..., None]
    R = _quantise(Rf) * mR[..., None]
    u = np.stack([ux, uy], axis=-1)
    if axis == 1:
        L, R = L.transpose(1, 0, 2), R.transpose(1, 0, 2)
        mL, mR = mL.T, mR.T
        u = u.transpose(1, 0, 2)[..., ::-1]
    return Canvas(np.ascontiguousarray(L), np.ascontiguousarray(R), np.ascontiguousarray(mL),
                  np.ascontiguousarray(mR), axis, np.ascontiguousarray(u), {"holes": holes})


def random_masks(seed: int, H: int, W: int, blobs: int = 6, p_empty: float = 0.0):
    """Two coverage masks made of random discs and rectangles (general,
    non-convex, possibly disconnected shapes for distance tests)."""
    rng = rng_for(111, seed, 0)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    out = []
    for _ in range(2):
        m = np.zeros((H, W), bool)
        if rng.uniform() >= p_empty:
            for _ in range(blobs):
                cx, cy = rng.uniform(-0.1, 1.1) * W, rng.uniform(-0.1, 1.1) * H
                if rng.uniform() < 0.5:
                    r = rng.uniform(0.03, 0.35) * max(H, W)
                    m |= (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
                else:
                    hw, hh = rng.uniform(0.02, 0.4) * W, rng.uniform(0.02, 0.4) * H
                    m |= (np.abs(xx - cx) <= hw) & (np.abs(yy - cy) <= hh)
        out.append(m.astype(np.uint8))
    return out[0], out[1]


def panorama_masks(rng, H: int, W: int, n_ring: int, top: bool = True, closed: bool = False):
    """Coverage of a photo set on a panorama canvas: n_ring photos side by
    side (seams running top to bottom, overlaps U[480, 960] x W / 9000
    wide, slanted and bowed edges) reaching from ~0.15 H (bowed) to the
    bottom, and, if ``top``, one photo over the full width from the top to
    ~0.3 H (bowed): its seam with the ring is a band of ~0.15 H. With
    ``closed`` the canvas wraps in x and the ring is closed: one more seam
    at column 0 (= W), which the first photo reaches leftwards and the last
    one rightwards, across the wrap."""
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    if closed:
        seams = [k * W / n_ring for k in range(n_ring)] + [float(W)]
        ov = rng.uniform(480.0, 960.0, n_ring) * W / 9000.0
        ov = np.append(ov, ov[0])
        edges = []
        for x, o in zip(seams, ov):
            slope = rng.uniform(-0.02, 0.02) * W / max(H, 1) / n_ring
            bow = rng.uniform(-0.1, 0.1) * o
            edges.append((_edge(rng, H, x - o / 2, slope, bow), _edge(rng, H, x + o / 2, slope, bow)))
        ring_top = _edge(rng, W, 0.15 * H, 0.0, rng.uniform(-0.02, 0.02) * H)
        masks = []
        for k in range(n_ring):
            lo, hi = edges[k][0], edges[k + 1][1]  # photo k: from seam k's left edge to seam k + 1's right one
            m = (np.mod(xx - lo[:, None], W) < (hi - lo)[:, None]) & (yy >= ring_top[None, :])
            masks.append(m.astype(np.uint8))
        if top:
            bottom = _edge(rng, W, 0.30 * H, 0.0, rng.uniform(-0.02, 0.02) * H)
            masks.append((yy <= bottom[None, :]).astype(np.uint8))
        return masks
    seams = [(k + 1) * W / n_ring for k in range(n_ring - 1)]
    ov = rng.uniform(480.0, 960.0, len(seams)) * W / 9000.0
    lefts, rights = [np.zeros(H) - 1.0], []
    for x, o in zip(seams, ov):
        slope = rng.uniform(-0.02, 0.02) * W / max(H, 1) / n_ring
        rights.append(_edge(rng, H, x + o / 2, slope, rng.uniform(-0.1, 0.1) * o))
        lefts.append(_edge(rng, H, x - o / 2, slope, rng.uniform(-0.1, 0.1) * o))
    rights.append(np.zeros(H) + W)
    ring_top = _edge(rng, W, 0.15 * H, 0.0, rng.uniform(-0.02, 0.02) * H)
    masks = [((xx > lo[:, None]) & (xx < hi[:, None]) & (yy >= ring_top[None, :])).astype(np.uint8)
             for lo, hi in zip(lefts, rights)]
    if top:
        bottom = _edge(rng, W, 0.30 * H, 0.0, rng.uniform(-0.02, 0.02) * H)
        masks.append((yy <= bottom[None, :]).astype(np.uint8))
    return masks


def make_panorama_photos(seed: int, H: int, W: int, n_ring: int = 6, top: bool = True, max_ux: float = 6.0,
                         max_uy: float = 2.0, noise: float = 2.0, device=None, closed: bool = False):
    """A photo set placed on one H x W canvas (seed slot cfg = 120): one
    scene texture seen by every photo through its own smooth residual
    misalignment (|u| <= max_ux, max_uy px), exposure gain U[0.95, 1.05]
    and sensor noise, zero outside the photo's coverage. Returns a list of
    (image H x W x 3 uint8, mask H x W uint8, axis, side) in merge order:
    the ring left to right (axis 0, side 0), then the top photo (axis 1,
    side 1). Arrays are numpy, or torch tensors on ``device`` (evaluated
    there). ``closed``: a 360-degree panorama (scene, misalignment fields
    and coverage periodic in x; seed slot cfg = 121) whose last ring photo
    overlaps the first across column W - 1 / 0."""
    rng = rng_for(121 if closed else 120, seed, 0)
    masks = panorama_masks(rng, H, W, n_ring, top, closed=closed)
    tex = Texture(rng, H, W, periodic=closed)
    sigma = max(8.0, 0.05 * min(H, W))
    out = []
    for i, m in enumerate(masks):
        gain = float(rng.uniform(0.95, 1.05))
        if device is None:
            ux = smooth_field(rng, H, W, sigma, max_ux)
            uy = smooth_field(rng, H, W, sigma, max_uy)
            yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
            f = gain * tex(xx + ux, yy + uy)
            if noise:
                f = f + rng.normal(0.0, noise, f.shape)
            img = _quantise(f) * m[..., None]
        else:
            import torch

            ux = _smooth_field_torch(rng, H, W, sigma, max_ux, device)
            uy = _smooth_field_torch(rng, H, W, sigma, max_uy, device)
            gen = torch.Generator(device=device)
            gen.manual_seed(int(rng.integers(0, 2 ** 62)))
            yy, xx = torch.meshgrid(torch.arange(H, device=device, dtype=torch.float64),
                                    torch.arange(W, device=device, dtype=torch.float64), indexing="ij")
            f = gain * _texture_torch(tex, xx + ux, yy + uy)
            if noise:
                f += noise * torch.randn(f.shape, generator=gen, device=device)
            mt = torch.from_numpy(m).to(device)
            img = f.round_().clamp_(0, 255).to(torch.uint8) * mt[..., None]
            m = mt
        last_top = top and i == len(masks) - 1
        out.append((img, m, 1 if last_top else 0, 1 if last_top else 0))
    return out


# ---------------------------------------------------------------------------
# Device-side evaluation for large streams (the 32-panorama workload): the
# recipe of ``make_config_strip`` with the per-pixel work (texture,
# smoothing of the flow noise, warp, sensor noise) evaluated by torch on
# the GPU. Two departures keep it fast and free of host synchronisation:
# the flow noise is drawn on a fixed FFT grid and cropped, and the sensor
# noise comes from a torch generator seeded from the strip's generator. The
# images are therefore not bit for bit those of the CPU path; they are used
# for throughput runs, not for parity.

def _texture_torch(tex: Texture, x, y):
    import torch

    out = torch.full(x.shape + (3,), 128.0, dtype=torch.float32, device=x.device)
    two_pi = 2.0 * np.pi
    cph = torch.tensor(np.cos(tex.phase), dtype=torch.float32, device=x.device)
    sph = torch.tensor(np.sin(tex.phase), dtype=torch.float32, device=x.device)
    for k in range(len(tex.amp)):
        arg = (two_pi * tex.freq[k]) * (x * np.cos(tex.theta[k]) + y * np.sin(tex.theta[k]))
        arg = (arg - two_pi * torch.round(arg / two_pi)).float()
        s, c = torch.sin(arg), torch.cos(arg)
        out += float(tex.amp[k]) * (s[..., None] * cph[k] + c[..., None] * sph[k])
    # rectangles composited arithmetically (no boolean indexing, which
    # would synchronise with the host once per rectangle)
    for r in range(len(tex.rects)):
        x0, y0, x1, y1 = tex.rects[r]
        if tex.period is None:
            m = (x >= x0) & (x < x1)
        else:
            m = torch.remainder(x - x0, tex.period) < x1 - x0
        m = (m & (y >= y0) & (y < y1)).float()
        out += m[..., None] * torch.tensor(tex.offset[r], dtype=torch.float32, device=x.device)
    return out


# FFT sizes of the flow-noise fields: every strip's field is cut from a
# field smoothed on one of these periodic grids, so only two transform
# shapes are ever planned on the device
_FIELD_GRIDS = ((4096, 1024), (9216, 1024))


def _smooth_field_torch(rng, H, W, sigma, max_abs, device):
    import torch

    gh, gw = next(((a, b) for a, b in _FIELD_GRIDS if H <= a and W <= b), (H, W))
    noise = torch.from_numpy(rng.standard_normal((gh, gw)).astype(np.float32)).to(device)
    fy = torch.fft.fftfreq(gh, device=device)[:, None]
    fx = torch.fft.rfftfreq(gw, device=device)[None, :]
    g = torch.exp(-2.0 * np.pi ** 2 * sigma ** 2 * (fx ** 2 + fy ** 2))
    f = torch.fft.irfft2(torch.fft.rfft2(noise) * g, s=(gh, gw))[:H, :W].double()
    m = f.abs().max()
    return f * (max_abs / m) if float(m) > 0 else f


def make_config_strip_device(cfg: int, pano: int, strip: int, device="cuda"):
    """(L, R, axis) as uint8 tensors on ``device`` for the panorama
    workloads (cfg 2 and 4); see the section comment."""
    import torch

    if cfg not in (2, 4):
        raise ValueError("device generation covers the panorama workloads (2, 4)")
    H, W, axis = strip_shapes(cfg, pano)[strip]
    rng = rng_for(cfg, pano, strip)
    h, w = (H, W) if axis == 0 else (W, H)  # generated in the frame where the seam runs vertically
    tex = Texture(rng, h, w)
    sigma = max(128.0, 0.15 * min(h, w))
    ux = _smooth_field_torch(rng, h, w, sigma, 40.0, device)
    uy = _smooth_field_torch(rng, h, w, sigma, 8.0, device)
    wb = int(rng.integers(64, 129))
    xb = float(rng.uniform(0.25 * w, 0.6 * w))
    dob = float(rng.uniform(30.0, 40.0))
    tex_o = Texture(rng, h, w)
    gain = float(rng.uniform(0.9, 1.1))
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(0, 2 ** 62)))
    yy, xx = torch.meshgrid(torch.arange(h, device=device, dtype=torch.float64),
                            torch.arange(w, device=device, dtype=torch.float64), indexing="ij")
    Lf = _texture_torch(tex, xx, yy)
    Rf = gain * _texture_torch(tex, xx + ux, yy + uy)
    in_l = ((xx >= xb) & (xx < xb + wb))[..., None]
    Lf = torch.where(in_l, _texture_torch(tex_o, xx, yy), Lf)
    in_r = ((xx + dob >= xb) & (xx + dob < xb + wb))[..., None]
    Rf = torch.where(in_r, gain * _texture_torch(tex_o, xx + dob, yy), Rf)
    Lf += 2.0 * torch.randn(Lf.shape, generator=gen, device=device)
    Rf += 2.0 * torch.randn(Rf.shape, generator=gen, device=device)
    L = Lf.round_().clamp_(0, 255).to(torch.uint8)
    R = Rf.round_().clamp_(0, 255).to(torch.uint8)
    if axis == 1:
        L = L.transpose(0, 1).contiguous()
        R = R.transpose(0, 1).contiguous()
    return L, R, axis
