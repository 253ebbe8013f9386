"""CPU oracle (test infrastructure only).

A plain, slow reference implementation of the stitching hot path, written
from the paper (Section III.C, eq. (1), Code 1) and the readings listed in
``oracle.c``'s header. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. It shares no code
with the GPU library: the C source is built by ``oracle/build.py`` into
``oracle/liboracle.so`` and called through ``ctypes`` with numpy arrays.

Integer stages return int32 arrays; floating-point stages return float64.
Flows are ``H x W x 2`` with (x, y) = (column, row) components.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u8p = ctypes.POINTER(ctypes.c_uint8)
i32p = ctypes.POINTER(ctypes.c_int32)
i64p = ctypes.POINTER(ctypes.c_int64)
f64p = ctypes.POINTER(ctypes.c_double)
c_int, c_long, c_double = ctypes.c_int, ctypes.c_long, ctypes.c_double


@dataclass(frozen=True)
class Params:
    """Parameters of the flow method and the blend (the paper publishes
    none of their values; these are the adopted defaults)."""

    levels: int = 6
    patch: int = 2        # P: (2P+1)^2 patch
    radius: int = 2       # R: search radius per level
    radius_coarse: int = 4
    prop_steps: int = 2   # T
    median: int = 1       # M: (2M+1)^2 median
    lk_patch: int = 2     # window (2P+1)^2
    lk_iters: int = 2
    lk_eps: float = 25.0
    k_sharp: float = 10.0  # kSoftmaxSharpness
    k_flowmag: float = 20.0  # kFlowMagCoef
    blend_mode: int = 0   # 0 softmax (Code 1), 1 linear
    gain_comp: int = 0    # 1: compensate R's intensity by the ratio of intensity sums (off by default)

    @staticmethod
    def lean(**kw) -> "Params":
        d = dict(patch=1, radius=1, radius_coarse=3, prop_steps=1, lk_patch=1, lk_iters=1, lk_eps=9.0)
        d.update(kw)
        return Params(**d)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "orc_num_threads": (c_int, []),
        "orc_set_num_threads": (None, [c_int]),
        "orc_luma": (None, [u8p, c_int, c_int, c_long, u8p]),
        "orc_pyr_down": (None, [u8p, c_int, c_int, u8p]),
        "orc_upsample": (None, [i32p, c_int, c_int, c_int, c_int, i32p]),
        "orc_search": (None, [u8p, u8p, c_int, c_int, i32p, c_int, c_int, i32p, i32p]),
        "orc_propagate": (None, [u8p, u8p, c_int, c_int, c_int, c_int, i32p, i32p]),
        "orc_median": (None, [i32p, c_int, c_int, c_int, i32p]),
        "orc_level_sizes": (None, [c_int, c_int, c_int, i32p, i32p]),
        "orc_flow_int": (None, [u8p, u8p, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, i32p, i32p]),
        "orc_refine": (None, [u8p, u8p, c_int, c_int, i32p, c_int, c_int, c_double, f64p]),
        "orc_gain_comp": (None, [u8p, u8p, c_long]),
        "orc_flow_bidirectional": (None, [u8p, u8p, c_int, c_int, c_long, c_long,
                                          c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_double, c_int,
                                          f64p, f64p, i32p, i32p, i32p, i32p]),
        "orc_blend_coef": (c_double, [c_int, c_int, c_int, c_int, c_int]),
        "orc_blend": (None, [f64p, f64p, f64p, f64p, f64p, c_int, c_int, c_int, c_double, c_double, c_int,
                             f64p, u8p]),
        "orc_energy": (c_double, [f64p, f64p, f64p, c_int, c_int, c_double, c_double, f64p, f64p, f64p]),
        "orc_refine_gd": (None, [f64p, f64p, f64p, c_int, c_int, c_int, c_double, c_double, c_double,
                                 c_double, f64p]),
        "orc_blend_grad": (None, [f64p, f64p, f64p, f64p, f64p, c_int, c_int, c_int, c_double, c_double,
                                  c_int, f64p, f64p, f64p, f64p, f64p]),
        "orc_lk_level": (None, [u8p, u8p, c_int, c_int, f64p, c_int, c_int, c_double, f64p]),
        "orc_flow_lk": (None, [u8p, u8p, c_int, c_int, c_int, c_int, c_int, c_double, f64p]),
        "orc_flow_lk_bidirectional": (None, [u8p, u8p, c_int, c_int, c_long, c_long, c_int, c_int, c_int, c_double,
                                             c_int, f64p, f64p]),
        "orc_canvas_dist2": (None, [u8p, u8p, c_long, c_int, c_int, c_int, c_long, i32p, i32p, i64p, i64p]),
        "orc_canvas_dist2_rows": (None, [u8p, u8p, c_long, c_int, c_int, c_int, c_long, i32p, i32p, i64p, i64p]),
        "orc_canvas_blend": (None, [u8p, u8p, c_long, c_int, c_int, c_int, c_long, i32p, i32p, f64p]),
        "orc_overlap_box": (None, [u8p, u8p, c_long, c_int, c_int, c_int, i32p]),
        "orc_composite": (None, [f64p, f64p, u8p, u8p, c_long, c_int, c_int, c_int, f64p, f64p, i32p, c_int, f64p,
                                 c_double, c_double, c_int, f64p, u8p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a, typ):
    if a is None:
        return None
    return a.ctypes.data_as(typ)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (for timing)."""
    _load().orc_set_num_threads(int(n))


def level_sizes(H: int, W: int, N: int):
    hs = np.zeros(N, np.int32)
    ws = np.zeros(N, np.int32)
    _load().orc_level_sizes(H, W, N, _p(hs, i32p), _p(ws, i32p))
    return [(int(h), int(w)) for h, w in zip(hs, ws)]


def luma(rgb: np.ndarray) -> np.ndarray:
    rgb = _u8(rgb)
    H, W, _ = rgb.shape
    Y = np.empty((H, W), np.uint8)
    _load().orc_luma(_p(rgb, u8p), H, W, W * 3, _p(Y, u8p))
    return Y


def gain_comp(yl: np.ndarray, yr: np.ndarray) -> np.ndarray:
    """R's intensity after exposure compensation (a new array)."""
    yl = _u8(yl)
    out = _u8(yr).copy()
    _load().orc_gain_comp(_p(yl, u8p), _p(out, u8p), out.size)
    return out


def pyr_down(Y: np.ndarray) -> np.ndarray:
    Y = _u8(Y)
    H, W = Y.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2), np.uint8)
    _load().orc_pyr_down(_p(Y, u8p), H, W, _p(out, u8p))
    return out


def pyramid(Y: np.ndarray, N: int):
    levels = [_u8(Y)]
    for _ in range(1, N):
        levels.append(pyr_down(levels[-1]))
    return levels


def upsample(Dc: np.ndarray, H: int, W: int) -> np.ndarray:
    Dc = _i32(Dc)
    out = np.empty((H, W, 2), np.int32)
    _load().orc_upsample(_p(Dc, i32p), Dc.shape[0], Dc.shape[1], H, W, _p(out, i32p))
    return out


def search(ref, tgt, centre=None, P=2, R=2):
    ref, tgt = _u8(ref), _u8(tgt)
    H, W = ref.shape
    D = np.empty((H, W, 2), np.int32)
    cost = np.empty((H, W), np.int32)
    c = None if centre is None else _i32(centre)
    _load().orc_search(_p(ref, u8p), _p(tgt, u8p), H, W, _p(c, i32p), P, R, _p(D, i32p), _p(cost, i32p))
    return D, cost


def propagate(ref, tgt, D, P=2, T=2):
    ref, tgt, D = _u8(ref), _u8(tgt), _i32(D)
    H, W = ref.shape
    out = np.empty_like(D)
    _load().orc_propagate(_p(ref, u8p), _p(tgt, u8p), H, W, P, T, _p(D, i32p), _p(out, i32p))
    return out


def median(D, M=1):
    D = _i32(D)
    H, W, _ = D.shape
    out = np.empty_like(D)
    _load().orc_median(_p(D, i32p), H, W, M, _p(out, i32p))
    return out


def _split_levels(flat, sizes):
    out, off = [], 0
    for h, w in sizes:
        out.append(flat[off:off + h * w * 2].reshape(h, w, 2))
        off += h * w * 2
    return out


def flow_int(yref, ytgt, params: Params = Params()):
    """Integer coarse-to-fine chain of one direction. Returns two lists
    (level 0 first): raw search results and final per-level flows."""
    yref, ytgt = _u8(yref), _u8(ytgt)
    H, W = yref.shape
    sizes = level_sizes(H, W, params.levels)
    tot = sum(h * w for h, w in sizes)
    s = np.empty(tot * 2, np.int32)
    f = np.empty(tot * 2, np.int32)
    _load().orc_flow_int(_p(yref, u8p), _p(ytgt, u8p), H, W, params.levels, params.patch, params.radius,
                         params.radius_coarse, params.prop_steps, params.median, _p(s, i32p), _p(f, i32p))
    return _split_levels(s, sizes), _split_levels(f, sizes)


def refine(A, B, D0, params: Params = Params()):
    A, B, D0 = _u8(A), _u8(B), _i32(D0)
    H, W = A.shape
    u = np.empty((H, W, 2), np.float64)
    _load().orc_refine(_p(A, u8p), _p(B, u8p), H, W, _p(D0, i32p), params.lk_patch, params.lk_iters,
                       params.lk_eps, _p(u, f64p))
    return u


def flow_bidirectional(L, R, params: Params = Params(), levels_out: bool = False):
    """Both flows of a strip. Returns (flow_lr, flow_rl) as float64, plus
    a dict of the per-level integer results if ``levels_out``."""
    L, R = _u8(L), _u8(R)
    H, W, _ = L.shape
    sizes = level_sizes(H, W, params.levels)
    tot = sum(h * w for h, w in sizes)
    flr = np.empty((H, W, 2), np.float64)
    frl = np.empty((H, W, 2), np.float64)
    bufs = [np.empty(tot * 2, np.int32) for _ in range(4)]
    _load().orc_flow_bidirectional(_p(L, u8p), _p(R, u8p), H, W, W * 3, W * 3, params.levels, params.patch,
                                   params.radius, params.radius_coarse, params.prop_steps, params.median,
                                   params.lk_patch, params.lk_iters, params.lk_eps, params.gain_comp, _p(flr, f64p),
                                   _p(frl, f64p), *[_p(b, i32p) for b in bufs])
    if not levels_out:
        return flr, frl
    names = ["search_lr", "final_lr", "search_rl", "final_rl"]
    return flr, frl, {n: _split_levels(b, sizes) for n, b in zip(names, bufs)}


def blend_coef(H: int, W: int, axis: int = 0) -> np.ndarray:
    lib = _load()
    return np.array([[lib.orc_blend_coef(x, y, H, W, axis) for x in range(W)] for y in range(H)])


def blend(L, R, flow_lr, flow_rl, blend=None, axis: int = 0, params: Params = Params()):
    """Code 1 over a strip. Returns (F float64 H x W x 3, F uint8)."""
    Ld, Rd = _f64(L), _f64(R)
    H, W, _ = Ld.shape
    flr, frl = _f64(flow_lr), _f64(flow_rl)
    b = None if blend is None else _f64(blend)
    F = np.empty((H, W, 3), np.float64)
    F8 = np.empty((H, W, 3), np.uint8)
    _load().orc_blend(_p(Ld, f64p), _p(Rd, f64p), _p(flr, f64p), _p(frl, f64p), _p(b, f64p), axis, H, W,
                      params.k_sharp, params.k_flowmag, params.blend_mode, _p(F, f64p), _p(F8, u8p))
    return F, F8


def energy(Ref, Tgt, u, lam=0.05, eps=1e-3, grads: bool = True):
    Ref, Tgt, u = _f64(Ref), _f64(Tgt), _f64(u)
    H, W, _ = Ref.shape
    if grads:
        gu = np.empty((H, W, 2))
        gr = np.empty((H, W, 3))
        gt = np.empty((H, W, 3))
    else:
        gu = gr = gt = None
    E = _load().orc_energy(_p(Ref, f64p), _p(Tgt, f64p), _p(u, f64p), H, W, lam, eps, _p(gu, f64p),
                           _p(gr, f64p), _p(gt, f64p))
    return (E, gu, gr, gt) if grads else E


# Multi-level energy: the energy summed over a float pyramid of the images
# and the flow (an extension for gradient refinement; not in the paper).

_BINOM = np.array([1.0, 4.0, 6.0, 4.0, 1.0])


def pyr_down_float(x):
    """One level of the float pyramid: the 5 x 5 binomial filter of the
    luma pyramid (weights w_i w_j / 256) with clamped indices, without
    rounding, decimated to ceil(H / 2) x ceil(W / 2); every channel of an
    H x W (x C) array alike."""
    x = np.asarray(x, dtype=np.float64)
    H, W = x.shape[:2]
    h, w = (H + 1) // 2, (W + 1) // 2
    out = np.zeros((h, w) + x.shape[2:])
    Y, X = 2 * np.arange(h), 2 * np.arange(w)
    for j in range(5):
        ry = np.clip(Y + j - 2, 0, H - 1)
        for i in range(5):
            rx = np.clip(X + i - 2, 0, W - 1)
            out += (_BINOM[j] * _BINOM[i] / 256.0) * x[ry][:, rx]
    return out


def pyr_down_float_adjoint(g, shape):
    """The transpose of ``pyr_down_float``: every coarse value g(Y, X) is
    added back, with its weight, onto the fine pixels its taps read
    (clamped taps pile up on the border pixels). ``shape``: the fine shape."""
    g = np.asarray(g, dtype=np.float64)
    H, W = shape[:2]
    h, w = g.shape[:2]
    gc = g.reshape(h, w, -1)
    out = np.zeros((H * W, gc.shape[2]))
    Y, X = 2 * np.arange(h), 2 * np.arange(w)
    for j in range(5):
        ry = np.clip(Y + j - 2, 0, H - 1)
        for i in range(5):
            rx = np.clip(X + i - 2, 0, W - 1)
            idx = (ry[:, None] * W + rx[None, :]).ravel()  # the fine pixel each coarse value's tap read
            wt = _BINOM[j] * _BINOM[i] / 256.0
            for c in range(gc.shape[2]):
                out[:, c] += np.bincount(idx, weights=wt * gc[:, :, c].ravel(), minlength=H * W)
    return out.reshape(tuple(shape))


def energy_ms(Ref, Tgt, u, levels: int, lam=0.05, eps=1e-3, grads: bool = True):
    """E_ms = sum over pyramid levels k = 0 .. levels - 1 of the energy of
    level k (``energy``), with Ref_k, Tgt_k the images reduced k times by
    ``pyr_down_float`` and u_k the flow reduced likewise and halved at each
    reduction (displacements in level-k pixels). Gradients with respect to
    the level-0 u, Ref and Tgt by the chain rule, coarse to fine:
    G_k = g_k + (1/2 for u) pyr_down_float_adjoint(G_{k+1})."""
    R, T, U = [_f64(Ref)], [_f64(Tgt)], [_f64(u)]
    for _ in range(1, levels):
        R.append(pyr_down_float(R[-1]))
        T.append(pyr_down_float(T[-1]))
        U.append(pyr_down_float(U[-1]) / 2.0)
    res = [energy(R[k], T[k], U[k], lam, eps, grads=grads) for k in range(levels)]
    if not grads:
        return float(sum(res))
    E = sum(r[0] for r in res)
    Gu, Gr, Gt = res[-1][1], res[-1][2], res[-1][3]
    for k in range(levels - 2, -1, -1):
        Gu = res[k][1] + 0.5 * pyr_down_float_adjoint(Gu, U[k].shape)
        Gr = res[k][2] + pyr_down_float_adjoint(Gr, R[k].shape)
        Gt = res[k][3] + pyr_down_float_adjoint(Gt, T[k].shape)
    return E, Gu, Gr, Gt


def refine_gd_ms(Ref, Tgt, u, levels: int, steps=20, eta=0.5, lam=0.05, eps=1e-3, clip=0.25):
    """Gradient descent on the multi-level energy, u <- u - clip(eta dE_ms/du,
    +-clip) per component, ``steps`` times; returns the flow."""
    u = _f64(u).copy()
    for _ in range(steps):
        _, gu, _, _ = energy_ms(Ref, Tgt, u, levels, lam, eps)
        u -= np.clip(eta * gu, -clip, clip)
    return u


def refine_gd(Ref, Tgt, u, steps=50, eta=0.5, lam=0.05, eps=1e-3, clip=0.25):
    Ref, Tgt = _f64(Ref), _f64(Tgt)
    u = _f64(u).copy()
    H, W, _ = Ref.shape
    hist = np.empty(steps + 1)
    _load().orc_refine_gd(_p(Ref, f64p), _p(Tgt, f64p), _p(u, f64p), H, W, steps, eta, lam, eps, clip,
                          _p(hist, f64p))
    return u, hist


def blend_grad(L, R, flow_lr, flow_rl, g_F, blend=None, axis: int = 0, params: Params = Params()):
    """Adjoint of Code 1. Returns (g_flow_lr, g_flow_rl, g_L, g_R)."""
    Ld, Rd = _f64(L), _f64(R)
    H, W, _ = Ld.shape
    flr, frl, gF = _f64(flow_lr), _f64(flow_rl), _f64(g_F)
    b = None if blend is None else _f64(blend)
    out = [np.empty((H, W, 2)), np.empty((H, W, 2)), np.empty((H, W, 3)), np.empty((H, W, 3))]
    _load().orc_blend_grad(_p(Ld, f64p), _p(Rd, f64p), _p(flr, f64p), _p(frl, f64p), _p(b, f64p), axis, H, W,
                           params.k_sharp, params.k_flowmag, params.blend_mode, _p(gF, f64p),
                           *[_p(o, f64p) for o in out])
    return tuple(out)


# ---------------------------------------------------------------------------
# Canvas (eq. (1) and Code 1 with coverage masks of any shape)


def _points(H, W, points):
    if points is None:
        ys, xs = np.mgrid[0:H, 0:W]
        return _i32(xs.ravel()), _i32(ys.ravel())
    pts = np.asarray(points)
    return _i32(pts[:, 0]), _i32(pts[:, 1])


def canvas_dist2(mask_L, mask_R, points=None, periodic: bool = False):
    """Squared distances (int64) from canvas points to the nearest Area1
    and Area2 pixel (-1 if that area is empty), by brute force. ``points``
    is an (n, 2) array of (x, y); None = every pixel (returned H x W).
    ``periodic``: the canvas wraps in x (column offsets the shorter way
    round)."""
    mL, mR = _u8(mask_L), _u8(mask_R)
    H, W = mL.shape
    xs, ys = _points(H, W, points)
    n = xs.size
    d1, d2 = np.empty(n, np.int64), np.empty(n, np.int64)
    _load().orc_canvas_dist2(_p(mL, u8p), _p(mR, u8p), W, H, W, int(periodic), n, _p(xs, i32p), _p(ys, i32p),
                             _p(d1, i64p), _p(d2, i64p))
    if points is None:
        return d1.reshape(H, W), d2.reshape(H, W)
    return d1, d2


def canvas_dist2_rows(mask_L, mask_R, points=None, periodic: bool = False):
    """The squared distances of ``canvas_dist2`` in two stages (nearest
    pixel of the area along every row, then the minimum over rows of
    dy^2 + dx^2): the same values, fast enough for long lists of points on
    large canvases."""
    mL, mR = _u8(mask_L), _u8(mask_R)
    H, W = mL.shape
    xs, ys = _points(H, W, points)
    n = xs.size
    d1, d2 = np.empty(n, np.int64), np.empty(n, np.int64)
    _load().orc_canvas_dist2_rows(_p(mL, u8p), _p(mR, u8p), W, H, W, int(periodic), n, _p(xs, i32p),
                                  _p(ys, i32p), _p(d1, i64p), _p(d2, i64p))
    if points is None:
        return d1.reshape(H, W), d2.reshape(H, W)
    return d1, d2


def canvas_blend(mask_L, mask_R, points=None, periodic: bool = False):
    """eq. (1) on a canvas (float64), at ``points`` or at every pixel."""
    mL, mR = _u8(mask_L), _u8(mask_R)
    H, W = mL.shape
    xs, ys = _points(H, W, points)
    out = np.empty(xs.size, np.float64)
    _load().orc_canvas_blend(_p(mL, u8p), _p(mR, u8p), W, H, W, int(periodic), xs.size, _p(xs, i32p),
                             _p(ys, i32p), _p(out, f64p))
    return out.reshape(H, W) if points is None else out


def overlap_box(mask_L, mask_R, periodic: bool = False):
    """Bounding box of Area3 as (x, y, w, h); zeros if there is none. On a
    periodic canvas the shortest circular run of columns holding Area3
    (x + w may exceed W)."""
    mL, mR = _u8(mask_L), _u8(mask_R)
    H, W = mL.shape
    box = np.zeros(4, np.int32)
    _load().orc_overlap_box(_p(mL, u8p), _p(mR, u8p), W, H, W, int(periodic), _p(box, i32p))
    return tuple(int(v) for v in box)


def composite(L, R, mask_L, mask_R, flow_lr, flow_rl, box, axis: int = 0, blend=None, params: Params = Params(),
              periodic: bool = False):
    """Code 1 over a canvas; flows cover the overlap box (on a periodic
    canvas its columns wrap). Returns (F float64 H x W x 3, F uint8)."""
    Ld, Rd = _f64(L), _f64(R)
    mL, mR = _u8(mask_L), _u8(mask_R)
    H, W, _ = Ld.shape
    flr, frl = _f64(flow_lr), _f64(flow_rl)
    b = None if blend is None else _f64(blend)
    bx = _i32(box)
    F = np.empty((H, W, 3), np.float64)
    F8 = np.empty((H, W, 3), np.uint8)
    _load().orc_composite(_p(Ld, f64p), _p(Rd, f64p), _p(mL, u8p), _p(mR, u8p), W, H, W, int(periodic), _p(flr, f64p),
                          _p(frl, f64p), _p(bx, i32p), axis, _p(b, f64p), params.k_sharp, params.k_flowmag,
                          params.blend_mode, _p(F, f64p), _p(F8, u8p))
    return F, F8


# ---------------------------------------------------------------------------
# Classic coarse-to-fine Lucas-Kanade (float flows at every level)


def lk_level(A, B, seed=None, P: int = 2, K: int = 4, eps: float = 25.0):
    """One pyramid level of the classic method: K Gauss-Newton steps from
    ``seed`` (H x W x 2, None = 0)."""
    A, B = _u8(A), _u8(B)
    H, W = A.shape
    sd = None if seed is None else _f64(seed)
    u = np.empty((H, W, 2), np.float64)
    _load().orc_lk_level(_p(A, u8p), _p(B, u8p), H, W, _p(sd, f64p), P, K, eps, _p(u, f64p))
    return u


def flow_lk(yref, ytgt, N: int, P: int = 2, K: int = 4, eps: float = 25.0):
    """One direction over the pyramid; returns every level's flow, level 0
    first."""
    yref, ytgt = _u8(yref), _u8(ytgt)
    H, W = yref.shape
    sizes = level_sizes(H, W, N)
    tot = sum(h * w for h, w in sizes)
    f = np.empty(tot * 2, np.float64)
    _load().orc_flow_lk(_p(yref, u8p), _p(ytgt, u8p), H, W, N, P, K, eps, _p(f, f64p))
    return _split_levels(f, sizes)


def flow_lk_bidirectional(L, R, params: Params = Params(), K: int | None = None):
    """Both flows of a strip with the classic method (K = params.lk_iters
    Gauss-Newton steps per level). Returns (levels_lr, levels_rl), each a
    list of H_k x W_k x 2 float64 flows, level 0 first."""
    L, R = _u8(L), _u8(R)
    H, W, _ = L.shape
    N = params.levels
    K = params.lk_iters if K is None else K
    sizes = level_sizes(H, W, N)
    tot = sum(h * w for h, w in sizes)
    a, b = np.empty(tot * 2, np.float64), np.empty(tot * 2, np.float64)
    _load().orc_flow_lk_bidirectional(_p(L, u8p), _p(R, u8p), H, W, W * 3, W * 3, N, params.lk_patch, K,
                                      params.lk_eps, params.gain_comp, _p(a, f64p), _p(b, f64p))
    return _split_levels(a, sizes), _split_levels(b, sizes)
