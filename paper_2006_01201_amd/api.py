"""Torch-facing wrapper of libabf: tensors in, tensors out.

PyTorch supplies device memory (the workspace and the outputs are
``torch.empty`` tensors) and the stream (the current stream); every step of
the computation runs in libabf's HIP kernels. Shape and dtype checks and
argument marshalling are all this module does.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, fields

import torch

from . import _abi

STAGES = ("luma", "pyramid", "search", "propagation", "refine", "blend")


@dataclass(frozen=True)
class Params:
    """Mirror of ``abf_params`` (include/abf.h) with the adopted defaults."""

    levels: int = 6
    patch: int = 2
    radius: int = 2
    radius_coarse: int = 4
    prop_steps: int = 2
    median: int = 1
    lk_patch: int = 2
    lk_iters: int = 2
    lk_eps: float = 25.0
    k_sharp: float = 10.0
    k_flowmag: float = 20.0
    blend_mode: int = 0
    gain_comp: int = 0  # exposure step off: colour correction is the caller's pre-processing
    flow_method: int = 0  # 0: integer search + refinement; 1: classic coarse-to-fine Lucas-Kanade

    def to_c(self) -> _abi.AbfParams:
        p = _abi.AbfParams()
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p

    @staticmethod
    def lean(**kw) -> "Params":
        d = dict(patch=1, radius=1, radius_coarse=3, prop_steps=1, lk_patch=1, lk_iters=1, lk_eps=9.0)
        d.update(kw)
        return Params(**d)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _img_u8(t: torch.Tensor, name: str):
    if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[2] != 3 or not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA uint8 tensor of shape (H, W, 3), got {t.dtype} {tuple(t.shape)}")
    if t.stride(2) != 1 or t.stride(1) != 3:
        raise ValueError(f"{name}: pixels must be interleaved RGB (strides (pitch, 3, 1)), got {t.stride()}")
    return t.shape[0], t.shape[1], t.stride(0)


def _mask(t: torch.Tensor, name: str):
    if t.dtype != torch.uint8 or t.dim() != 2 or not t.is_cuda or t.stride(1) != 1:
        raise ValueError(f"{name}: expected a CUDA uint8 (H, W) tensor with unit column stride, "
                         f"got {t.dtype} {tuple(t.shape)}")
    return t.shape[0], t.shape[1], t.stride(0)


def _f32(t: torch.Tensor, shape, name: str):
    if t.dtype != torch.float32 or tuple(t.shape) != tuple(shape) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous CUDA float32 tensor {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")
    return t.data_ptr()


class Batch:
    """Strip descriptors plus their output tensors, reusable across calls."""

    def __init__(self, strips, outputs, arr):
        self.strips = strips
        self.outputs = outputs
        self.arr = arr
        self.n = len(strips)


class Plan:
    """An abf_plan with its workspace."""

    def __init__(self, params: Params = Params(), max_strips: int = 1, max_pixels: int | None = None,
                 max_H: int = 4096, max_W: int = 4096, canvas: tuple[int, int] | None = None):
        """``canvas`` = (H, W): also size the workspace for canvases up to
        that size (canvas compositing)."""
        if max_pixels is None:
            max_pixels = max_strips * max_H * max_W
        self.params = params
        st, h = _abi.create_plan(params.to_c(), max_strips, max_pixels, max_H, max_W)
        _abi.check(st, None, "abf_create_plan")
        self.h = h
        nbytes = _abi.workspace_bytes(h)
        if canvas is not None:
            nbytes = max(nbytes, _abi.canvas_workspace_bytes(h, *canvas), _abi.merge_workspace_bytes(h, *canvas))
        self._bind(nbytes)

    def _bind(self, nbytes: int):
        """Allocates (torch) and binds a workspace of ``nbytes``."""
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        self._ws_off = (-base) % 256
        _abi.check(_abi.bind_workspace(self.h, base + self._ws_off, nbytes), self.h, "abf_bind_workspace")
        self.workspace_bytes = nbytes

    def _ensure_ms_workspace(self, H: int, W: int, levels: int):
        need = _abi.energy_ms_workspace_bytes(self.h, H, W, levels)
        if need > self.workspace_bytes:
            torch.cuda.current_stream().synchronize()  # the old workspace may still be in use
            self._bind(need)

    def close(self):
        if getattr(self, "h", None):
            _abi.destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the paper's calls ---------------------------------------------
    def flow_bidirectional(self, L: torch.Tensor, R: torch.Tensor, out=None):
        """FlowLtoR and FlowRtoL (float32 H x W x 2) of one strip."""
        H, W, pl = _img_u8(L, "L")
        H2, W2, pr = _img_u8(R, "R")
        if (H, W) != (H2, W2):
            raise ValueError("L and R differ in size")
        if out is None:
            flr = torch.empty((H, W, 2), dtype=torch.float32, device=L.device)
            frl = torch.empty((H, W, 2), dtype=torch.float32, device=L.device)
        else:
            flr, frl = out
        st = _abi.flow_bidirectional(self.h, L.data_ptr(), R.data_ptr(), H, W, pl, pr,
                                     _f32(flr, (H, W, 2), "flow_LtoR"), _f32(frl, (H, W, 2), "flow_RtoL"), _stream())
        _abi.check(st, self.h, "abf_flow_bidirectional")
        return flr, frl

    def flow_bidirectional_noalloc(self, L: torch.Tensor, R: torch.Tensor, out):
        """flow_bidirectional with the library's static scratch instead of
        the workspace (abf_flow_bidirectional_noalloc); ``out`` = the two
        caller-allocated flow tensors."""
        H, W, pl = _img_u8(L, "L")
        H2, W2, pr = _img_u8(R, "R")
        if (H, W) != (H2, W2):
            raise ValueError("L and R differ in size")
        flr, frl = out
        st = _abi.flow_bidirectional_noalloc(self.h, L.data_ptr(), R.data_ptr(), H, W, pl, pr,
                                             _f32(flr, (H, W, 2), "flow_LtoR"), _f32(frl, (H, W, 2), "flow_RtoL"),
                                             _stream())
        _abi.check(st, self.h, "abf_flow_bidirectional_noalloc")
        return flr, frl

    def blend_asymmetric(self, L, R, flow_lr, flow_rl, blend=None, axis: int = 0, f32: bool = False, out=None):
        """Code 1 over one strip; returns F (uint8 H x W x 3) and, if
        ``f32``, the unrounded composite (float32 H x W x 3)."""
        H, W, pl = _img_u8(L, "L")
        _, _, pr = _img_u8(R, "R")
        if out is None:
            F = torch.empty((H, W, 3), dtype=torch.uint8, device=L.device)
        else:
            F = out
        _, _, pf = _img_u8(F, "F")
        Ff = torch.empty((H, W, 3), dtype=torch.float32, device=L.device) if f32 else None
        bp = _f32(blend, (H, W), "blend") if blend is not None else None
        st = _abi.blend_asymmetric(self.h, L.data_ptr(), R.data_ptr(), _f32(flow_lr, (H, W, 2), "flow_LtoR"),
                                   _f32(flow_rl, (H, W, 2), "flow_RtoL"), bp, axis, H, W, pl, pr, F.data_ptr(), pf,
                                   Ff.data_ptr() if Ff is not None else None, _stream())
        _abi.check(st, self.h, "abf_blend_asymmetric")
        return (F, Ff) if f32 else F

    def make_batch(self, strips, f32: bool = False) -> Batch:
        """strips: sequence of (L, R, axis) or (L, R, axis, blend). Allocates
        the outputs once; ``stitch`` can then be called repeatedly."""
        arr = (_abi.AbfStrip * len(strips))()
        outs = []
        keep = []
        for i, s in enumerate(strips):
            L, R, axis = s[0], s[1], s[2]
            blend = s[3] if len(s) > 3 else None
            H, W, pl = _img_u8(L, "L")
            _, _, pr = _img_u8(R, "R")
            o = {
                "flow_lr": torch.empty((H, W, 2), dtype=torch.float32, device=L.device),
                "flow_rl": torch.empty((H, W, 2), dtype=torch.float32, device=L.device),
                "F": torch.empty((H, W, 3), dtype=torch.uint8, device=L.device),
                "F_f32": torch.empty((H, W, 3), dtype=torch.float32, device=L.device) if f32 else None,
            }
            d = arr[i]
            d.L, d.R, d.H, d.W, d.pitch_L, d.pitch_R, d.axis = L.data_ptr(), R.data_ptr(), H, W, pl, pr, axis
            d.blend = _f32(blend, (H, W), "blend") if blend is not None else None
            d.flow_LtoR, d.flow_RtoL = o["flow_lr"].data_ptr(), o["flow_rl"].data_ptr()
            d.F, d.pitch_F = o["F"].data_ptr(), 3 * W
            d.F_f32 = o["F_f32"].data_ptr() if f32 else None
            outs.append(o)
            keep.append(s)
        return Batch(keep, outs, arr)

    def stitch(self, batch: Batch, use_graph: bool = True):
        st = _abi.stitch_strips(self.h, batch.arr, batch.n, int(use_graph), _stream())
        _abi.check(st, self.h, "abf_stitch_strips")
        return batch.outputs

    def stitch_strips(self, strips, use_graph: bool = True, f32: bool = False):
        return self.stitch(self.make_batch(strips, f32), use_graph)

    def tune(self, batch: Batch):
        _abi.check(_abi.tune(self.h, batch.arr, batch.n, _stream()), self.h, "abf_tune")

    def profile(self, batch: Batch, reps: int = 5):
        """Mean ms per launch, indexed [stage][level] (eager launches
        bracketed by HIP events on the current stream)."""
        st, ms = _abi.profile(self.h, batch.arr, batch.n, reps, _stream())
        _abi.check(st, self.h, "abf_profile")
        return ms

    def get_launch(self, stage: int, size_class: int):
        st, th, g = _abi.get_launch(self.h, stage, size_class)
        _abi.check(st, self.h, "abf_get_launch")
        return th, g

    def set_launch(self, stage: int, size_class: int, tile_h: int, grid: int):
        _abi.check(_abi.set_launch(self.h, stage, size_class, tile_h, grid), self.h, "abf_set_launch")

    # -- differentiable path (float images) ------------------------------
    def energy(self, ref, tgt, u, lam: float = 0.05, eps: float = 1e-3, grads: bool = True,
               deterministic: bool = False):
        """Photometric Charbonnier + lam * TV energy of flow ``u`` (float32
        H x W x 2) between float32 RGB images (H x W x 3). Returns E (a
        1-element tensor) and, if ``grads``, dE/du, dE/dref, dE/dtgt."""
        H, W = u.shape[0], u.shape[1]
        E = torch.empty(1, dtype=torch.float32, device=u.device)
        gu = torch.empty_like(u) if grads else None
        gr = torch.empty_like(ref) if grads else None
        gt = torch.empty_like(tgt) if grads else None
        st = _abi.energy(self.h, _f32(ref, (H, W, 3), "ref"), _f32(tgt, (H, W, 3), "tgt"), _f32(u, (H, W, 2), "u"),
                         H, W, lam, eps, E.data_ptr(), gu.data_ptr() if grads else None,
                         gr.data_ptr() if grads else None, gt.data_ptr() if grads else None, int(deterministic),
                         _stream())
        _abi.check(st, self.h, "abf_energy")
        return (E, gu, gr, gt) if grads else E

    def refine_flow(self, ref, tgt, u, steps: int = 50, eta: float = 0.5, lam: float = 0.05, eps: float = 1e-3,
                    clip: float = 0.25):
        """``steps`` gradient-descent steps on the energy, in place on ``u``."""
        H, W = u.shape[0], u.shape[1]
        st = _abi.refine_flow(self.h, _f32(ref, (H, W, 3), "ref"), _f32(tgt, (H, W, 3), "tgt"),
                              _f32(u, (H, W, 2), "u"), H, W, steps, eta, lam, eps, clip, _stream())
        _abi.check(st, self.h, "abf_refine_flow")
        return u

    def energy_ms(self, ref, tgt, u, levels: int, lam: float = 0.05, eps: float = 1e-3, grads: bool = True,
                  deterministic: bool = False):
        """The energy summed over ``levels`` levels of a float pyramid of
        the images and the flow; returns E and, if ``grads``, its gradients
        with respect to the level-0 u, ref and tgt (pyramid levels built
        and dropped within the call)."""
        H, W = u.shape[0], u.shape[1]
        self._ensure_ms_workspace(H, W, levels)
        E = torch.empty(1, dtype=torch.float32, device=u.device)
        gu = torch.empty_like(u) if grads else None
        gr = torch.empty_like(ref) if grads else None
        gt = torch.empty_like(tgt) if grads else None
        st = _abi.energy_ms(self.h, _f32(ref, (H, W, 3), "ref"), _f32(tgt, (H, W, 3), "tgt"),
                            _f32(u, (H, W, 2), "u"), H, W, levels, lam, eps, E.data_ptr(),
                            gu.data_ptr() if grads else None, gr.data_ptr() if grads else None,
                            gt.data_ptr() if grads else None, int(deterministic), _stream())
        _abi.check(st, self.h, "abf_energy_ms")
        return (E, gu, gr, gt) if grads else E

    def refine_flow_ms(self, ref, tgt, u, levels: int, steps: int = 20, eta: float = 0.5, lam: float = 0.05,
                       eps: float = 1e-3, clip: float = 0.25):
        """``steps`` gradient-descent steps on the multi-level energy, in
        place on ``u``."""
        H, W = u.shape[0], u.shape[1]
        self._ensure_ms_workspace(H, W, levels)
        st = _abi.refine_flow_ms(self.h, _f32(ref, (H, W, 3), "ref"), _f32(tgt, (H, W, 3), "tgt"),
                                 _f32(u, (H, W, 2), "u"), H, W, levels, steps, eta, lam, eps, clip, _stream())
        _abi.check(st, self.h, "abf_refine_flow_ms")
        return u

    def refine_strips(self, items, steps: int = 20, eta: float = 0.5, lam: float = 0.05, eps: float = 1e-3,
                      clip: float = 0.25):
        """Batched ``refine_flow``: items are (ref, tgt, u) triples; every u
        is refined in place, one launch per step for all of them."""
        arr = (_abi.AbfRefineStrip * len(items))()
        for i, (ref, tgt, u) in enumerate(items):
            H, W = u.shape[0], u.shape[1]
            arr[i].Ref = _f32(ref, (H, W, 3), "ref")
            arr[i].Tgt = _f32(tgt, (H, W, 3), "tgt")
            arr[i].u = _f32(u, (H, W, 2), "u")
            arr[i].H, arr[i].W = H, W
        st = _abi.refine_strips(self.h, arr, len(items), steps, eta, lam, eps, clip, _stream())
        _abi.check(st, self.h, "abf_refine_strips")
        return [it[2] for it in items]

    def blend_f32(self, L, R, flow_lr, flow_rl, blend=None, axis: int = 0):
        """Code 1 over float32 RGB images; returns F (float32 H x W x 3)."""
        H, W = L.shape[0], L.shape[1]
        F = torch.empty((H, W, 3), dtype=torch.float32, device=L.device)
        st = _abi.blend_asymmetric_f32(self.h, _f32(L, (H, W, 3), "L"), _f32(R, (H, W, 3), "R"),
                                       _f32(flow_lr, (H, W, 2), "flow_LtoR"), _f32(flow_rl, (H, W, 2), "flow_RtoL"),
                                       _f32(blend, (H, W), "blend") if blend is not None else None, axis, H, W,
                                       F.data_ptr(), _stream())
        _abi.check(st, self.h, "abf_blend_asymmetric_f32")
        return F

    def blend_backward(self, L, R, flow_lr, flow_rl, g_F, blend=None, axis: int = 0, deterministic: bool = False):
        """Adjoint of Code 1: (dF/dflow_LtoR, dF/dflow_RtoL, dF/dL, dF/dR)
        contracted with g_F; ``deterministic`` sums the image gradients in
        an order-independent fixed point (bitwise repeatable)."""
        H, W = L.shape[0], L.shape[1]
        out = [torch.empty((H, W, 2), dtype=torch.float32, device=L.device) for _ in range(2)]
        out += [torch.empty((H, W, 3), dtype=torch.float32, device=L.device) for _ in range(2)]
        st = _abi.blend_backward(self.h, _f32(L, (H, W, 3), "L"), _f32(R, (H, W, 3), "R"),
                                 _f32(flow_lr, (H, W, 2), "flow_LtoR"), _f32(flow_rl, (H, W, 2), "flow_RtoL"),
                                 _f32(blend, (H, W), "blend") if blend is not None else None, axis, H, W,
                                 _f32(g_F, (H, W, 3), "g_F"), *[o.data_ptr() for o in out], int(deterministic),
                                 _stream())
        _abi.check(st, self.h, "abf_blend_backward")
        return tuple(out)

    # -- inspection ------------------------------------------------------
    # -- canvas compositing (eq. (1) and Code 1 with general areas) ----
    def overlap_box(self, mask_L, mask_R, out=None, periodic: bool = False):
        """Bounding box (x, y, w, h) of Area3: a host tuple (synchronises),
        or, with ``out`` (int32 CUDA tensor of 4), written there without
        synchronising. ``periodic``: the canvas wraps in x (a 360-degree
        panorama) and the box's columns may run past W - 1 to 0."""
        H, W, pm = _mask(mask_L, "mask_L")
        if _mask(mask_R, "mask_R") != (H, W, pm):
            raise ValueError("mask_L and mask_R differ in shape or pitch")
        box = torch.empty(4, dtype=torch.int32, device=mask_L.device) if out is None else out
        if box.dtype != torch.int32 or box.numel() != 4 or not box.is_cuda or not box.is_contiguous():
            raise ValueError("out: expected a contiguous CUDA int32 tensor of 4")
        st = _abi.overlap_box(self.h, mask_L.data_ptr(), mask_R.data_ptr(), H, W, pm, int(periodic), box.data_ptr(),
                              _stream())
        _abi.check(st, self.h, "abf_overlap_box")
        return box if out is not None else tuple(int(v) for v in box.cpu())

    def canvas_blend(self, mask_L, mask_R, distances: bool = False, out=None, periodic: bool = False):
        """eq. (1) over the canvas (float32 H x W, into ``out`` if given);
        with ``distances`` also the squared distances to Area1 and Area2
        (int32, -1 = empty)."""
        H, W, pm = _mask(mask_L, "mask_L")
        if _mask(mask_R, "mask_R") != (H, W, pm):
            raise ValueError("mask_L and mask_R differ in shape or pitch")
        dev = mask_L.device
        B = torch.empty((H, W), dtype=torch.float32, device=dev) if out is None else out
        _f32(B, (H, W), "out")
        d1 = torch.empty((H, W), dtype=torch.int32, device=dev) if distances else None
        d2 = torch.empty((H, W), dtype=torch.int32, device=dev) if distances else None
        st = _abi.canvas_blend(self.h, mask_L.data_ptr(), mask_R.data_ptr(), H, W, pm, int(periodic), B.data_ptr(), W,
                               d1.data_ptr() if distances else None, d2.data_ptr() if distances else None, W,
                               _stream())
        _abi.check(st, self.h, "abf_canvas_blend")
        return (B, d1, d2) if distances else B

    def composite_canvas(self, L, R, mask_L, mask_R, flow_lr, flow_rl, box, axis: int = 0, blend=None,
                         f32: bool = False, out=None, periodic: bool = False):
        """Code 1 over the canvas; flows cover the overlap ``box``. Returns
        F (uint8 H x W x 3) and, if ``f32``, the unrounded composite."""
        H, W, pl = _img_u8(L, "L")
        H2, W2, pr = _img_u8(R, "R")
        Hm, Wm, pm = _mask(mask_L, "mask_L")
        if (H, W) != (H2, W2) or (H, W) != (Hm, Wm) or _mask(mask_R, "mask_R") != (Hm, Wm, pm):
            raise ValueError("canvas inputs differ in size")
        bx, by, bw, bh = (int(v) for v in box)
        F = torch.empty((H, W, 3), dtype=torch.uint8, device=L.device) if out is None else out
        _, _, pf = _img_u8(F, "F")
        Ff = torch.empty((H, W, 3), dtype=torch.float32, device=L.device) if f32 else None
        fl = fr = None
        if bw > 0 and bh > 0:
            fl = _f32(flow_lr, (bh, bw, 2), "flow_LtoR")
            fr = _f32(flow_rl, (bh, bw, 2), "flow_RtoL")
        bp, pb = None, 0
        if blend is not None:
            if blend.dtype != torch.float32 or blend.dim() != 2 or tuple(blend.shape) != (H, W) or blend.stride(1) != 1:
                raise ValueError("blend: expected a CUDA float32 (H, W) tensor with unit column stride")
            bp, pb = blend.data_ptr(), blend.stride(0)
        st = _abi.composite_canvas(self.h, L.data_ptr(), R.data_ptr(), mask_L.data_ptr(), mask_R.data_ptr(), H, W,
                                   pl, pr, pm, int(periodic), fl, fr, (bx, by, bw, bh), axis, bp, pb, F.data_ptr(), pf,
                                   Ff.data_ptr() if Ff is not None else None, _stream())
        _abi.check(st, self.h, "abf_composite_canvas")
        return (F, Ff) if f32 else F

    def stitch_canvas(self, L, R, mask_L, mask_R, axis: int = 0, f32: bool = False):
        """The whole pair: overlap box, both flows on its crops, eq. (1)
        and Code 1 over the canvas. Returns (F[, F_f32], box, flow_lr,
        flow_rl)."""
        box = self.overlap_box(mask_L, mask_R)
        bx, by, bw, bh = box
        flr = frl = None
        if bw > 0 and bh > 0:
            flr, frl = self.flow_bidirectional(L[by:by + bh, bx:bx + bw], R[by:by + bh, bx:bx + bw])
        res = self.composite_canvas(L, R, mask_L, mask_R, flr, frl, box, axis=axis, f32=f32)
        return (*res, box, flr, frl) if f32 else (res, box, flr, frl)

    def merge_photos(self, photos, out=None, periodic: bool = False):
        """Repeated pairwise merging of photos placed on one canvas.
        ``photos``: list of (image uint8 H x W x 3, mask uint8 H x W, axis,
        side), merged in list order (photo 0 starts the canvas); with
        ``periodic`` the canvas wraps in x and the ring closes across it.
        Returns (canvas uint8 H x W x 3, coverage uint8 H x W, boxes)."""
        if not photos:
            raise ValueError("no photos")
        H, W, pm = _mask(photos[0][1], "mask")
        arr = (_abi.AbfPhoto * len(photos))()
        keep = []
        for i, (img, mask, axis, side) in enumerate(photos):
            h, w, pi = _img_u8(img, f"photo {i}")
            if (h, w) != (H, W) or _mask(mask, f"mask {i}") != (H, W, pm):
                raise ValueError(f"photo {i}: canvas size or mask pitch differs")
            arr[i] = _abi.AbfPhoto(img.data_ptr(), mask.data_ptr(), pi, axis, side)
            keep.append((img, mask))
        dev = photos[0][0].device
        canvas = torch.empty((H, W, 3), dtype=torch.uint8, device=dev) if out is None else out
        spare = torch.empty_like(canvas)
        cov = torch.empty((H, pm), dtype=torch.uint8, device=dev)[:, :W]
        _, _, pc = _img_u8(canvas, "out")
        st, boxes = _abi.merge_photos(self.h, arr, len(photos), H, W, pm, int(periodic), canvas.data_ptr(), pc,
                                      spare.data_ptr(), spare.stride(0), cov.data_ptr(), _stream())
        _abi.check(st, self.h, "abf_merge_photos")
        return canvas, cov, boxes

    def lk_level_flow(self, strip: int, level: int, direction: int) -> torch.Tensor:
        """Flow method 1: the float64 flow (H x W x 2) of pyramid level
        ``level`` >= 1 of the last flow call (its x and y planes)."""
        comps = []
        for kind in (1, 2):
            st, ptr, H, W, pitch = _abi.workspace_view(self.h, kind, strip, level, direction)
            _abi.check(st, self.h, "abf_workspace_view")
            off = ptr - self._ws.data_ptr()
            comps.append(self._ws[off:off + H * pitch * 8].view(torch.float64).view(H, pitch)[:, :W])
        return torch.stack(comps, dim=-1).clone()

    def view(self, kind: int, strip: int, level: int, direction: int) -> torch.Tensor:
        """A copy of one intermediate of the last flow call: kind 0 luma
        (uint8 H x W), 1 raw search / 2 final integer flow (int16 H x W x 2)."""
        st, ptr, H, W, pitch = _abi.workspace_view(self.h, kind, strip, level, direction)
        _abi.check(st, self.h, "abf_workspace_view")
        off = ptr - self._ws.data_ptr()
        if kind == 0:
            t = self._ws[off:off + H * pitch].view(H, pitch)[:, :W]
        else:
            t = self._ws[off:off + H * pitch * 4].view(torch.int16).view(H, pitch, 2)[:, :W]
        return t.clone()
