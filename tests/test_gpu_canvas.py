"""GPU parity of canvas compositing (eq. (1) with coverage masks of any
shape, Code 1 with its Area1 / Area2 / else branches) against the CPU
oracle: the overlap box and the squared distances bit for bit, the Blend
map within two float32 ulps of the oracle's double, the composite within
0.5/255 (uint8 equal away from rounding boundaries)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_01201_amd import synth

pytestmark = pytest.mark.gpu

F_TOL = 0.5 / 255.0
B_TOL = 1.2e-7


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_01201_amd import api as _api

    return _api


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pitched(a, extra):
    """A device view of `a` whose rows are `extra` elements longer."""
    H, W = a.shape[:2]
    big = np.zeros((H, W + extra) + a.shape[2:], a.dtype)
    big[:, :W] = a
    return dev(big)[:, :W]


def plan_for(api, H, W, **kw):
    return api.Plan(api.Params(**kw), max_strips=1, max_H=max(H, 8), max_W=max(W, 8), canvas=(H, W))


MASKS = {
    "blobs_23x41": lambda: synth.random_masks(1, 23, 41),
    "blobs_64x33": lambda: synth.random_masks(2, 64, 33),
    "row_1x57": lambda: synth.random_masks(4, 1, 57),
    "column_49x1": lambda: synth.random_masks(5, 49, 1),
    "blobs_130x97": lambda: synth.random_masks(6, 130, 97, blobs=9),
    "blobs_75x300": lambda: synth.random_masks(8, 75, 300, blobs=4),
    "sparse_200x70": lambda: synth.random_masks(9, 200, 70, blobs=2),
    "one_empty_60x50": lambda: synth.random_masks(10, 60, 50, p_empty=0.5),
    "pair_96x160": lambda: (lambda c: (c.mask_L, c.mask_R))(synth.make_canvas(3, 96, 160, holes=2)),
    "pair_axis1_150x90": lambda: (lambda c: (c.mask_L, c.mask_R))(synth.make_canvas(4, 150, 90, axis=1)),
}


def _single_pixels():
    mL = np.zeros((40, 37), np.uint8)
    mR = np.zeros((40, 37), np.uint8)
    mL[3, 5] = 1
    mR[35, 30] = 1
    mL[20:, 10:] = 1
    mR[20:, 10:] = 1
    return mL, mR


MASKS["single_pixels_40x37"] = _single_pixels
MASKS["identical_30x30"] = lambda: (np.ones((30, 30), np.uint8), np.ones((30, 30), np.uint8))


@pytest.mark.parametrize("name", list(MASKS))
def test_overlap_box_distances_and_blend(api, name):
    mL, mR = MASKS[name]()
    H, W = mL.shape
    plan = plan_for(api, H, W)
    print(f"[gpu] canvas distances {name}", flush=True)
    pad = 5 if H % 2 else 0  # odd heights use pitched masks
    dL, dR = (pitched(mL, pad), pitched(mR, pad)) if pad else (dev(mL), dev(mR))
    assert plan.overlap_box(dL, dR) == oracle.overlap_box(mL, mR)
    B, d1, d2 = plan.canvas_blend(dL, dR, distances=True)
    torch.cuda.synchronize()
    o1, o2 = oracle.canvas_dist2(mL, mR)
    assert np.array_equal(d1.cpu().numpy().astype(np.int64), o1)
    assert np.array_equal(d2.cpu().numpy().astype(np.int64), o2)
    oB = oracle.canvas_blend(mL, mR)
    assert np.abs(B.cpu().numpy().astype(np.float64) - oB).max() <= B_TOL
    # the Blend-only launch (no distances) searches only Area3 pixels
    B2 = plan.canvas_blend(dL, dR)
    torch.cuda.synchronize()
    assert torch.equal(B, B2)


def test_large_canvas_sampled(api):
    # 4000 x 2400 pair canvas (two side photos, 2 Area1 islands inside the
    # overlap): distances checked one by one at sampled pixels
    rng = synth.rng_for(113, 0, 0)
    mL, mR = synth.canvas_masks(rng, 4000, 2400, 0.3, holes=2)
    H, W = mL.shape
    plan = plan_for(api, H, W)
    print("[gpu] canvas distances 4000x2400 sampled", flush=True)
    dL, dR = dev(mL), dev(mR)
    assert plan.overlap_box(dL, dR) == oracle.overlap_box(mL, mR)
    B, d1, d2 = plan.canvas_blend(dL, dR, distances=True)
    torch.cuda.synchronize()
    a = (mL > 0) + 2 * (mR > 0)
    ys, xs = np.nonzero(a == 3)
    pick = rng.choice(len(xs), 300, replace=False)
    pts = np.concatenate([np.stack([xs[pick], ys[pick]], 1),
                          np.stack([rng.integers(0, W, 100), rng.integers(0, H, 100)], 1),
                          np.array([[0, 0], [W - 1, H - 1], [0, H - 1], [W - 1, 0]])])
    o1, o2 = oracle.canvas_dist2(mL, mR, pts)
    g1 = d1.cpu().numpy()[pts[:, 1], pts[:, 0]]
    g2 = d2.cpu().numpy()[pts[:, 1], pts[:, 0]]
    assert np.array_equal(g1.astype(np.int64), o1)
    assert np.array_equal(g2.astype(np.int64), o2)
    oB = oracle.canvas_blend(mL, mR, pts)
    assert np.abs(B.cpu().numpy()[pts[:, 1], pts[:, 0]].astype(np.float64) - oB).max() <= B_TOL
    # properties at every pixel: 0 inside the area, positive outside it
    h1, h2 = d1.cpu().numpy(), d2.cpu().numpy()
    assert (h1[a == 1] == 0).all() and (h1[a != 1] > 0).all()
    assert (h2[a == 2] == 0).all() and (h2[a != 2] > 0).all()


def test_large_canvas_full_rows_and_columns(api):
    # the same 4000 x 2400 canvas: every pixel of 8 full rows and 8 full
    # columns (51 200 points), through both Area1 islands inside the overlap
    # and across the overlap box, against the oracle's exact distances
    from scipy import ndimage

    rng = synth.rng_for(113, 0, 0)
    mL, mR = synth.canvas_masks(rng, 4000, 2400, 0.3, holes=2)
    H, W = mL.shape
    plan = plan_for(api, H, W)
    print("[gpu] canvas distances 4000x2400, 8 full rows and 8 full columns", flush=True)
    B, d1, d2 = plan.canvas_blend(dev(mL), dev(mR), distances=True)
    torch.cuda.synchronize()
    a = (mL > 0) + 2 * (mR > 0)
    lab, n = ndimage.label(a == 1)
    sizes = ndimage.sum(np.ones_like(lab), lab, range(1, n + 1))
    islands = [k + 1 for k in np.argsort(sizes)[:-1]]  # every component but the main Area1
    assert len(islands) >= 2
    cents = ndimage.center_of_mass(np.ones_like(lab), lab, islands[:2])
    bx, by, bw, bh = oracle.overlap_box(mL, mR)
    rows = [int(c[0]) for c in cents] + [by + 1, by + bh - 2] + [by + bh * k // 5 for k in range(1, 5)]
    cols = [int(c[1]) for c in cents] + [bx + 1, bx + bw - 2] + [bx + bw * k // 5 for k in range(1, 5)]
    pts = np.concatenate([np.stack([np.arange(W), np.full(W, r)], 1) for r in rows] +
                         [np.stack([np.full(H, c), np.arange(H)], 1) for c in cols])
    o1, o2 = oracle.canvas_dist2_rows(mL, mR, pts)
    g1 = d1.cpu().numpy()[pts[:, 1], pts[:, 0]].astype(np.int64)
    g2 = d2.cpu().numpy()[pts[:, 1], pts[:, 0]].astype(np.int64)
    assert np.array_equal(g1, o1)
    assert np.array_equal(g2, o2)
    # eq. (1) from the exact distances, at the Area3 points
    on3 = a[pts[:, 1], pts[:, 0]] == 3
    oB = np.sqrt(o1) / (np.sqrt(o1) + np.sqrt(o2))
    gB = B.cpu().numpy()[pts[:, 1], pts[:, 0]].astype(np.float64)
    assert np.abs(gB[on3] - oB[on3]).max() <= B_TOL
    print(f"canvas rows {rows} columns {cols}: {len(pts)} points, {int(on3.sum())} in Area3, all equal", flush=True)


def _check_F(F8, Ff, oF):
    assert np.abs(Ff - oF).max() <= F_TOL
    r = oF - np.floor(oF)
    safe = np.abs(r - 0.5) > F_TOL
    o8 = np.clip(np.floor(oF + 0.5), 0, 255).astype(np.uint8)
    assert np.array_equal(F8[safe], o8[safe])
    assert np.abs(F8.astype(int) - o8.astype(int)).max() <= 1


def _flows(seed, bh, bw, scale):
    r = synth.rng_for(114, seed, 0)
    return (r.uniform(-scale, scale, (bh, bw, 2)).astype(np.float32),
            r.uniform(-scale, scale, (bh, bw, 2)).astype(np.float32))


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("mode", ["eq1", "user", "linear"])
def test_composite_parity(api, axis, mode):
    c = synth.make_canvas(5 + axis, 90, 140, axis=axis, holes=1)
    H, W = c.mask_L.shape
    box = oracle.overlap_box(c.mask_L, c.mask_R)
    flr, frl = _flows(axis, box[3], box[2], 6.0)
    blend = synth.rng_for(115, axis, 0).uniform(0, 1, (H, W)).astype(np.float32) if mode == "user" else None
    kw = dict(blend_mode=1) if mode == "linear" else {}
    plan = plan_for(api, H, W, **kw)
    print(f"[gpu] composite axis {axis} {mode}", flush=True)
    F8, Ff = plan.composite_canvas(pitched(c.L, 7), dev(c.R), dev(c.mask_L), dev(c.mask_R), dev(flr), dev(frl), box,
                                   axis=axis, blend=None if blend is None else dev(blend), f32=True)
    torch.cuda.synchronize()
    op = oracle.Params(**kw)
    oF, _ = oracle.composite(c.L, c.R, c.mask_L, c.mask_R, flr, frl, box, axis=axis, blend=blend, params=op)
    _check_F(F8.cpu().numpy(), Ff.cpu().numpy(), oF)


def test_composite_box_smaller_than_area3_and_pitched_output(api):
    c = synth.make_canvas(7, 64, 100, holes=1)
    H, W = c.mask_L.shape
    bx, by, bw, bh = oracle.overlap_box(c.mask_L, c.mask_R)
    box = (bx + 2, by + 1, bw - 5, bh - 3)
    flr, frl = _flows(3, box[3], box[2], 3.0)
    plan = plan_for(api, H, W)
    print("[gpu] composite small box", flush=True)
    out = torch.zeros((H, W + 3, 3), dtype=torch.uint8, device="cuda")[:, 1:W + 1]
    F8, Ff = plan.composite_canvas(dev(c.L), dev(c.R), dev(c.mask_L), dev(c.mask_R), dev(flr), dev(frl), box,
                                   f32=True, out=out)
    torch.cuda.synchronize()
    oF, _ = oracle.composite(c.L, c.R, c.mask_L, c.mask_R, flr, frl, box)
    _check_F(F8.cpu().numpy(), Ff.cpu().numpy(), oF)
    full = out.cpu().numpy()
    assert F8.data_ptr() == out.data_ptr() and np.array_equal(full, F8.cpu().numpy())


def test_composite_without_overlap(api):
    # side by side without overlap: no flow, Area1 / Area2 copies and zeros
    H, W = 20, 30
    mL = np.zeros((H, W), np.uint8)
    mR = np.zeros((H, W), np.uint8)
    mL[:, :12] = 1
    mR[2:, 15:] = 1
    s = synth.make_random(9, H, W)
    plan = plan_for(api, H, W)
    print("[gpu] composite without overlap", flush=True)
    assert plan.overlap_box(dev(mL), dev(mR)) == (0, 0, 0, 0)
    F8 = plan.composite_canvas(dev(s.L), dev(s.R), dev(mL), dev(mR), None, None, (0, 0, 0, 0))
    torch.cuda.synchronize()
    oF, o8 = oracle.composite(s.L, s.R, mL, mR, np.zeros((0, 0, 2)), np.zeros((0, 0, 2)), (0, 0, 0, 0))
    assert np.array_equal(F8.cpu().numpy(), o8)


def test_stitch_canvas_end_to_end(api):
    # box -> both flows on the box crops -> eq. (1) -> Code 1. The flows
    # are checked against the oracle's; the composite against the oracle's
    # given the oracle's flows; and stitch_canvas against the GPU's own
    # composite of its own flows
    c = synth.make_canvas(8, 320, 400, holes=1)
    H, W = c.mask_L.shape
    plan = plan_for(api, H, W, levels=4)
    print("[gpu] stitch_canvas 320x400", flush=True)
    dL, dR, mL, mR = dev(c.L), dev(c.R), dev(c.mask_L), dev(c.mask_R)
    F8, Ff, box, flr, frl = plan.stitch_canvas(dL, dR, mL, mR, f32=True)
    torch.cuda.synchronize()
    obox = oracle.overlap_box(c.mask_L, c.mask_R)
    assert box == obox
    bx, by, bw, bh = obox
    of_lr, of_rl = oracle.flow_bidirectional(c.L[by:by + bh, bx:bx + bw], c.R[by:by + bh, bx:bx + bw],
                                             oracle.Params(levels=4))
    assert np.abs(flr.cpu().numpy() - of_lr).max() <= 1e-2
    assert np.abs(frl.cpu().numpy() - of_rl).max() <= 1e-2
    G8 = plan.composite_canvas(dL, dR, mL, mR, flr, frl, box)
    torch.cuda.synchronize()
    assert torch.equal(F8, G8)
    f_lr, f_rl = of_lr.astype(np.float32), of_rl.astype(np.float32)
    O8, Of = plan.composite_canvas(dL, dR, mL, mR, dev(f_lr), dev(f_rl), obox, f32=True)
    torch.cuda.synchronize()
    oF, _ = oracle.composite(c.L, c.R, c.mask_L, c.mask_R, f_lr, f_rl, obox)
    _check_F(O8.cpu().numpy(), Of.cpu().numpy(), oF)


def test_canvas_limits_are_enforced(api):
    plan = api.Plan(api.Params(), max_strips=1, max_H=64, max_W=64)
    m = torch.ones((4000, 3000), dtype=torch.uint8, device="cuda")
    with pytest.raises(Exception, match="workspace"):
        plan.canvas_blend(m, m)
    small = plan_for(api, 16, 16)
    m = torch.ones((16, 16), dtype=torch.uint8, device="cuda")
    img = torch.zeros((16, 16, 3), dtype=torch.uint8, device="cuda")
    f = torch.zeros((16, 16, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        small.composite_canvas(img, img, m, m, f, f, (1, 0, 16, 16))
    # sides beyond 32767 (row distances are uint16) are refused
    wide = torch.ones((1, 32768), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        small.overlap_box(wide, wide)
    with pytest.raises(ValueError):
        small.canvas_blend(wide, wide)


def test_distances_are_bitwise_repeatable(api):
    mL, mR = synth.random_masks(12, 300, 500, blobs=8)
    plan = plan_for(api, 300, 500)
    print("[gpu] canvas distances twice", flush=True)
    a = [t.clone() for t in plan.canvas_blend(dev(mL), dev(mR), distances=True)]
    b = plan.canvas_blend(dev(mL), dev(mR), distances=True)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))


# ----------------------------------------------------------------------------
# Periodic canvas (360-degree panorama: column W - 1 next to column 0)


def _wrapped_masks(seed, H, W):
    # random blobs rolled so that shapes cross the wrap, plus column clusters
    # of Area3 at both ends (the box wraps)
    mL, mR = synth.random_masks(seed, H, W, blobs=5)
    s = W // 3 + seed
    mL, mR = np.roll(mL, s, 1), np.roll(mR, s, 1)
    mL[H // 4:H // 2, :4] = 1
    mR[H // 4:H // 2, :4] = 1
    mL[H // 3:, W - 5:] = 1
    mR[H // 3:, W - 5:] = 1
    return mL, mR


PERIODIC = {
    "wrapped_40x71": lambda: _wrapped_masks(31, 40, 71),
    "wrapped_97x130": lambda: _wrapped_masks(32, 97, 130),
    "wrapped_1x90": lambda: _wrapped_masks(33, 1, 90),
    "blobs_64x33": lambda: synth.random_masks(2, 64, 33),
    "identical_30x30": lambda: (np.ones((30, 30), np.uint8), np.ones((30, 30), np.uint8)),
    "ring_seam_90x360": lambda: (lambda ph: (ph[0][1] | ph[1][1], ph[2][1]))(
        synth.make_panorama_photos(4, 90, 360, n_ring=3, closed=True)),
}


@pytest.mark.parametrize("name", list(PERIODIC))
def test_periodic_box_distances_and_blend(api, name):
    mL, mR = PERIODIC[name]()
    H, W = mL.shape
    plan = plan_for(api, H, W)
    print(f"[gpu] periodic canvas distances {name}", flush=True)
    dL, dR = dev(mL), dev(mR)
    assert plan.overlap_box(dL, dR, periodic=True) == oracle.overlap_box(mL, mR, periodic=True)
    B, d1, d2 = plan.canvas_blend(dL, dR, distances=True, periodic=True)
    torch.cuda.synchronize()
    o1, o2 = oracle.canvas_dist2(mL, mR, periodic=True)
    assert np.array_equal(d1.cpu().numpy().astype(np.int64), o1)
    assert np.array_equal(d2.cpu().numpy().astype(np.int64), o2)
    oB = oracle.canvas_blend(mL, mR, periodic=True)
    assert np.abs(B.cpu().numpy().astype(np.float64) - oB).max() <= B_TOL
    B2 = plan.canvas_blend(dL, dR, periodic=True)
    torch.cuda.synchronize()
    assert torch.equal(B, B2)


@pytest.mark.parametrize("seed", range(6))
def test_periodic_box_of_column_clusters(api, seed):
    # one to three column clusters of Area3, often across the wrap, on
    # canvases whose widths are not multiples of the occupancy words
    rng = np.random.default_rng(40 + seed)
    H, W = 13, [37, 64, 100, 161, 33, 250][seed]
    mL = np.zeros((H, W), np.uint8)
    mR = np.zeros((H, W), np.uint8)
    for _ in range(int(rng.integers(1, 4))):
        c0, n = int(rng.integers(0, W)), int(rng.integers(1, 12))
        cols = (c0 + np.arange(n)) % W
        r0 = int(rng.integers(0, H - 3))
        mL[r0:r0 + 3, cols] = 1
        mR[r0:r0 + 3, cols] = 1
    plan = plan_for(api, H, W)
    print(f"[gpu] periodic box clusters {seed}", flush=True)
    assert plan.overlap_box(dev(mL), dev(mR), periodic=True) == oracle.overlap_box(mL, mR, periodic=True)
    assert plan.overlap_box(dev(mL), dev(mR)) == oracle.overlap_box(mL, mR)


@pytest.mark.parametrize("mode", ["eq1", "user"])
def test_periodic_composite_with_a_wrapped_box(api, mode):
    # the last photo of a closed ring against the photos before it: Area3 at
    # its left seam and across the wrap, one box over the wrap
    H, W = 90, 360
    ph = synth.make_panorama_photos(4, H, W, n_ring=3, closed=True)
    mL = ph[0][1] | ph[1][1]
    mR = ph[2][1]
    L = np.where(ph[1][1][..., None] > 0, ph[1][0], ph[0][0])
    R = ph[2][0]
    box = oracle.overlap_box(mL, mR, periodic=True)
    bx, by, bw, bh = box
    assert bx + bw > W  # the box wraps
    flr, frl = _flows(9, bh, bw, 5.0)
    blend = synth.rng_for(116, 0, 0).uniform(0, 1, (H, W)).astype(np.float32) if mode == "user" else None
    plan = plan_for(api, H, W)
    print(f"[gpu] periodic composite {mode}", flush=True)
    F8, Ff = plan.composite_canvas(dev(L), dev(R), dev(mL), dev(mR), dev(flr), dev(frl), box,
                                   blend=None if blend is None else dev(blend), f32=True, periodic=True)
    torch.cuda.synchronize()
    oF, _ = oracle.composite(L, R, mL, mR, flr, frl, box, blend=blend, periodic=True)
    _check_F(F8.cpu().numpy(), Ff.cpu().numpy(), oF)
