"""Pins of the oracle's canvas functions (eq. (1) with coverage masks of any
shape, Code 1's Area1 / Area2 / else branches), against what the
mathematics fixes: scipy's exact Euclidean distance transform, the
closed-form ramp of a rectangular overlap, swap and transpose symmetries,
the empty-area limits, and the strip blend on a rectangular overlap."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2006_01201_amd import synth


def areas(mL, mR):
    return (mL > 0).astype(int) + 2 * (mR > 0).astype(int)


@pytest.mark.parametrize("seed,H,W", [(1, 23, 41), (2, 64, 33), (3, 17, 90), (4, 1, 57), (5, 49, 1)])
def test_dist2_equals_scipy_edt(seed, H, W):
    mL, mR = synth.random_masks(seed, H, W)
    a = areas(mL, mR)
    d1, d2 = oracle.canvas_dist2(mL, mR)
    for k, d in ((1, d1), (2, d2)):
        if not (a == k).any():
            assert (d == -1).all()
            continue
        # distance_transform_edt: distance of every nonzero element to the
        # nearest zero element, so the zeros are the pixels of area k
        e = ndimage.distance_transform_edt(a != k)
        assert np.array_equal(d, np.rint(e * e).astype(np.int64))


@pytest.mark.parametrize("seed,H,W", [(1, 23, 41), (3, 17, 90), (4, 1, 57), (5, 49, 1), (11, 120, 77),
                                      (12, 60, 50)])
def test_two_stage_dist2_equals_scipy_edt_and_brute_force(seed, H, W):
    mL, mR = synth.random_masks(seed, H, W, p_empty=0.3 if seed == 12 else 0.0)
    a = areas(mL, mR)
    r1, r2 = oracle.canvas_dist2_rows(mL, mR)
    b1, b2 = oracle.canvas_dist2(mL, mR)
    assert np.array_equal(r1, b1) and np.array_equal(r2, b2)
    for k, d in ((1, r1), (2, r2)):
        if (a == k).any():
            e = ndimage.distance_transform_edt(a != k)
            assert np.array_equal(d, np.rint(e * e).astype(np.int64))
        else:
            assert (d == -1).all()
    pts = np.array([[0, 0], [W - 1, H - 1], [W // 2, H // 3]])
    p1, p2 = oracle.canvas_dist2_rows(mL, mR, pts)
    assert np.array_equal(p1, b1[pts[:, 1], pts[:, 0]]) and np.array_equal(p2, b2[pts[:, 1], pts[:, 0]])


def test_dist2_points_equal_full_canvas():
    mL, mR = synth.random_masks(7, 30, 45)
    d1, d2 = oracle.canvas_dist2(mL, mR)
    pts = np.array([[0, 0], [44, 29], [13, 7], [44, 0], [0, 29], [21, 15]])
    p1, p2 = oracle.canvas_dist2(mL, mR, pts)
    assert np.array_equal(p1, d1[pts[:, 1], pts[:, 0]])
    assert np.array_equal(p2, d2[pts[:, 1], pts[:, 0]])


@pytest.mark.parametrize("H,W,b,a", [(9, 20, 6, 15), (1, 12, 1, 11), (5, 8, 3, 4)])
def test_rectangular_overlap_gives_the_strip_ramp(H, W, b, a):
    # L covers columns [0, a), R covers [b, W): Area3 = [b, a) is a strip of
    # width a - b whose Blend is (x' + 1) / (width + 1), x' = x - b
    mL = np.zeros((H, W), np.uint8)
    mR = np.zeros((H, W), np.uint8)
    mL[:, :a] = 1
    mR[:, b:] = 1
    B = oracle.canvas_blend(mL, mR)
    xs = np.arange(W)
    want = np.where(xs < b, 0.0, np.where(xs >= a, 1.0, (xs - b + 1) / (a - b + 1)))
    assert np.allclose(B, want[None, :], rtol=0, atol=1e-15)
    if a > b:
        strip = oracle.blend_coef(H, a - b, 0)
        assert np.allclose(B[:, b:a], strip, rtol=0, atol=1e-15)
    # the same layout turned by 90 degrees ramps along y (axis 1)
    BT = oracle.canvas_blend(mL.T.copy(), mR.T.copy())
    assert np.allclose(BT, want[:, None].repeat(H, 1), rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_swap_and_transpose_symmetry(seed):
    mL, mR = synth.random_masks(seed, 26, 37)
    B = oracle.canvas_blend(mL, mR)
    S = oracle.canvas_blend(mR, mL)
    assert np.allclose(S, 1.0 - B, rtol=0, atol=1e-15)
    T = oracle.canvas_blend(mL.T.copy(), mR.T.copy())
    assert np.array_equal(T, B.T)
    a = areas(mL, mR)
    assert (B[a == 1] == 0).all() and (B[a == 2] == 1).all() and (B[a == 0] == 0.5).all()
    inner = B[a == 3]
    assert ((inner > 0) & (inner < 1)).all()


def test_empty_areas_take_the_limits():
    H, W = 7, 9
    full = np.ones((H, W), np.uint8)
    half = np.zeros((H, W), np.uint8)
    half[:, :5] = 1
    # Area1 empty (L inside R): Lmin is infinite, Blend -> 1
    B = oracle.canvas_blend(half, full)
    assert (B[:, :5] == 1.0).all() and (B[:, 5:] == 1.0).all()
    # Area2 empty: Blend -> 0 on Area3
    B = oracle.canvas_blend(full, half)
    assert (B[:, :5] == 0.0).all() and (B[:, 5:] == 0.0).all()
    # both empty (identical coverage): 0.5 on Area3 and outside
    B = oracle.canvas_blend(half, half)
    assert (B == 0.5).all()
    d1, d2 = oracle.canvas_dist2(half, half)
    assert (d1 == -1).all() and (d2 == -1).all()


def test_overlap_box():
    c = synth.make_canvas(1, 60, 90, holes=1)
    ys, xs = np.nonzero((c.mask_L > 0) & (c.mask_R > 0))
    want = (xs.min(), ys.min(), xs.max() - xs.min() + 1, ys.max() - ys.min() + 1)
    assert oracle.overlap_box(c.mask_L, c.mask_R) == tuple(int(v) for v in want)
    z = np.zeros((4, 5), np.uint8)
    assert oracle.overlap_box(z, z + 1) == (0, 0, 0, 0)


def _flows(seed, bh, bw, scale=4.0):
    r = synth.rng_for(112, seed, 0)
    return (r.uniform(-scale, scale, (bh, bw, 2)), r.uniform(-scale, scale, (bh, bw, 2)))


@pytest.mark.parametrize("axis", [0, 1])
def test_composite_branches(axis):
    c = synth.make_canvas(4, 48, 70, axis=axis, holes=1)
    box = oracle.overlap_box(c.mask_L, c.mask_R)
    flr, frl = _flows(1, box[3], box[2])
    F, F8 = oracle.composite(c.L, c.R, c.mask_L, c.mask_R, flr, frl, box, axis=axis)
    a = areas(c.mask_L, c.mask_R)
    assert np.array_equal(F8[a == 1], c.L[a == 1])
    assert np.array_equal(F8[a == 2], c.R[a == 2])
    assert (F8[a == 0] == 0).all()
    # an Area3 pixel that the box does not cover has no flow: 0
    small = (box[0] + 1, box[1] + 1, box[2] - 2, box[3] - 2)
    _, G8 = oracle.composite(c.L, c.R, c.mask_L, c.mask_R, flr[1:-1, 1:-1], frl[1:-1, 1:-1], small, axis=axis)
    x, y = np.meshgrid(np.arange(c.L.shape[1]), np.arange(c.L.shape[0]))
    outside = (a == 3) & ((x < small[0]) | (x >= small[0] + small[2]) | (y < small[1]) | (y >= small[1] + small[3]))
    assert outside.any() and (G8[outside] == 0).all()


@pytest.mark.parametrize("axis", [0, 1])
def test_composite_rectangular_overlap_equals_the_strip_blend(axis):
    # a full-height (full-width for axis 1) rectangular overlap: Area3 is the
    # box, eq. (1) is the strip ramp, and Code 1 on it is the strip blend
    H, W, b, a = 20, 50, 18, 37
    mL = np.zeros((H, W), np.uint8)
    mR = np.zeros((H, W), np.uint8)
    mL[:, :a] = 1
    mR[:, b:] = 1
    s = synth.make_random(5, H, W)
    L, R = s.L, s.R
    if axis == 1:
        mL, mR, L, R = mL.T.copy(), mR.T.copy(), L.transpose(1, 0, 2).copy(), R.transpose(1, 0, 2).copy()
    box = oracle.overlap_box(mL, mR)
    bx, by, bw, bh = box
    flr, frl = _flows(2, bh, bw)
    F, F8 = oracle.composite(L, R, mL, mR, flr, frl, box, axis=axis)
    sF, sF8 = oracle.blend(L[by:by + bh, bx:bx + bw], R[by:by + bh, bx:bx + bw], flr, frl, axis=axis)
    assert np.allclose(F[by:by + bh, bx:bx + bw], sF, rtol=0, atol=1e-12)
    assert np.array_equal(F8[by:by + bh, bx:bx + bw], sF8)
    # an explicit Blend map equal to eq. (1) gives the same composite
    G, G8 = oracle.composite(L, R, mL, mR, flr, frl, box, axis=axis, blend=oracle.canvas_blend(mL, mR))
    assert np.array_equal(G8, F8) and np.allclose(G, F, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------
# Periodic canvas (a 360-degree panorama: column W - 1 neighbours column 0)


@pytest.mark.parametrize("seed,H,W", [(21, 23, 41), (22, 40, 64), (23, 1, 57), (24, 33, 2), (25, 17, 90)])
def test_periodic_dist2_equals_scipy_edt_on_three_tiles(seed, H, W):
    # the periodic distance of a pixel is its plain distance in the middle
    # copy of the canvas tiled three times along x (no nearest pixel is more
    # than half a period away, so one copy on each side suffices)
    mL, mR = synth.random_masks(seed, H, W)
    a = areas(mL, mR)
    d1, d2 = oracle.canvas_dist2(mL, mR, periodic=True)
    r1, r2 = oracle.canvas_dist2_rows(mL, mR, periodic=True)
    assert np.array_equal(r1, d1) and np.array_equal(r2, d2)
    a3 = np.tile(a, (1, 3))
    for k, d in ((1, d1), (2, d2)):
        if not (a == k).any():
            assert (d == -1).all()
            continue
        e = ndimage.distance_transform_edt(a3 != k)[:, W:2 * W]
        assert np.array_equal(d, np.rint(e * e).astype(np.int64))
    # never farther than the plain distance
    p1, p2 = oracle.canvas_dist2(mL, mR)
    assert ((d1 <= p1) | (p1 < 0)).all() and ((d2 <= p2) | (p2 < 0)).all()


@pytest.mark.parametrize("shift", [1, 17, 40])
def test_periodic_blend_commutes_with_rolling(shift):
    H, W = 30, 53
    mL, mR = synth.random_masks(26, H, W)
    B = oracle.canvas_blend(mL, mR, periodic=True)
    Br = oracle.canvas_blend(np.roll(mL, shift, 1), np.roll(mR, shift, 1), periodic=True)
    assert np.array_equal(Br, np.roll(B, shift, 1))


def _brute_circular_box(occ):
    # the shortest run [x, x + w) (mod W) of columns holding every occupied
    # column, by trying every start; of equally short runs, the one whose
    # complementary empty run starts at the smallest column
    W = occ.size
    cols = np.flatnonzero(occ)
    best = None
    for x in range(W):
        w = int(((cols - x) % W).max()) + 1
        key = (w, (x + w) % W)
        if best is None or key < best[0]:
            best = (key, x, w)
    return (0, W) if best[2] == W else (best[1], best[2])


def test_periodic_box_tie_takes_the_first_empty_run():
    # occupied columns 0 and 10 of 20: two empty runs of 9 columns, starting
    # at 1 and at 11; the first is skipped, so the box runs from 10 over the
    # wrap to 0
    mL = np.zeros((3, 20), np.uint8)
    mL[1, [0, 10]] = 1
    assert oracle.overlap_box(mL, mL, periodic=True) == (10, 1, 11, 1)
    assert _brute_circular_box(mL.any(0)) == (10, 11)


@pytest.mark.parametrize("seed", range(8))
def test_periodic_box_is_the_shortest_circular_cover(seed):
    rng = np.random.default_rng(seed)
    H, W = 11, 37
    mL = np.zeros((H, W), np.uint8)
    mR = np.zeros((H, W), np.uint8)
    occ = np.zeros(W, bool)
    # two or three column clusters, one of them often across the wrap
    for _ in range(int(rng.integers(1, 4))):
        c0, n = int(rng.integers(0, W)), int(rng.integers(1, 9))
        cols = (c0 + np.arange(n)) % W
        r0 = int(rng.integers(0, H - 2))
        mL[r0:r0 + 3, cols] = 1
        mR[r0:r0 + 3, cols] = 1
        occ[cols] = True
    mL[:, :5] = 1  # Area1 elsewhere
    x, y, w, h = oracle.overlap_box(mL, mR, periodic=True)
    bx, bw = _brute_circular_box(occ)
    assert (x, w) == (bx, bw)
    rows = np.flatnonzero(((mL > 0) & (mR > 0)).any(1))
    assert (y, h) == (rows[0], rows[-1] - rows[0] + 1)
    # every Area3 pixel lies in the box, read modulo W
    ys, xs = np.nonzero((mL > 0) & (mR > 0))
    assert (((xs - x) % W) < w).all()


def test_periodic_box_of_contiguous_columns_is_the_plain_box():
    mL, mR = synth.random_masks(27, 25, 60)
    mL[:, 50:] = 0
    mR[:, :10] = 0
    assert oracle.overlap_box(mL, mR, periodic=True) == oracle.overlap_box(mL, mR)
    full = np.ones((4, 9), np.uint8)
    assert oracle.overlap_box(full, full, periodic=True) == (0, 0, 9, 4)


@pytest.mark.parametrize("shift", [9, 31])
def test_periodic_composite_commutes_with_rolling(shift):
    # Code 1 on a periodic canvas depends on columns only through their
    # circular order: rolling every input (and the box) rolls the output,
    # including a box that the roll makes wrap past column W - 1
    H, W = 24, 48
    rng = np.random.default_rng(28)
    mL = np.zeros((H, W), np.uint8)
    mR = np.zeros((H, W), np.uint8)
    mL[:, :30] = 1
    mR[:, 18:] = 1
    mR[5:9, 22:26] = 0  # an Area1 island inside the overlap
    L = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    R = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    box = oracle.overlap_box(mL, mR, periodic=True)
    bx, by, bw, bh = box
    flr = rng.uniform(-3, 3, (bh, bw, 2))
    frl = rng.uniform(-3, 3, (bh, bw, 2))
    F, F8 = oracle.composite(L, R, mL, mR, flr, frl, box, periodic=True)
    rb = oracle.overlap_box(np.roll(mL, shift, 1), np.roll(mR, shift, 1), periodic=True)
    assert rb == ((bx + shift) % W, by, bw, bh)
    Fr, F8r = oracle.composite(np.roll(L, shift, 1), np.roll(R, shift, 1), np.roll(mL, shift, 1),
                               np.roll(mR, shift, 1), flr, frl, rb, periodic=True)
    assert np.array_equal(Fr, np.roll(F, shift, 1)) and np.array_equal(F8r, np.roll(F8, shift, 1))
    # the box's Area3 part is the strip blend of the box crops (read modulo W)
    cols = (rb[0] + np.arange(bw)) % W
    Lc = np.roll(L, shift, 1)[by:by + bh][:, cols]
    Rc = np.roll(R, shift, 1)[by:by + bh][:, cols]
    Bc = oracle.canvas_blend(np.roll(mL, shift, 1), np.roll(mR, shift, 1), periodic=True)[by:by + bh][:, cols]
    Fs, _ = oracle.blend(Lc, Rc, flr, frl, blend=Bc, axis=0)
    a3 = ((np.roll(mL, shift, 1) > 0) & (np.roll(mR, shift, 1) > 0))[by:by + bh][:, cols]
    assert np.array_equal(Fr[by:by + bh][:, cols][a3], Fs[a3])
