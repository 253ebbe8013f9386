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
