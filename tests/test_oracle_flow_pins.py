"""Pins of the CPU oracle's flow stages against facts fixed outside it:
textbook definitions computed by library routines, brute force on tiny
inputs, closed forms and invariants (flow: Section III.C.1 of the paper).
"""
import numpy as np
import pytest
from scipy import ndimage

from paper_2006_01201_amd import synth


# ---------------------------------------------------------------- luma
def test_luma_gray_is_identity(orc):
    v = np.arange(256, dtype=np.uint8)
    rgb = np.stack([v, v, v], axis=-1)[None]
    assert np.array_equal(orc.luma(rgb)[0], v)


def test_luma_close_to_bt601(orc):
    rgb = synth.random_bytes(1, (64, 64, 3))
    y = orc.luma(rgb).astype(np.float64)
    ref = 0.299 * rgb[..., 0] + 0.587 * rgb[..., 1] + 0.114 * rgb[..., 2]
    assert np.abs(y - ref).max() < 1.5


def test_luma_channel_order(orc):
    # pure red and pure blue differ by the BT.601 weights (0.299 vs 0.114)
    red = np.zeros((1, 1, 3), np.uint8)
    red[..., 0] = 255
    blue = np.zeros((1, 1, 3), np.uint8)
    blue[..., 2] = 255
    assert abs(int(orc.luma(red)[0, 0]) - 0.299 * 255) < 1.5
    assert abs(int(orc.luma(blue)[0, 0]) - 0.114 * 255) < 1.5


# ------------------------------------------------------------- pyramid
@pytest.mark.parametrize("shape", [(16, 16), (17, 23), (5, 7), (1, 9), (64, 3)])
def test_pyr_down_equals_textbook_convolution(orc, shape):
    Y = synth.random_bytes(7, shape)
    k1 = np.array([1, 4, 6, 4, 1], np.int64)
    s = ndimage.convolve(Y.astype(np.int64), np.outer(k1, k1), mode="nearest")
    expect = ((s[::2, ::2] + 128) >> 8).astype(np.uint8)
    got = orc.pyr_down(Y)
    assert got.shape == ((shape[0] + 1) // 2, (shape[1] + 1) // 2)
    assert np.array_equal(got, expect)


def test_pyramid_of_constant_is_constant(orc):
    for v in (0, 1, 127, 255):
        levels = orc.pyramid(np.full((37, 50), v, np.uint8), 5)
        for lv in levels:
            assert (lv == v).all()
    assert [lv.shape for lv in levels] == [(37, 50), (19, 25), (10, 13), (5, 7), (3, 4)]


def test_level_sizes_ceil(orc):
    assert orc.level_sizes(4000, 768, 6) == [(4000, 768), (2000, 384), (1000, 192), (500, 96), (250, 48), (125, 24)]
    assert orc.level_sizes(600, 9000, 6)[-1] == (19, 282)


# ---------------------------------------------------------- upsample
def test_upsample_nearest_doubled(orc):
    Dc = synth.rng_for(103, 0, 0).integers(-9, 10, size=(5, 7, 2)).astype(np.int32)
    for H, W in [(10, 14), (9, 13)]:
        expect = np.repeat(np.repeat(2 * Dc, 2, axis=0), 2, axis=1)[:H, :W]
        assert np.array_equal(orc.upsample(Dc, H, W), expect)


# ------------------------------------------------------------ search
def brute_search(ref, tgt, centre, P, R):
    """Exhaustive search by a different route: clamped gathers for every
    candidate, cost volume, then a lexicographic sort of the key."""
    H, W = ref.shape
    yy, xx = np.mgrid[0:H, 0:W]
    cands = [(i, j) for j in range(-R, R + 1) for i in range(-R, R + 1)]
    costs = np.zeros((len(cands), H, W), np.int64)
    for n, (i, j) in enumerate(cands):
        dx = centre[..., 0] + i
        dy = centre[..., 1] + j
        for b in range(-P, P + 1):
            for a in range(-P, P + 1):
                r = ref[np.clip(yy + b, 0, H - 1), np.clip(xx + a, 0, W - 1)].astype(np.int64)
                t = tgt[np.clip(yy + b + dy, 0, H - 1), np.clip(xx + a + dx, 0, W - 1)].astype(np.int64)
                costs[n] += np.abs(r - t)
    l1 = np.array([abs(i) + abs(j) for i, j in cands])
    key = costs * 10000 + l1[:, None, None] * 100 + np.arange(len(cands))[:, None, None]
    best = np.argmin(key, axis=0)
    off = np.array(cands)[best]
    return np.stack([centre[..., 0] + off[..., 0], centre[..., 1] + off[..., 1]], -1), costs.min(axis=0)


@pytest.mark.parametrize("seed,levels,R,P", [(0, 256, 3, 2), (1, 3, 2, 2), (2, 2, 3, 1), (3, 5, 1, 2), (4, 256, 4, 2)])
def test_search_equals_brute_force(orc, seed, levels, R, P):
    shape = (12, 16)
    ref = synth.random_levels(seed, shape, levels)
    tgt = synth.random_levels(seed + 50, shape, levels)
    centre = synth.rng_for(104, seed, 0).integers(-3, 4, size=shape + (2,)).astype(np.int32)
    for c in (np.zeros_like(centre), centre):
        D, cost = orc.search(ref, tgt, c, P=P, R=R)
        Db, cb = brute_search(ref, tgt, c, P, R)
        assert np.array_equal(D, Db)
        assert np.array_equal(cost, cb)


def test_search_ties_prefer_centre_then_l1(orc):
    # constant images: every candidate costs 0, so the centre must win
    z = np.full((9, 11), 100, np.uint8)
    c = np.zeros((9, 11, 2), np.int32)
    c[..., 0] = 3
    c[..., 1] = -2
    D, cost = orc.search(z, z, c, P=2, R=2)
    assert (cost == 0).all() and np.array_equal(D, c)


# ------------------------------------------------------- propagation
def brute_propagate_step(ref, tgt, D, P, allowed=None):
    # allowed: optional (5, H, W) mask of the candidates (own, left, right,
    # up, down) a pixel may take
    H, W = ref.shape
    yy, xx = np.mgrid[0:H, 0:W]
    nbs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    big = np.iinfo(np.int64).max
    costs = np.full((5, H, W), big, np.int64)
    vecs = np.zeros((5, H, W, 2), np.int64)
    for k, (ox, oy) in enumerate(nbs):
        qx, qy = xx + ox, yy + oy
        ok = (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
        if allowed is not None:
            ok &= allowed[k]
        d = D[np.clip(qy, 0, H - 1), np.clip(qx, 0, W - 1)].astype(np.int64)
        c = np.zeros((H, W), np.int64)
        for b in range(-P, P + 1):
            for a in range(-P, P + 1):
                r = ref[np.clip(yy + b, 0, H - 1), np.clip(xx + a, 0, W - 1)].astype(np.int64)
                t = tgt[np.clip(yy + b + d[..., 1], 0, H - 1), np.clip(xx + a + d[..., 0], 0, W - 1)]
                c += np.abs(r - t.astype(np.int64))
        costs[k] = np.where(ok, c, big)
        vecs[k] = d
    best = np.argmin(costs, axis=0)  # first minimum = earlier candidate
    return np.take_along_axis(vecs, best[None, ..., None], axis=0)[0]


@pytest.mark.parametrize("seed,T", [(0, 1), (1, 2), (2, 3)])
def test_propagate_equals_brute_force(orc, seed, T):
    shape = (10, 13)
    ref = synth.random_levels(seed, shape, 4)
    tgt = synth.random_levels(seed + 9, shape, 4)
    D = synth.rng_for(105, seed, 0).integers(-3, 4, size=shape + (2,)).astype(np.int32)
    expect = D.astype(np.int64)
    for _ in range(T):
        expect = brute_propagate_step(ref, tgt, expect, 2)
    assert np.array_equal(orc.propagate(ref, tgt, D, P=2, T=T), expect)


def test_propagate_never_increases_cost(orc):
    s = synth.make_random(3, 48, 40, max_ux=5, max_uy=2)
    yr, yl = orc.luma(s.R), orc.luma(s.L)
    D = synth.rng_for(106, 0, 0).integers(-6, 7, size=(48, 40, 2)).astype(np.int32)
    D2 = orc.propagate(yr, yl, D, P=2, T=1)

    def cost(Dv):
        c = np.zeros((48, 40), np.int64)
        _, c0 = orc.search(yr, yl, Dv, P=2, R=0)
        return c0

    assert (cost(D2) <= cost(D)).all()


@pytest.mark.parametrize("seed,levels,shape", [(0, 3, (11, 15)), (1, 256, (12, 17)), (2, 6, (9, 9)), (3, 2, (13, 10))])
def test_first_step_needs_only_neighbours_across_the_coarse_cell(orc, seed, levels, shape):
    # After the search around the upsampled coarser flow, a neighbour in the
    # pixel's own 2 x 2 cell has the pixel's search window, and the search
    # took the minimum over it, so the first propagation step is unchanged
    # when each pixel weighs only the neighbour across each edge of its cell:
    # left at even x, right at odd x, up at even y, down at odd y. Odd sizes
    # leave a last coarse row / column that covers one fine row / column.
    H, W = shape
    ref = synth.random_levels(seed + 20, shape, levels)
    tgt = synth.random_levels(seed + 70, shape, levels)
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    Dc = synth.rng_for(107, seed, 0).integers(-2, 3, size=(Hc, Wc, 2)).astype(np.int32)
    D, _ = orc.search(ref, tgt, orc.upsample(Dc, H, W), P=2, R=2)
    yy, xx = np.mgrid[0:H, 0:W]
    allowed = np.stack([np.ones((H, W), bool), xx % 2 == 0, xx % 2 == 1, yy % 2 == 0, yy % 2 == 1])
    full = brute_propagate_step(ref, tgt, D, 2)
    assert np.array_equal(brute_propagate_step(ref, tgt, D, 2, allowed), full)
    assert np.array_equal(orc.propagate(ref, tgt, D, P=2, T=1), full)
    # and some pixels do change in the step, so the restriction is exercised
    assert (full != D).any()


# ------------------------------------------------------------ median
@pytest.mark.parametrize("shape", [(9, 9), (1, 5), (7, 2), (16, 31)])
def test_median_equals_library(orc, shape):
    D = synth.rng_for(107, shape[0], shape[1]).integers(-50, 50, size=shape + (2,)).astype(np.int32)
    got = orc.median(D, M=1)
    for comp in range(2):
        expect = ndimage.median_filter(D[..., comp], size=3, mode="nearest")
        assert np.array_equal(got[..., comp], expect)


# ------------------------------------------------------- whole chain
def test_identical_inputs_give_zero_flow(orc):
    s = synth.make_random(5, 96, 64)
    p = orc.Params(levels=4)
    flr, frl, lv = orc.flow_bidirectional(s.L, s.L, p, levels_out=True)
    assert (flr == 0).all() and (frl == 0).all()
    for name in lv:
        for d in lv[name]:
            assert (d == 0).all()


def _shifted_pair(seed, H, W, sx, sy, pad=24):
    tex = synth.Texture(synth.rng_for(108, seed, 0), H + 2 * pad, W + 2 * pad)
    yy, xx = np.mgrid[0:H + 2 * pad, 0:W + 2 * pad].astype(np.float64)
    big = np.clip(np.rint(tex(xx, yy)), 0, 255).astype(np.uint8)
    L = big[pad:pad + H, pad:pad + W]
    R = big[pad + sy:pad + sy + H, pad + sx:pad + sx + W]  # R(p) = L(p + s)
    return np.ascontiguousarray(L), np.ascontiguousarray(R)


@pytest.mark.parametrize("s", [(3, 0), (-5, 2), (7, -1)])
def test_integer_shift_is_recovered_exactly(orc, s):
    H, W = 96, 128
    L, R = _shifted_pair(11, H, W, *s)
    # the exposure step would rescale R (its border content differs from L's)
    p = orc.Params(levels=3, gain_comp=0)
    flr, frl, lv = orc.flow_bidirectional(L, R, p, levels_out=True)
    m = max(abs(s[0]), abs(s[1])) + p.patch + p.prop_steps + p.median + 2
    inner = (slice(m, H - m), slice(m, W - m))
    # R(p) = L(p + s): FlowRtoL = s and FlowLtoR = -s, integer and refined
    assert (lv["final_rl"][0][inner] == np.array(s)).all()
    assert (lv["final_lr"][0][inner] == -np.array(s)).all()
    assert (frl[inner] == np.array(s, float)).all()
    assert (flr[inner] == -np.array(s, float)).all()


def test_bidirectional_consistency_on_smooth_field(orc):
    st = synth.make_config_strip(0, 0, 0)
    p = orc.Params(levels=3)
    flr, frl = orc.flow_bidirectional(st.L, st.R, p)
    H, W = st.H, st.W
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    # FlowLtoR(q) + FlowRtoL(q + FlowLtoR(q)) ~ 0
    back_x = synth.bilinear_field(frl[..., 0], xx + flr[..., 0], yy + flr[..., 1])
    back_y = synth.bilinear_field(frl[..., 1], xx + flr[..., 0], yy + flr[..., 1])
    err = np.hypot(flr[..., 0] + back_x, flr[..., 1] + back_y)
    m = 10
    inner = err[m:H - m, m:W - m]
    assert (inner <= 0.5).mean() >= 0.95


def test_flow_accuracy_against_ground_truth(orc):
    st = synth.make_config_strip(0, 0, 0)
    flr, frl = orc.flow_bidirectional(st.L, st.R, orc.Params(levels=3))
    m = 8
    sl = (slice(m, -m), slice(m, -m))
    epe = np.hypot(*(frl - st.flow_rl_gt).transpose(2, 0, 1))[sl][st.valid_rl[sl]]
    assert np.median(epe) < 0.5


# ----------------------------------------------------------- refine
def _ramp(H, W, fn):
    yy, xx = np.mgrid[0:H, 0:W]
    return fn(xx, yy).astype(np.uint8)


def test_refine_x_ramp_closed_form(orc):
    # A = 2x + 10, B(x) = A(x - s): one Gauss-Newton step shrinks the error
    # by 1 / (a^2 + 1) with a = 2 (window sum 25 a^2 against eps = 25)
    H, W, s = 32, 48, 3
    A = _ramp(H, W, lambda x, y: 2 * x + 10)
    B = _ramp(H, W, lambda x, y: 2 * (x - s) + 10 + 0 * y)
    D0 = np.zeros((H, W, 2), np.int32)
    D0[..., 0] = s - 1
    u = orc.refine(A, B, D0, orc.Params())
    inner = (slice(6, H - 6), slice(8, W - 8))
    assert np.allclose(u[inner][..., 0], s - 1.0 / 25.0, atol=1e-12)
    assert np.allclose(u[inner][..., 1], 0.0, atol=1e-12)


def test_refine_y_ramp_closed_form(orc):
    H, W, s = 48, 32, -2
    A = _ramp(H, W, lambda x, y: 2 * y + 20 + 0 * x)
    B = _ramp(H, W, lambda x, y: 2 * (y - s) + 20 + 0 * x)
    D0 = np.zeros((H, W, 2), np.int32)
    D0[..., 1] = s + 1
    u = orc.refine(A, B, D0, orc.Params())
    inner = (slice(8, H - 8), slice(6, W - 6))
    assert np.allclose(u[inner][..., 1], s + 1.0 / 25.0, atol=1e-12)
    assert np.allclose(u[inner][..., 0], 0.0, atol=1e-12)


def test_refine_diagonal_ramp_cross_term(orc):
    # A = x + y + 10: H = 25 [[2, 1], [1, 2]], each step moves both
    # components by -(ex + ey) / 3; from (sx - 1, sy) two steps give
    # (sx - 5/9, sy + 4/9)
    H, W, sx, sy = 40, 40, 2, 2
    A = _ramp(H, W, lambda x, y: x + y + 10)
    B = _ramp(H, W, lambda x, y: x + y + 10 - sx - sy)
    D0 = np.zeros((H, W, 2), np.int32)
    D0[..., 0] = sx - 1
    D0[..., 1] = sy
    u = orc.refine(A, B, D0, orc.Params())
    inner = (slice(8, H - 8), slice(8, W - 8))
    assert np.allclose(u[inner][..., 0], sx - 5.0 / 9.0, atol=1e-12)
    assert np.allclose(u[inner][..., 1], sy + 4.0 / 9.0, atol=1e-12)


@pytest.mark.parametrize("side", [-1, 1])
def test_refine_clamp_holds_one_pixel_from_the_seed(orc, side):
    # A = 2x + 10, B(x) = A(x - s), seed 3 px from the answer: the first
    # Gauss-Newton step moves by 3 * 100 / 125 = 2.4 px, past the +-1 px
    # band around the seed, so the clamp holds it at seed +- 1; the second
    # step (2 px off, a 1.6 px move) is clamped again. Without the clamp the
    # two steps would end 0.12 px from s.
    H, W, s = 32, 64, 3
    A = _ramp(H, W, lambda x, y: 2 * x + 10 + 0 * y)
    B = _ramp(H, W, lambda x, y: 2 * (x - s) + 10 + 0 * y)
    D0 = np.zeros((H, W, 2), np.int32)
    D0[..., 0] = s + 3 * side
    u = orc.refine(A, B, D0, orc.Params())
    inner = (slice(6, H - 6), slice(12, W - 12))
    assert (u[inner][..., 0] == s + 2 * side).all()
    assert (u[inner][..., 1] == 0.0).all()
    # one step: the clamp binds after the first move as well
    u1 = orc.refine(A, B, D0, orc.Params(lk_iters=1))
    assert (u1[inner][..., 0] == s + 2 * side).all()


def test_refine_clamp_on_the_vertical_component(orc):
    H, W, s = 64, 32, -2
    A = _ramp(H, W, lambda x, y: 2 * y + 20 + 0 * x)
    B = _ramp(H, W, lambda x, y: 2 * (y - s) + 20 + 0 * x)
    D0 = np.zeros((H, W, 2), np.int32)
    D0[..., 1] = s - 3
    u = orc.refine(A, B, D0, orc.Params())
    inner = (slice(12, H - 12), slice(6, W - 6))
    assert (u[inner][..., 1] == s - 2).all()
    assert (u[inner][..., 0] == 0.0).all()


def test_refine_keeps_exact_integer_flow(orc):
    L, R = _shifted_pair(12, 40, 40, 2, -1)
    yl, yr = orc.luma(L), orc.luma(R)
    D0 = np.zeros((40, 40, 2), np.int32)
    D0[...] = (2, -1)
    u = orc.refine(yr, yl, D0, orc.Params())
    inner = (slice(6, 34), slice(6, 34))
    assert (u[inner] == np.array([2.0, -1.0])).all()


def test_refine_subpixel_sinusoid(orc):
    # band-limited pattern shifted by a known sub-pixel amount
    H, W, s = 32, 64, 0.4
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    pat = lambda x, y: 128 + 60 * np.sin(2 * np.pi * x / 23.0) + 40 * np.cos(2 * np.pi * y / 19.0)
    A = np.rint(pat(xx, yy)).astype(np.uint8)
    B = np.rint(pat(xx - s, yy)).astype(np.uint8)  # A(p) ~ B(p + s)
    u = orc.refine(A, B, np.zeros((H, W, 2), np.int32), orc.Params())
    inner = (slice(6, H - 6), slice(6, W - 6))
    assert np.median(np.abs(u[inner][..., 0] - s)) < 0.05


# ------------------------------------------------- exposure compensation
def test_gain_comp_unit_gain_is_identity(orc):
    y = synth.random_bytes(20, (31, 47))
    assert np.array_equal(orc.gain_comp(y, y), y)


def test_gain_comp_recovers_exact_gain(orc):
    # R = L scaled by a known gain (mid-range values, no clipping): the
    # compensated R is L up to the two roundings (within 1 gray level)
    r = synth.rng_for(121, 0, 0)
    yl = r.integers(60, 180, size=(40, 50)).astype(np.uint8)
    for g in (0.9, 0.93, 1.07, 1.1):
        yr = np.clip(np.rint(yl * g), 0, 255).astype(np.uint8)
        out = orc.gain_comp(yl, yr)
        assert np.abs(out.astype(int) - yl.astype(int)).max() <= 1


def test_gain_comp_fixed_point_formula(orc):
    yl = np.array([[10, 20, 30, 255]], np.uint8)
    yr = np.array([[5, 10, 15, 200]], np.uint8)
    a = (int(yl.sum()) << 16) // int(yr.sum())
    expect = np.minimum(255, (yr.astype(np.int64) * a + (1 << 15)) >> 16)
    assert np.array_equal(orc.gain_comp(yl, yr), expect.astype(np.uint8))
    z = np.zeros((2, 3), np.uint8)
    assert np.array_equal(orc.gain_comp(yl[:, :3].repeat(2, 0), z), z)


def test_gain_compensated_flow_is_accurate_under_exposure_gain(orc):
    st = synth.make_random(21, 96, 160, max_ux=6, max_uy=2)
    R = np.clip(np.rint(st.R.astype(float) * 0.9), 0, 255).astype(np.uint8)
    m = 12
    sl = (slice(m, -m), slice(m, -m))
    for gain, bound in ((1, 0.5), (0, None)):
        _, frl = orc.flow_bidirectional(st.L, R, orc.Params(levels=3, gain_comp=gain))
        e = np.hypot(*(frl - st.flow_rl_gt).transpose(2, 0, 1))[sl][st.valid_rl[sl]]
        if bound is not None:
            assert np.median(e) < bound
