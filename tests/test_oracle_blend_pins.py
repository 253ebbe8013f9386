"""Pins of the CPU oracle's blend (eq. (1) and Code 1 of the paper) and of
the flow-refinement energy and adjoints (an extension) against closed
forms, brute-force distances, the literal form of Code 1 and FP64 central
differences."""
import math

import numpy as np
import pytest

from paper_2006_01201_amd import synth


# ------------------------------------------------------------ eq. (1)
@pytest.mark.parametrize("H,W,axis", [(7, 5, 0), (4, 9, 1), (1, 1, 0), (3, 64, 0)])
def test_blend_coef_from_brute_force_distances(orc, H, W, axis):
    # Canvas: Area1 is the column left of the strip (axis 0) or the row
    # above it (axis 1); Area2 the column right / row below. Minimum
    # Euclidean distances are taken over all pixel centres of each area.
    got = orc.blend_coef(H, W, axis)
    for y in range(H):
        for x in range(W):
            if axis == 0:
                a1 = [(-1, yy) for yy in range(-3, H + 3)]
                a2 = [(W, yy) for yy in range(-3, H + 3)]
            else:
                a1 = [(xx, -1) for xx in range(-3, W + 3)]
                a2 = [(xx, H) for xx in range(-3, W + 3)]
            lmin = min(math.hypot(x - ax, y - ay) for ax, ay in a1)
            rmin = min(math.hypot(x - ax, y - ay) for ax, ay in a2)
            assert abs(got[y, x] - lmin / (lmin + rmin)) < 1e-15


# ------------------------------------------------------------ Code 1
def _imgs(seed, H=24, W=32):
    s = synth.make_random(seed, H, W, max_ux=4, max_uy=2)
    return s.L, s.R


def _flows(seed, H, W, scale=5.0):
    r = synth.rng_for(110, seed, 0)
    return r.uniform(-scale, scale, (H, W, 2)), r.uniform(-scale, scale, (H, W, 2))


def test_weight_zero_returns_L_exactly(orc):
    L, R = _imgs(1)
    H, W, _ = L.shape
    flr, frl = _flows(1, H, W)
    F, F8 = orc.blend(L, R, flr, frl, blend=np.zeros((H, W)))
    assert np.array_equal(F8, L)
    # |F - L| <= 255 * sigma(-kS)
    assert np.abs(F - L).max() <= 255.0 / (1.0 + math.exp(10.0)) + 1e-12


def test_weight_one_returns_R_exactly(orc):
    L, R = _imgs(2)
    H, W, _ = L.shape
    flr, frl = _flows(2, H, W)
    F, F8 = orc.blend(L, R, flr, frl, blend=np.ones((H, W)))
    assert np.array_equal(F8, R)


def test_linear_mode_is_exact_at_endpoints(orc):
    L, R = _imgs(3)
    H, W, _ = L.shape
    flr, frl = _flows(3, H, W)
    lin = orc.Params(blend_mode=1)
    F0, _ = orc.blend(L, R, flr, frl, blend=np.zeros((H, W)), params=lin)
    F1, _ = orc.blend(L, R, flr, frl, blend=np.ones((H, W)), params=lin)
    assert np.array_equal(F0, L.astype(float)) and np.array_equal(F1, R.astype(float))


def test_same_image_zero_flow_returns_it(orc):
    L, _ = _imgs(4)
    H, W, _ = L.shape
    z = np.zeros((H, W, 2))
    F, F8 = orc.blend(L, L, z, z)
    assert np.abs(F - L).max() < 1e-12 and np.array_equal(F8, L)


def test_warp_direction_and_scaling(orc):
    # linear weights, Blend = 1/2 everywhere: L is displaced by
    # FlowRtoL * Blend and R by FlowLtoR * (1 - Blend) (the warp of Code 1)
    L, R = _imgs(5, 32, 48)
    H, W, _ = L.shape
    frl = np.zeros((H, W, 2))
    frl[..., 0] = 6.0  # L sampled 3 px to the right
    flr = np.zeros((H, W, 2))
    flr[..., 1] = -4.0  # R sampled 2 px up
    F, _ = orc.blend(L, R, flr, frl, blend=np.full((H, W), 0.5), params=orc.Params(blend_mode=1))
    Ls = np.roll(L.astype(float), -3, axis=1)
    Rs = np.roll(R.astype(float), 2, axis=0)
    inner = (slice(4, H - 4), slice(4, W - 4))
    assert np.allclose(F[inner], 0.5 * Ls[inner] + 0.5 * Rs[inner], atol=1e-12)


def test_softmax_matches_literal_code1(orc):
    # constant colours, so only the weights matter; the softmax weights of
    # Code 1 written out with exp (fine at these magnitudes)
    H, W = 3, 50
    a, b = 40.0, 200.0
    L = np.full((H, W, 3), a)
    R = np.full((H, W, 3), b)
    r = synth.rng_for(111, 0, 0)
    flr = r.uniform(-30, 30, (H, W, 2))
    frl = r.uniform(-30, 30, (H, W, 2))
    kS, kF = 10.0, 20.0
    F, _ = orc.blend(L, R, flr, frl)
    for y in range(H):
        for x in range(W):
            blend = (x + 1) / (W + 1)
            blendL, blendR = 1 - blend, blend
            mag_rl = math.hypot(*frl[y, x]) / W
            mag_lr = math.hypot(*flr[y, x]) / W
            expL = math.exp(kS * blendL * (1 + kF * mag_rl))
            expR = math.exp(kS * blendR * (1 + kF * mag_lr))
            expect = a * expL / (expL + expR) + b * expR / (expL + expR)
            assert abs(F[y, x, 0] - expect) < 1e-9


def test_half_weight_equal_magnitudes(orc):
    H, W = 1, 1
    L = np.full((H, W, 3), 10.0)
    R = np.full((H, W, 3), 30.0)
    f = np.array([[[3.0, 4.0]]])
    g = np.array([[[-4.0, 3.0]]])
    F, _ = orc.blend(L, R, f, g, blend=np.full((1, 1), 0.5))
    assert abs(F[0, 0, 0] - 20.0) < 1e-12


def test_non_finite_flow_is_zero(orc):
    L, R = _imgs(6)
    H, W, _ = L.shape
    flr, frl = _flows(6, H, W)
    bad_lr, bad_rl = flr.copy(), frl.copy()
    bad_lr[::3, ::2, 0] = np.nan
    bad_rl[1::4, ::3, 1] = np.inf
    ref_lr, ref_rl = flr.copy(), frl.copy()
    ref_lr[::3, ::2, 0] = 0
    ref_rl[1::4, ::3, 1] = 0
    F1, _ = orc.blend(L, R, bad_lr, bad_rl)
    F2, _ = orc.blend(L, R, ref_lr, ref_rl)
    assert np.array_equal(F1, F2)


def test_axis1_is_transpose_of_axis0(orc):
    L, R = _imgs(7, 20, 28)
    flr, frl = _flows(7, 20, 28)
    F0, _ = orc.blend(L, R, flr, frl, axis=0)
    tr = lambda a: np.ascontiguousarray(a.transpose(1, 0, 2))
    F1, _ = orc.blend(tr(L), tr(R), tr(flr[..., ::-1]), tr(frl[..., ::-1]), axis=1)
    assert np.allclose(tr(F1), F0, atol=1e-9)


# ------------------------------------------------------------ energy
def test_energy_closed_form_identical_images(orc):
    s = synth.make_random(8, 16, 12, float_out=True)
    H, W = 16, 12
    lam, eps = 0.05, 1e-3
    E = orc.energy(s.L, s.L, np.zeros((H, W, 2)), lam, eps, grads=False)
    assert abs(E - H * W * (3 * eps + 2 * lam * eps)) < 1e-12


def test_energy_zero_flow_is_charbonnier_of_difference(orc):
    s = synth.make_random(9, 16, 12, float_out=True)
    lam, eps = 0.05, 1e-3
    r = s.L.astype(float) - s.R.astype(float)
    E = orc.energy(s.R, s.L, np.zeros((16, 12, 2)), lam, eps, grads=False)
    assert abs(E - (np.sqrt(r ** 2 + eps ** 2).sum() + 2 * lam * eps * 16 * 12)) < 1e-9


def test_energy_tv_of_linear_flow(orc):
    # u_x = a * x: forward difference a everywhere except the last column
    H, W, a = 6, 7, 0.3
    lam, eps = 0.05, 1e-3
    img = np.full((H, W, 3), 0.5)
    u = np.zeros((H, W, 2))
    u[..., 0] = a * np.arange(W)[None, :]
    E = orc.energy(img, img, u, lam, eps, grads=False)
    tv = H * (W - 1) * math.sqrt(a * a + eps * eps) + H * 1 * eps + H * W * eps
    assert abs(E - (H * W * 3 * eps + lam * tv)) < 1e-12


def _fd_points(u, H, W, n, seed, margin=4):
    r = synth.rng_for(112, seed, 0)
    pts = []
    while len(pts) < n:
        y, x = int(r.integers(margin, H - margin)), int(r.integers(margin, W - margin))
        fr = u[y, x] - np.floor(u[y, x])
        if ((fr > 0.05) & (fr < 0.95)).all():
            pts.append((y, x))
    return pts


def test_energy_gradients_match_central_differences(orc):
    st = synth.make_config_strip(3, 0, 0)
    rows, cols = slice(992, 1056), slice(240, 272)
    Ref = st.R[rows, cols].astype(np.float64)
    Tgt = st.L[rows, cols].astype(np.float64)
    u = st.flow_rl_gt[rows, cols].astype(np.float64) * 0.05 + 0.3
    H, W = Ref.shape[:2]
    lam, eps, h = 0.05, 1e-3, 1e-6
    E, gu, gr, gt = orc.energy(Ref, Tgt, u, lam, eps)
    for (y, x) in _fd_points(u, H, W, 12, 0):
        for m in range(2):
            up, um = u.copy(), u.copy()
            up[y, x, m] += h
            um[y, x, m] -= h
            fd = (orc.energy(Ref, Tgt, up, lam, eps, False) - orc.energy(Ref, Tgt, um, lam, eps, False)) / (2 * h)
            assert abs(fd - gu[y, x, m]) <= 1e-6 * max(1.0, abs(fd))
        for c in range(3):
            for img, g in ((Ref, gr), (Tgt, gt)):
                ip, im = img.copy(), img.copy()
                ip[y, x, c] += h
                im[y, x, c] -= h
                args_p = (ip, Tgt) if img is Ref else (Ref, ip)
                args_m = (im, Tgt) if img is Ref else (Ref, im)
                fd = (orc.energy(*args_p, u, lam, eps, False) - orc.energy(*args_m, u, lam, eps, False)) / (2 * h)
                assert abs(fd - g[y, x, c]) <= 1e-6 * max(1.0, abs(fd))


def test_gradient_descent_lowers_energy(orc):
    st = synth.make_config_strip(3, 0, 0)
    rows, cols = slice(992, 1056), slice(240, 272)
    Ref = st.R[rows, cols].astype(np.float64)
    Tgt = st.L[rows, cols].astype(np.float64)
    u0 = np.rint(st.flow_rl_gt[rows, cols].astype(np.float64))
    u, hist = orc.refine_gd(Ref, Tgt, u0, steps=20)
    assert hist[-1] < hist[0]
    assert np.all(hist >= 0)


@pytest.mark.parametrize("sign", [-1, 1])
def test_descent_step_is_clipped(orc, sign):
    # lambda = 0, Tgt a ramp in x (slope a per channel) and Ref a constant
    # above (sign -1) or below (sign +1) every Tgt value: the residual keeps
    # its sign, so dE/du_x = 3 a rho'(r) has the sign of the residual and
    # |eta dE/du_x| = 50 * 3 * 0.005 ~ 0.75 > 0.25; every step is clipped to
    # exactly 0.25 px against the gradient, and dE/du_y = 0 leaves u_y alone.
    H, W, a = 8, 64, 0.005
    xx = np.arange(W, dtype=np.float64)[None, :, None]
    Tgt = np.broadcast_to(0.1 + a * xx, (H, W, 3)).copy()
    Ref = np.full((H, W, 3), 0.95 if sign < 0 else 0.0)
    u0 = np.zeros((H, W, 2))
    u0[..., 0] = 10.0
    u0[..., 1] = 0.3
    steps = 6
    u, hist = orc.refine_gd(Ref, Tgt, u0, steps=steps, eta=50.0, lam=0.0, eps=1e-3, clip=0.25)
    # samples stay inside the ramp (x + 10 +- 1.5 within [0, W - 2])
    inner = (slice(None), slice(2, W - 14))
    assert (u[inner][..., 0] == 10.0 - sign * 0.25 * steps).all()
    assert (u[..., 1] == 0.3).all()
    # eta * |g| below the clip: the plain step eta * 3 a rho'(r), rho' = r / sqrt(r^2 + eps^2)
    u, _ = orc.refine_gd(Ref, Tgt, u0, steps=1, eta=5.0, lam=0.0, eps=1e-3, clip=0.25)
    r = 0.1 + a * (xx[0, :, 0] + 10.0) - Ref[0, 0, 0]
    step = 5.0 * 3 * a * r / np.sqrt(r * r + 1e-6)
    assert np.allclose(u[0, 2:W - 14, 0], 10.0 - step[2:W - 14], rtol=0, atol=1e-12)


def test_blend_adjoint_matches_central_differences(orc):
    s = synth.make_random(13, 20, 24, float_out=True, max_ux=3, max_uy=1)
    L = s.L.astype(np.float64) * 255
    R = s.R.astype(np.float64) * 255
    H, W = 20, 24
    r = synth.rng_for(113, 0, 0)
    flr = r.uniform(-3, 3, (H, W, 2)) + 0.37
    frl = r.uniform(-3, 3, (H, W, 2)) + 0.21
    gF = r.standard_normal((H, W, 3))
    glr, grl, gL, gR = orc.blend_grad(L, R, flr, frl, gF)
    f = lambda *a: float((orc.blend(*a)[0] * gF).sum())
    h = 1e-6
    t = ((np.arange(W) + 1) / (W + 1))[None, :, None]
    # sample positions of both warps away from the bilinear kinks
    pos = np.concatenate([frl * t, flr * (1 - t)], axis=-1)
    pts = _fd_points(pos, H, W, 10, 1, margin=5)
    for (y, x) in pts:
        for m in range(2):
            for arr, g, which in ((flr, glr, 0), (frl, grl, 1)):
                ap, am = arr.copy(), arr.copy()
                ap[y, x, m] += h
                am[y, x, m] -= h
                if which == 0:
                    fd = (f(L, R, ap, frl) - f(L, R, am, frl)) / (2 * h)
                else:
                    fd = (f(L, R, flr, ap) - f(L, R, flr, am)) / (2 * h)
                assert abs(fd - g[y, x, m]) <= 1e-6 * max(1.0, abs(fd))
        for c in range(3):
            # F is linear in the image values: a unit step is exact
            for img, g, which in ((L, gL, 0), (R, gR, 1)):
                ip, im = img.copy(), img.copy()
                ip[y, x, c] += 1.0
                im[y, x, c] -= 1.0
                fd = (f(ip, R, flr, frl) - f(im, R, flr, frl)) / 2.0 if which == 0 else \
                    (f(L, ip, flr, frl) - f(L, im, flr, frl)) / 2.0
                assert abs(fd - g[y, x, c]) <= 1e-9 * max(1.0, abs(fd))
