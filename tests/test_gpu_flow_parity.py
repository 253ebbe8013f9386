"""GPU parity of the flow and blend path against the CPU oracle.

Integer stages (luma pyramid, raw search, propagated + median flows) are
compared bit for bit at every level; the refined flows within 1e-2 px; the
blend (given the same float32 flows, taken from the oracle) within 0.5/255
of a gray level on the unrounded composite, and the rounded uint8 output
equal wherever the oracle's composite is farther than that bound from a
rounding boundary (and within 1 elsewhere).
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2006_01201_amd import synth

pytestmark = pytest.mark.gpu

FLOW_TOL = 1e-2
F_TOL = 0.5 / 255.0


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_01201_amd import api as _api

    return _api


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def o_params(p):
    return oracle.Params(**{k: getattr(p, k) for k in oracle.Params.__dataclass_fields__})


def _crop(cfg, strip, rows):
    st = synth.make_config_strip(cfg, 0, strip)
    return st.L[rows].copy(), st.R[rows].copy(), st.axis


CASES = {
    "cfg0": lambda: (lambda s: (s.L, s.R, s.axis, 3))(synth.make_config_strip(0, 0, 0)),
    "ragged_37x53": lambda: (lambda s: (s.L, s.R, 0, 3))(synth.make_random(1, 37, 53, max_ux=4, max_uy=2)),
    "occluder_130x197": lambda: (lambda s: (s.L, s.R, 0, 4))(
        synth.make_random(2, 130, 197, max_ux=10, max_uy=3, occluder=True)),
    "axis1_61x300": lambda: (lambda s: (s.L, s.R, 1, 4))(synth.make_random(3, 61, 300, axis=1, max_ux=8, max_uy=2)),
    "tiny_3x5": lambda: (lambda s: (s.L, s.R, 0, 2))(synth.make_random(4, 3, 5, max_ux=1, max_uy=1)),
    "single_row_1x70": lambda: (lambda s: (s.L, s.R, 0, 2))(synth.make_random(5, 1, 70, max_ux=2, max_uy=0)),
    "noise_tie_rich_40x72": lambda: (synth.random_levels(6, (40, 72, 3), 3), synth.random_levels(7, (40, 72, 3), 3),
                                     0, 3),
    "cfg1_rows_0_320": lambda: (*_crop(1, 0, slice(0, 320)), 6),
    # every gradient parallel to (1, 1): each window's normal matrix is
    # rank one plus eps I, the refinement's worst-conditioned case
    "diagonal_edges_90x120": lambda: (*_diagonal_pair(90, 120, 2.4), 0, 3),
    # flows that carry every sample of a border tile past the image edge
    "off_edge_shift_48x77": lambda: (*_shift_pair(48, 77, 21, 3), 0, 3),
    "off_edge_shift_neg_37x70": lambda: (*_shift_pair(37, 70, -25, -6), 0, 3),
}


def _shift_pair(H, W, sx, sy):
    big = synth.make_random(11, H + 64, W + 64, max_ux=0.0, max_uy=0.0, noise=0.0).L
    L = big[32:32 + H, 32:32 + W]
    R = big[32 + sy:32 + sy + H, 32 + sx:32 + sx + W]  # R(p) = L(p + s)
    return np.ascontiguousarray(L), np.ascontiguousarray(R)


def _diagonal_pair(H, W, s):
    # a texture of x + y only: random steps of 0..255 every 3 to 6 px,
    # softened by a 3-tap box; R(p) = L(p + (s, 0)) by linear interpolation
    r = synth.rng_for(123, H, W)
    n = H + W + 64
    steps = np.repeat(r.integers(0, 256, n), r.integers(3, 7, n))[:n + 8].astype(np.float64)
    prof = np.convolve(steps, np.ones(3) / 3.0, mode="same")
    t = np.arange(H)[:, None] + np.arange(W)[None, :] + 16.0
    def at(u):
        i = np.floor(u).astype(int)
        f = u - i
        return prof[i] * (1 - f) + prof[i + 1] * f
    L = np.clip(np.rint(at(t)), 0, 255).astype(np.uint8)
    R = np.clip(np.rint(at(t + s)), 0, 255).astype(np.uint8)
    return np.repeat(L[..., None], 3, axis=2), np.repeat(R[..., None], 3, axis=2)


def run_case(api, name, params=None):
    L, R, axis, levels = CASES[name]()
    p = api.Params(levels=levels) if params is None else dataclasses.replace(params, levels=levels)
    H, W = L.shape[:2]
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] case {name} {H}x{W} levels {p.levels}", flush=True)
    flr, frl = plan.flow_bidirectional(to_dev(L), to_dev(R))
    torch.cuda.synchronize()
    views = {}
    for lvl in range(p.levels):
        for d in range(2):
            views[(0, lvl, d)] = plan.view(0, 0, lvl, d).cpu().numpy()
            views[(1, lvl, d)] = plan.view(1, 0, lvl, d).cpu().numpy().astype(np.int32)
            views[(2, lvl, d)] = plan.view(2, 0, lvl, d).cpu().numpy().astype(np.int32)
    plan.close()
    return L, R, axis, p, flr.cpu().numpy(), frl.cpu().numpy(), views


@pytest.mark.parametrize("name", list(CASES))
def test_flow_parity(api, name):
    L, R, axis, p, g_lr, g_rl, views = run_case(api, name)
    op = o_params(p)
    o_lr, o_rl, lv = oracle.flow_bidirectional(L, R, op, levels_out=True)
    yl, yr = oracle.luma(L), oracle.luma(R)
    if p.gain_comp:
        yr = oracle.gain_comp(yl, yr)
    pyrL = oracle.pyramid(yl, p.levels)
    pyrR = oracle.pyramid(yr, p.levels)
    for k in range(p.levels):
        assert np.array_equal(views[(0, k, 0)], pyrL[k]), f"luma pyramid L level {k}"
        assert np.array_equal(views[(0, k, 1)], pyrR[k]), f"luma pyramid R level {k}"
        for d, tag in ((0, "lr"), (1, "rl")):
            assert np.array_equal(views[(1, k, d)], lv["search_" + tag][k]), f"search {tag} level {k}"
            assert np.array_equal(views[(2, k, d)], lv["final_" + tag][k]), f"final {tag} level {k}"
    assert np.abs(g_lr - o_lr).max() <= FLOW_TOL
    assert np.abs(g_rl - o_rl).max() <= FLOW_TOL


def test_flow_parity_lean_preset(api):
    L, R, axis, p, g_lr, g_rl, views = run_case(api, "occluder_130x197", api.Params.lean())
    op = o_params(p)
    o_lr, o_rl, lv = oracle.flow_bidirectional(L, R, op, levels_out=True)
    for k in range(p.levels):
        for d, tag in ((0, "lr"), (1, "rl")):
            assert np.array_equal(views[(2, k, d)], lv["final_" + tag][k]), f"final {tag} level {k}"
    assert np.abs(g_lr - o_lr).max() <= FLOW_TOL
    assert np.abs(g_rl - o_rl).max() <= FLOW_TOL


@pytest.mark.parametrize("T,M,R", [(0, 0, 1), (1, 0, 3), (0, 1, 2), (4, 1, 2), (3, 0, 4)])
def test_flow_parity_param_grid(api, T, M, R):
    s = synth.make_random(9, 70, 90, max_ux=6, max_uy=2)
    p = api.Params(levels=3, prop_steps=T, median=M, radius=R, radius_coarse=R)
    plan = api.Plan(p, max_strips=1, max_H=70, max_W=90)
    print(f"[gpu] param grid T={T} M={M} R={R}", flush=True)
    flr, frl = plan.flow_bidirectional(to_dev(s.L), to_dev(s.R))
    d0 = plan.view(2, 0, 0, 1).cpu().numpy().astype(np.int32)
    o_lr, o_rl, lv = oracle.flow_bidirectional(s.L, s.R, o_params(p), levels_out=True)
    assert np.array_equal(d0, lv["final_rl"][0])
    assert np.abs(frl.cpu().numpy() - o_rl).max() <= FLOW_TOL
    assert np.abs(flr.cpu().numpy() - o_lr).max() <= FLOW_TOL


@pytest.mark.parametrize("R,Rc", [(2, 2), (4, 4), (1, 4)])
def test_flow_parity_patch3x3(api, R, Rc):
    # 3x3 patches in the search and the propagation at every radius
    L, R_img, _, _ = CASES["occluder_130x197"]()
    H, W = L.shape[:2]
    p = api.Params(levels=4, patch=1, radius=R, radius_coarse=Rc)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] 3x3 patches R={R} Rc={Rc}", flush=True)
    flr, frl = plan.flow_bidirectional(to_dev(L), to_dev(R_img))
    torch.cuda.synchronize()
    o_lr, o_rl, lv = oracle.flow_bidirectional(L, R_img, o_params(p), levels_out=True)
    for k in range(p.levels):
        for d, tag in ((0, "lr"), (1, "rl")):
            assert np.array_equal(plan.view(1, 0, k, d).cpu().numpy().astype(np.int32), lv["search_" + tag][k])
            assert np.array_equal(plan.view(2, 0, k, d).cpu().numpy().astype(np.int32), lv["final_" + tag][k])
    assert np.abs(flr.cpu().numpy() - o_lr).max() <= FLOW_TOL
    assert np.abs(frl.cpu().numpy() - o_rl).max() <= FLOW_TOL


@pytest.mark.parametrize("levels", [1, 8, 12])
def test_flow_parity_pyramid_depths(api, levels):
    # one level (the search at the coarse radius with no centre) and
    # pyramids that reach 1 x 1 and repeat it up to the maximum depth
    L, R, _, _ = CASES["ragged_37x53"]()
    H, W = L.shape[:2]
    p = api.Params(levels=levels)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] pyramid depth {levels}", flush=True)
    flr, frl = plan.flow_bidirectional(to_dev(L), to_dev(R))
    torch.cuda.synchronize()
    o_lr, o_rl, lv = oracle.flow_bidirectional(L, R, o_params(p), levels_out=True)
    for k in range(levels):
        for d, tag in ((0, "lr"), (1, "rl")):
            g = plan.view(2, 0, k, d).cpu().numpy().astype(np.int32)
            assert np.array_equal(g, lv["final_" + tag][k]), f"final {tag} level {k}"
    assert np.abs(flr.cpu().numpy() - o_lr).max() <= FLOW_TOL
    assert np.abs(frl.cpu().numpy() - o_rl).max() <= FLOW_TOL


@pytest.mark.parametrize("kw", [dict(lk_patch=3, lk_iters=3), dict(lk_patch=1, lk_iters=4, lk_eps=4.0),
                                dict(lk_iters=8, lk_eps=100.0), dict(lk_iters=0), dict(gain_comp=1)],
                         ids=["window7_K3", "window3_K4_eps4", "K8_eps100", "K0", "exposure_step"])
def test_flow_parity_refinement_params(api, kw):
    # the refinement's other windows (3x3, 7x7), step counts (none, up to
    # the maximum 8) and regularisations, and the path with the exposure
    # step
    L, R, axis, p, g_lr, g_rl, views = run_case(api, "occluder_130x197", dataclasses.replace(api.Params(), **kw))
    o_lr, o_rl, lv = oracle.flow_bidirectional(L, R, o_params(p), levels_out=True)
    for k in range(p.levels):
        for d, tag in ((0, "lr"), (1, "rl")):
            assert np.array_equal(views[(2, k, d)], lv["final_" + tag][k]), f"final {tag} level {k}"
    assert np.abs(g_lr - o_lr).max() <= FLOW_TOL
    assert np.abs(g_rl - o_rl).max() <= FLOW_TOL
    if kw.get("lk_iters") == 0:
        # no Gauss-Newton step: the refined flow is the integer flow
        assert np.array_equal(g_lr, views[(2, 0, 0)].astype(np.float32))
        assert np.array_equal(g_rl, views[(2, 0, 1)].astype(np.float32))


@pytest.mark.parametrize("ks,kf", [(60.0, 80.0), (0.5, 0.0)], ids=["sharp", "flat"])
def test_blend_softmax_parameters(api, ks, kf):
    # a sharp softmax (exponents in the hundreds, nearly a hard switch) and
    # a flat one without the flow-magnitude term
    L, R, axis, levels = CASES["occluder_130x197"]()
    H, W = L.shape[:2]
    p = api.Params(levels=levels, k_sharp=ks, k_flowmag=kf)
    op = o_params(p)
    o_lr, o_rl = oracle.flow_bidirectional(L, R, op)
    f_lr, f_rl = o_lr.astype(np.float32), o_rl.astype(np.float32)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] blend kS={ks} kF={kf}", flush=True)
    F8, Ff = plan.blend_asymmetric(to_dev(L), to_dev(R), to_dev(f_lr), to_dev(f_rl), axis=axis, f32=True)
    oF, _ = oracle.blend(L, R, f_lr, f_rl, axis=axis, params=op)
    _check_blend(F8.cpu().numpy(), Ff.cpu().numpy(), oF)


def _check_blend(F8, Ff, oF):
    assert np.abs(Ff - oF).max() <= F_TOL
    r = oF - np.floor(oF)
    safe = np.abs(r - 0.5) > F_TOL
    o8 = np.clip(np.floor(oF + 0.5), 0, 255).astype(np.uint8)
    assert np.array_equal(F8[safe], o8[safe])
    assert np.abs(F8.astype(int) - o8.astype(int)).max() <= 1


@pytest.mark.parametrize("name", ["cfg0", "ragged_37x53", "axis1_61x300", "cfg1_rows_0_320"])
@pytest.mark.parametrize("mode", ["eq1", "user", "linear"])
def test_blend_parity(api, name, mode):
    L, R, axis, levels = CASES[name]()
    H, W = L.shape[:2]
    p = api.Params(levels=levels, blend_mode=1 if mode == "linear" else 0)
    op = o_params(p)
    o_lr, o_rl = oracle.flow_bidirectional(L, R, op)
    f_lr, f_rl = o_lr.astype(np.float32), o_rl.astype(np.float32)
    blend = synth.rng_for(120, H, W).uniform(0, 1, (H, W)).astype(np.float32) if mode == "user" else None
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] blend {name} {mode}", flush=True)
    F8, Ff = plan.blend_asymmetric(to_dev(L), to_dev(R), to_dev(f_lr), to_dev(f_rl),
                                   blend=None if blend is None else to_dev(blend), axis=axis, f32=True)
    oF, _ = oracle.blend(L, R, f_lr, f_rl, blend=blend, axis=axis, params=op)
    _check_blend(F8.cpu().numpy(), Ff.cpu().numpy(), oF)


def test_blend_non_finite_flows(api):
    L, R, axis, levels = CASES["ragged_37x53"]()
    H, W = L.shape[:2]
    r = synth.rng_for(121, 0, 0)
    f_lr = r.uniform(-5, 5, (H, W, 2)).astype(np.float32)
    f_rl = r.uniform(-5, 5, (H, W, 2)).astype(np.float32)
    f_lr[::3, ::2, 0] = np.nan
    f_rl[1::4, ::3, 1] = np.inf
    f_rl[2::5, 1::3, 0] = -np.inf
    p = api.Params(levels=levels)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print("[gpu] blend non-finite", flush=True)
    F8, Ff = plan.blend_asymmetric(to_dev(L), to_dev(R), to_dev(f_lr), to_dev(f_rl), axis=0, f32=True)
    oF, _ = oracle.blend(L, R, f_lr, f_rl, axis=0, params=o_params(p))
    _check_blend(F8.cpu().numpy(), Ff.cpu().numpy(), oF)


def test_blend_large_flows_and_pitched_images(api):
    # displacements far outside the strip (clamped sampling) and images
    # whose rows are padded (pitch > 3 W)
    H, W = 48, 80
    s = synth.make_random(8, H, W)
    r = synth.rng_for(122, 0, 0)
    f_lr = r.uniform(-150, 150, (H, W, 2)).astype(np.float32)
    f_rl = r.uniform(-150, 150, (H, W, 2)).astype(np.float32)
    padL = np.zeros((H, W + 7, 3), np.uint8)
    padR = np.zeros((H, W + 3, 3), np.uint8)
    padL[:, :W] = s.L
    padR[:, :W] = s.R
    p = api.Params(levels=3)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print("[gpu] blend large flows, pitched", flush=True)
    F8, Ff = plan.blend_asymmetric(to_dev(padL)[:, :W], to_dev(padR)[:, :W], to_dev(f_lr), to_dev(f_rl), axis=0,
                                   f32=True)
    oF, _ = oracle.blend(s.L, s.R, f_lr, f_rl, axis=0, params=o_params(p))
    _check_blend(F8.cpu().numpy(), Ff.cpu().numpy(), oF)


def test_flow_pitched_images(api):
    s = synth.make_random(10, 50, 70, max_ux=5)
    padL = np.zeros((50, 75, 3), np.uint8)
    padR = np.zeros((50, 71, 3), np.uint8)
    padL[:, :70] = s.L
    padR[:, :70] = s.R
    p = api.Params(levels=3)
    plan = api.Plan(p, max_strips=1, max_H=50, max_W=70)
    print("[gpu] flow pitched", flush=True)
    flr, frl = plan.flow_bidirectional(to_dev(padL)[:, :70], to_dev(padR)[:, :70])
    o_lr, o_rl = oracle.flow_bidirectional(s.L, s.R, o_params(p))
    assert np.abs(flr.cpu().numpy() - o_lr).max() <= FLOW_TOL
    assert np.abs(frl.cpu().numpy() - o_rl).max() <= FLOW_TOL


def test_plan_limits_are_enforced(api):
    p = api.Params(levels=3)
    plan = api.Plan(p, max_strips=1, max_H=32, max_W=32)
    L = torch.zeros((33, 32, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        plan.flow_bidirectional(L, L)
    with pytest.raises(ValueError):
        plan.flow_bidirectional(L[:, :, :2], L[:, :, :2])


@pytest.mark.parametrize("pad,start", [(1, 0), (2, 1), (3, 3), (5, 2)])
def test_blend_into_pitched_output(api, pad, start):
    # F written into a view of a larger buffer: every row starts at another
    # byte alignment; the view's bytes equal a contiguous output and the
    # bytes around it stay untouched
    L, R, axis, levels = CASES["ragged_37x53"]()
    H, W = L.shape[:2]
    p = api.Params(levels=levels)
    op = o_params(p)
    o_lr, o_rl = oracle.flow_bidirectional(L, R, op)
    args = (to_dev(L), to_dev(R), to_dev(o_lr.astype(np.float32)), to_dev(o_rl.astype(np.float32)))
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] blend pitched output pad {pad} start {start}", flush=True)
    ref = plan.blend_asymmetric(*args, axis=axis)
    big = torch.full((H, W + pad, 3), 77, dtype=torch.uint8, device="cuda")
    view = big[:, start:start + W]
    plan.blend_asymmetric(*args, axis=axis, out=view)
    torch.cuda.synchronize()
    b = big.cpu().numpy()
    assert np.array_equal(b[:, start:start + W], ref.cpu().numpy())
    outside = np.ones((H, W + pad), bool)
    outside[:, start:start + W] = False
    assert (b[outside] == 77).all()
