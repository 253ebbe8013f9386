"""GPU parity of the differentiable path (energy, its gradients, gradient
descent refinement, Code 1 on float images and its adjoint) against the
FP64 CPU oracle, which is itself pinned to central differences."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_01201_amd import synth

pytestmark = pytest.mark.gpu

LAM, EPS = 0.05, 1e-3


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_01201_amd import api as _api

    return _api


@pytest.fixture(scope="module")
def cfg3():
    return synth.make_config_strip(3, 0, 0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def grad_close(g, o, rel=1e-3):
    g = g.astype(np.float64)
    assert np.linalg.norm(g - o) <= rel * max(np.linalg.norm(o), 1e-30)
    assert np.abs(g - o).max() <= rel * max(np.abs(o).max(), 1e-30)


def _energy_case(api, Ref, Tgt, u, deterministic):
    H, W = u.shape[:2]
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    E, gu, gr, gt = plan.energy(dev(Ref), dev(Tgt), dev(u), LAM, EPS, grads=True, deterministic=deterministic)
    torch.cuda.synchronize()
    oE, ogu, ogr, ogt = oracle.energy(Ref.astype(np.float64), Tgt.astype(np.float64), u.astype(np.float64), LAM, EPS)
    assert abs(float(E.item()) - oE) <= 1e-5 * oE
    grad_close(gu.cpu().numpy(), ogu)
    grad_close(gr.cpu().numpy(), ogr)
    grad_close(gt.cpu().numpy(), ogt)
    return plan, (E, gu, gr, gt)


@pytest.mark.parametrize("deterministic", [False, True])
def test_energy_and_gradients_fd_crop(api, cfg3, deterministic):
    rows, cols = slice(992, 1056), slice(240, 272)
    Ref, Tgt = cfg3.R[rows, cols], cfg3.L[rows, cols]
    u = cfg3.flow_rl_gt[rows, cols]
    print(f"[gpu] energy crop deterministic={deterministic}", flush=True)
    _energy_case(api, Ref, Tgt, u, deterministic)


def test_energy_and_gradients_full_strip(api, cfg3):
    u = cfg3.flow_rl_gt
    print("[gpu] energy full strip 2048x512", flush=True)
    _energy_case(api, cfg3.R, cfg3.L, u, True)


def test_deterministic_image_gradient_is_bitwise_repeatable(api, cfg3):
    rows, cols = slice(0, 512), slice(0, 512)
    Ref, Tgt, u = cfg3.R[rows, cols], cfg3.L[rows, cols], cfg3.flow_rl_gt[rows, cols]
    plan = api.Plan(api.Params(), max_strips=1, max_H=512, max_W=512)
    print("[gpu] deterministic energy twice", flush=True)
    a = [t.clone() for t in plan.energy(dev(Ref), dev(Tgt), dev(u), LAM, EPS, deterministic=True)]
    b = plan.energy(dev(Ref), dev(Tgt), dev(u), LAM, EPS, deterministic=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def _refine_crop(cfg3):
    rows, cols = slice(900, 1156), slice(128, 384)
    Ref, Tgt = cfg3.R[rows, cols], cfg3.L[rows, cols]
    u0 = np.rint(cfg3.flow_rl_gt[rows, cols]).astype(np.float32)
    return Ref, Tgt, u0, cfg3.flow_rl_gt[rows, cols].astype(np.float64)


def test_refine_flow_one_step_matches_oracle(api, cfg3):
    Ref, Tgt, u0, _ = _refine_crop(cfg3)
    H, W = u0.shape[:2]
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    print("[gpu] refine_flow 1 step", flush=True)
    u = dev(u0)
    plan.refine_flow(dev(Ref), dev(Tgt), u, steps=1, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
    o, _ = oracle.refine_gd(Ref, Tgt, u0, steps=1, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
    d = np.abs(u.cpu().numpy() - o).max()
    print(f"refine_flow 1 step: max {d:.3g} px")
    assert d <= 1e-2


def _quantise(a):
    return np.clip(np.rint(a.astype(np.float64) * 255.0), 0, 255).astype(np.uint8)


def test_cfg3_search_then_50_steps_every_step(api, cfg3):
    # the 2048 x 512 float strip: the search path on its uint8 quantisation
    # (6 levels), then 50 descent steps on FlowRtoL over the float images,
    # each step checked at every pixel against the oracle's step taken from
    # the GPU's own previous iterate (a step is a function of its input, so
    # this bounds every step; the FP32 and FP64 trajectories themselves part
    # where a clipped step's sign flips)
    H, W = cfg3.H, cfg3.W
    L8, R8 = _quantise(cfg3.L), _quantise(cfg3.R)
    p = api.Params(levels=6)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print("[gpu] cfg3 search + 50 descent steps, each checked", flush=True)
    flr, frl = plan.flow_bidirectional(torch.from_numpy(L8).cuda(), torch.from_numpy(R8).cuda())
    torch.cuda.synchronize()
    o_lr, o_rl = oracle.flow_bidirectional(L8, R8, oracle.Params(levels=6))
    e = max(np.abs(flr.cpu().numpy() - o_lr).max(), np.abs(frl.cpu().numpy() - o_rl).max())
    assert e <= 1e-2, e
    ref, tgt = dev(cfg3.R), dev(cfg3.L)
    u = frl.clone()
    uk = u.cpu().numpy()
    start = uk.copy()
    worst = 0.0
    for k in range(50):
        plan.refine_flow(ref, tgt, u, steps=1, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
        g = u.cpu().numpy()
        o, _ = oracle.refine_gd(cfg3.R, cfg3.L, uk, steps=1, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
        d = float(np.abs(g - o).max())
        worst = max(worst, d)
        assert d <= 1e-2, (k, d)
        uk = g
    # the 50 steps of one call are the same computation
    u50 = frl.clone()
    plan.refine_flow(ref, tgt, u50, steps=50, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
    assert torch.equal(u50, u)
    m = 8
    sl = (slice(m, H - m), slice(m, W - m))
    epe = lambda f: np.hypot(*(f - cfg3.flow_rl_gt).transpose(2, 0, 1))[sl][cfg3.valid_rl[sl]]
    e0, e1 = epe(start), epe(uk)
    E0 = oracle.energy(cfg3.R, cfg3.L, start, LAM, EPS, grads=False)
    E1 = oracle.energy(cfg3.R, cfg3.L, uk, LAM, EPS, grads=False)
    print(f"cfg3: search flows within {e:.3g} px; every descent step within {worst:.3g} px of the oracle's; "
          f"E {E0:.1f} -> {E1:.1f}; EPE(RtoL) median {np.median(e0):.4f} -> {np.median(e1):.4f} px, "
          f"mean {e0.mean():.4f} -> {e1.mean():.4f} px", flush=True)
    assert E1 < E0


def test_refine_strips_every_step(api, cfg3):
    # the batched descent over uneven crops, 20 steps one batched call at a
    # time, every strip of every step checked against the oracle's step from
    # the GPU's previous iterate; 20 single steps equal one 20-step call
    crops = [(slice(0, 200), slice(0, 300)), (slice(300, 420), slice(100, 377)), (slice(1000, 1003), slice(5, 9)),
             (slice(1500, 1757), slice(200, 461))]
    plan = api.Plan(api.Params(), max_strips=4, max_H=512, max_W=512)
    print("[gpu] refine_strips, 20 steps each checked", flush=True)
    host = [(cfg3.R[r, c], cfg3.L[r, c], np.rint(cfg3.flow_rl_gt[r, c]).astype(np.float32)) for r, c in crops]
    items = [(dev(a), dev(b), dev(u)) for a, b, u in host]
    whole = [(dev(a), dev(b), dev(u)) for a, b, u in host]
    uk = [u for _, _, u in host]
    worst = 0.0
    for k in range(20):
        plan.refine_strips(items, steps=1)
        torch.cuda.synchronize()
        for i, ((a, b, _), (_, _, ug)) in enumerate(zip(host, items)):
            g = ug.cpu().numpy()
            o, _ = oracle.refine_gd(a, b, uk[i], steps=1, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
            d = float(np.abs(g - o).max())
            worst = max(worst, d)
            assert d <= 1e-2, (k, i, d)
            uk[i] = g
    plan.refine_strips(whole, steps=20)
    torch.cuda.synchronize()
    for (_, _, a), (_, _, b) in zip(items, whole):
        assert torch.equal(a, b)
    print(f"refine_strips: every step within {worst:.3g} px of the oracle's", flush=True)


def _blend_inputs(seed, H=48, W=64, scale=6.0):
    s = synth.make_random(seed, H, W, float_out=True, max_ux=4, max_uy=2)
    r = synth.rng_for(140, seed, 0)
    flr = r.uniform(-scale, scale, (H, W, 2)).astype(np.float32)
    frl = r.uniform(-scale, scale, (H, W, 2)).astype(np.float32)
    return (s.L * 255).astype(np.float32), (s.R * 255).astype(np.float32), flr, frl


@pytest.mark.parametrize("axis", [0, 1])
def test_blend_f32_forward(api, axis):
    L, R, flr, frl = _blend_inputs(1)
    H, W = L.shape[:2]
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] blend_f32 axis {axis}", flush=True)
    F = plan.blend_f32(dev(L), dev(R), dev(flr), dev(frl), axis=axis).cpu().numpy()
    oF, _ = oracle.blend(L, R, flr, frl, axis=axis)
    assert np.abs(F - oF).max() <= 0.5 / 255


@pytest.mark.parametrize("axis,user_blend", [(0, False), (1, False), (0, True)])
def test_blend_backward(api, axis, user_blend):
    L, R, flr, frl = _blend_inputs(2)
    H, W = L.shape[:2]
    gF = synth.rng_for(141, 0, 0).standard_normal((H, W, 3)).astype(np.float32)
    blend = synth.rng_for(142, 0, 0).uniform(0, 1, (H, W)).astype(np.float32) if user_blend else None
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] blend backward axis {axis} user {user_blend}", flush=True)
    g = plan.blend_backward(dev(L), dev(R), dev(flr), dev(frl), dev(gF), blend=None if blend is None else dev(blend),
                            axis=axis)
    o = oracle.blend_grad(L, R, flr, frl, gF, blend=blend, axis=axis)
    for a, b in zip(g, o):
        grad_close(a.cpu().numpy(), b)


@pytest.mark.parametrize("scale", [1.0, 2.0 ** 40, 2.0 ** -60])
def test_blend_backward_deterministic(api, scale):
    # the order-independent image gradients: bitwise repeatable, equal to
    # the oracle's at any value scale of g_F (the fixed-point scale follows
    # the largest |g_F|: no overflow for large values, no loss for tiny ones)
    L, R, flr, frl = _blend_inputs(4)
    H, W = L.shape[:2]
    gF = (synth.rng_for(143, 0, 0).standard_normal((H, W, 3)) * scale).astype(np.float32)
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] deterministic blend backward, g_F scale {scale:g}", flush=True)
    args = (dev(L), dev(R), dev(flr), dev(frl), dev(gF))
    a = [t.clone() for t in plan.blend_backward(*args, deterministic=True)]
    b = plan.blend_backward(*args, deterministic=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    o = oracle.blend_grad(L, R, flr, frl, gF.astype(np.float64))
    for x, y in zip(a, o):
        grad_close(x.cpu().numpy(), y)


def test_autograd_functions(api, cfg3):
    from paper_2006_01201_amd import autograd as ag

    rows, cols = slice(992, 1056), slice(240, 272)
    Ref, Tgt, u = dev(cfg3.R[rows, cols]), dev(cfg3.L[rows, cols]), dev(cfg3.flow_rl_gt[rows, cols])
    plan = api.Plan(api.Params(), max_strips=1, max_H=64, max_W=32)
    print("[gpu] autograd", flush=True)
    u.requires_grad_(True)
    Ref.requires_grad_(True)
    Tgt.requires_grad_(True)
    E = ag.flow_energy(plan, u, Ref, Tgt, LAM, EPS)
    gu, gr, gt = torch.autograd.grad(2.0 * E, (u, Ref, Tgt))
    _, du, dr, dt = plan.energy(Ref.detach(), Tgt.detach(), u.detach(), LAM, EPS, deterministic=True)
    assert torch.equal(gu, 2 * du) and torch.equal(gr, 2 * dr) and torch.equal(gt, 2 * dt)

    L, R, flr, frl = (dev(a) for a in _blend_inputs(3, 32, 40))
    for t in (L, R, flr, frl):
        t.requires_grad_(True)
    F = ag.asym_blend(plan, L, R, flr, frl, None, 0)
    gF = torch.ones_like(F)
    grads = torch.autograd.grad(F, (flr, frl, L, R), gF)
    direct = plan.blend_backward(L.detach(), R.detach(), flr.detach(), frl.detach(), gF)
    for a, b in zip(grads, direct):
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-5)


def test_refine_strips_equals_per_strip_calls(api, cfg3):
    # uneven crops refined together, against one refine_flow call each
    crops = [(slice(0, 200), slice(0, 300)), (slice(300, 420), slice(100, 377)), (slice(1000, 1003), slice(5, 9))]
    items, ref = [], []
    plan = api.Plan(api.Params(), max_strips=4, max_H=512, max_W=512)
    print("[gpu] refine_strips", flush=True)
    for steps in (3, 4):
        items, ref = [], []
        for rows, cols in crops:
            R_, T_, u0 = cfg3.R[rows, cols], cfg3.L[rows, cols], np.rint(cfg3.flow_rl_gt[rows, cols])
            items.append((dev(R_), dev(T_), dev(u0)))
            ua = dev(u0)
            plan.refine_flow(dev(R_), dev(T_), ua, steps=steps)
            ref.append(ua)
        plan.refine_strips(items, steps=steps)
        torch.cuda.synchronize()
        for (_, _, u), r in zip(items, ref):
            assert torch.equal(u, r)
