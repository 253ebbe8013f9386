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


@pytest.mark.parametrize("steps", [1, 2])
def test_refine_flow_steps_match_oracle(api, cfg3, steps):
    # one descent step is a function of its input: it must match elementwise
    # (the second step starts from the GPU's and the oracle's own first step,
    # which agree to ~1e-3 px)
    Ref, Tgt, u0, _ = _refine_crop(cfg3)
    H, W = u0.shape[:2]
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] refine_flow {steps} step(s)", flush=True)
    u = dev(u0)
    plan.refine_flow(dev(Ref), dev(Tgt), u, steps=steps, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
    o, _ = oracle.refine_gd(Ref, Tgt, u0, steps=steps, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
    d = np.abs(u.cpu().numpy() - o).max(axis=2)
    print(f"refine_flow {steps}: max {d.max():.3g}, within 1e-2 px {100 * (d <= 1e-2).mean():.3f}%")
    if steps == 1:
        assert d.max() <= 1e-2
    else:
        assert (d <= 1e-2).mean() >= 0.999


def test_refine_flow_50_steps_reaches_oracle_accuracy(api, cfg3):
    # With a Charbonnier eps of 1e-3 most steps are clipped to 0.25 px and the
    # descent ends oscillating around the optimum, so FP32 and FP64
    # trajectories part where a step's sign flips. Compared: what the two
    # reach (energy, endpoint error against the ground truth).
    Ref, Tgt, u0, gt = _refine_crop(cfg3)
    H, W = u0.shape[:2]
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    print("[gpu] refine_flow 50 steps", flush=True)
    u = dev(u0)
    plan.refine_flow(dev(Ref), dev(Tgt), u, steps=50, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
    g = u.cpu().numpy().astype(np.float64)
    o, hist = oracle.refine_gd(Ref, Tgt, u0, steps=50, eta=0.5, lam=LAM, eps=EPS, clip=0.25)
    Eg = oracle.energy(Ref, Tgt, g, LAM, EPS, grads=False)
    m = 8
    sl = (slice(m, -m), slice(m, -m))
    epe_g = np.hypot(*(g - gt).transpose(2, 0, 1))[sl]
    epe_o = np.hypot(*(o - gt).transpose(2, 0, 1))[sl]
    epe_0 = np.hypot(*(u0 - gt).transpose(2, 0, 1))[sl]
    d = np.abs(g - o).max(axis=2)
    print(f"50 steps: E oracle {hist[-1]:.2f} gpu {Eg:.2f} (start {hist[0]:.2f}); EPE median start "
          f"{np.median(epe_0):.4f} oracle {np.median(epe_o):.4f} gpu {np.median(epe_g):.4f}; "
          f"|gpu - oracle| <= 1e-2 px at {100 * (d <= 1e-2).mean():.1f}%")
    assert hist[-1] < hist[0] and Eg < hist[0]
    assert abs(Eg - hist[-1]) <= 0.01 * hist[-1]
    assert abs(np.median(epe_g) - np.median(epe_o)) <= 0.02
    assert abs(np.mean(epe_g) - np.mean(epe_o)) <= 0.02


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
