"""GPU parity of the multi-level energy (the energy summed over a float
pyramid of the images and the flow) and of its gradients, which the
coarse levels reach through the pyramid's adjoint kernel, against the FP64
oracle (itself pinned to central differences); its descent, step by step;
and its autograd wrapper."""
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


def f64(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("shape,levels,det", [((64, 32), 3, True), ((61, 45), 4, False), ((256, 200), 6, True),
                                              ((1, 9), 2, True)])
def test_energy_ms_and_gradients(api, cfg3, shape, levels, det):
    H, W = shape
    r0, c0 = 900, 150
    Ref, Tgt = cfg3.R[r0:r0 + H, c0:c0 + W], cfg3.L[r0:r0 + H, c0:c0 + W]
    u = cfg3.flow_rl_gt[r0:r0 + H, c0:c0 + W] + synth.rng_for(130, H, W).uniform(-1, 1, (H, W, 2))
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] energy_ms {H}x{W} levels {levels} deterministic {det}", flush=True)
    E, gu, gr, gt = plan.energy_ms(dev(Ref), dev(Tgt), dev(u), levels, LAM, EPS, deterministic=det)
    torch.cuda.synchronize()
    oE, ogu, ogr, ogt = oracle.energy_ms(f64(Ref), f64(Tgt), f64(u), levels, LAM, EPS)
    assert abs(float(E.item()) - oE) <= 1e-5 * oE
    grad_close(gu.cpu().numpy(), ogu)
    grad_close(gr.cpu().numpy(), ogr)
    grad_close(gt.cpu().numpy(), ogt)
    # E alone (no gradient pass) is the same number
    E2 = plan.energy_ms(dev(Ref), dev(Tgt), dev(u), levels, LAM, EPS, grads=False)
    torch.cuda.synchronize()
    assert float(E2.item()) == float(E.item())


def test_energy_ms_one_level_is_the_energy(api, cfg3):
    rows, cols = slice(992, 1056), slice(240, 272)
    Ref, Tgt, u = dev(cfg3.R[rows, cols]), dev(cfg3.L[rows, cols]), dev(cfg3.flow_rl_gt[rows, cols])
    plan = api.Plan(api.Params(), max_strips=1, max_H=64, max_W=32)
    print("[gpu] energy_ms levels 1", flush=True)
    a = plan.energy_ms(Ref, Tgt, u, 1, LAM, EPS, deterministic=True)
    b = plan.energy(Ref, Tgt, u, LAM, EPS, deterministic=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_energy_ms_full_strip_deterministic_and_repeatable(api, cfg3):
    # the 2048 x 512 strip, 6 levels: parity, and bit-identical gradients on a
    # second call
    plan = api.Plan(api.Params(), max_strips=1, max_H=2048, max_W=512)
    Ref, Tgt, u = dev(cfg3.R), dev(cfg3.L), dev(cfg3.flow_rl_gt)
    print("[gpu] energy_ms full strip, 6 levels", flush=True)
    a = [t.clone() for t in plan.energy_ms(Ref, Tgt, u, 6, LAM, EPS, deterministic=True)]
    b = plan.energy_ms(Ref, Tgt, u, 6, LAM, EPS, deterministic=True)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    oE, ogu, ogr, ogt = oracle.energy_ms(f64(cfg3.R), f64(cfg3.L), f64(cfg3.flow_rl_gt), 6, LAM, EPS)
    assert abs(float(a[0].item()) - oE) <= 1e-5 * oE
    grad_close(a[1].cpu().numpy(), ogu)
    grad_close(a[2].cpu().numpy(), ogr)
    grad_close(a[3].cpu().numpy(), ogt)


def test_refine_flow_ms_steps_match_oracle(api, cfg3):
    # every descent step from the GPU's own iterate: one oracle step on it
    # lands within 1e-2 px of the GPU's next iterate at every pixel
    H, W = 128, 96
    r0, c0 = 960, 200
    Ref, Tgt = cfg3.R[r0:r0 + H, c0:c0 + W], cfg3.L[r0:r0 + H, c0:c0 + W]
    u0 = cfg3.flow_rl_gt[r0:r0 + H, c0:c0 + W] + synth.rng_for(131, 0, 0).uniform(-1, 1, (H, W, 2))
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    dR, dT = dev(Ref), dev(Tgt)
    u = dev(u0)
    print("[gpu] refine_flow_ms 10 steps, 4 levels", flush=True)
    worst = 0.0
    for k in range(10):
        prev = u.cpu().numpy().astype(np.float64)
        plan.refine_flow_ms(dR, dT, u, 4, steps=1)
        torch.cuda.synchronize()
        want = oracle.refine_gd_ms(f64(Ref), f64(Tgt), prev, 4, steps=1)
        worst = max(worst, float(np.abs(u.cpu().numpy() - want).max()))
    assert worst <= 1e-2, worst
    # the energy went down over the steps
    E0 = oracle.energy_ms(f64(Ref), f64(Tgt), f64(u0), 4, grads=False)
    E1 = oracle.energy_ms(f64(Ref), f64(Tgt), u.cpu().numpy().astype(np.float64), 4, grads=False)
    assert E1 < E0


def test_flow_energy_ms_autograd(api, cfg3):
    from paper_2006_01201_amd import autograd

    rows, cols = slice(992, 1056), slice(240, 272)
    Ref, Tgt = cfg3.R[rows, cols], cfg3.L[rows, cols]
    u0 = cfg3.flow_rl_gt[rows, cols]
    plan = api.Plan(api.Params(), max_strips=1, max_H=64, max_W=32)
    u = dev(u0).requires_grad_(True)
    r = dev(Ref).requires_grad_(True)
    t = dev(Tgt).requires_grad_(True)
    print("[gpu] FlowEnergyMS autograd", flush=True)
    E = autograd.flow_energy_ms(plan, u, r, t, 3, LAM, EPS)
    (2.0 * E).backward()
    torch.cuda.synchronize()
    oE, ogu, ogr, ogt = oracle.energy_ms(f64(Ref), f64(Tgt), f64(u0), 3, LAM, EPS)
    assert abs(float(E.item()) - oE) <= 1e-5 * oE
    grad_close(u.grad.cpu().numpy(), 2 * ogu)
    grad_close(r.grad.cpu().numpy(), 2 * ogr)
    grad_close(t.grad.cpu().numpy(), 2 * ogt)
