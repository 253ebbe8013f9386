"""torch.autograd.Function wrappers over libabf's hand-written adjoints.

FlowEnergy: the photometric Charbonnier + TV energy of a flow between two
float RGB images; its backward recomputes the warped samples (nothing but
the inputs is saved) and calls the energy-gradient kernel.
FlowEnergyMS: the same energy summed over a float pyramid of the images
and the flow; only the level-0 inputs are saved, and the backward
recomputes the pyramid levels and carries the coarse gradients down
through the pyramid's adjoint kernel.
AsymBlend: Code 1 over float RGB images; its backward calls the Code 1
adjoint kernel.
refine_flow: gradient descent on the energy, run on the stream without an
autograd tape.
"""
from __future__ import annotations

import torch

from .api import Plan


class FlowEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan: Plan, u, ref, tgt, lam: float = 0.05, eps: float = 1e-3):
        u, ref, tgt = u.contiguous(), ref.contiguous(), tgt.contiguous()
        E = plan.energy(ref, tgt, u, lam, eps, grads=False)
        ctx.plan, ctx.lam, ctx.eps = plan, lam, eps
        ctx.save_for_backward(u, ref, tgt)
        return E[0]

    @staticmethod
    def backward(ctx, gE):
        u, ref, tgt = ctx.saved_tensors
        # deterministic scatter for dE/dtgt: repeatable gradients
        _, gu, gr, gt = ctx.plan.energy(ref, tgt, u, ctx.lam, ctx.eps, grads=True, deterministic=True)
        return None, gu * gE, gr * gE, gt * gE, None, None


class FlowEnergyMS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan: Plan, u, ref, tgt, levels: int, lam: float = 0.05, eps: float = 1e-3):
        u, ref, tgt = u.contiguous(), ref.contiguous(), tgt.contiguous()
        E = plan.energy_ms(ref, tgt, u, levels, lam, eps, grads=False)
        ctx.plan, ctx.levels, ctx.lam, ctx.eps = plan, levels, lam, eps
        ctx.save_for_backward(u, ref, tgt)
        return E[0]

    @staticmethod
    def backward(ctx, gE):
        u, ref, tgt = ctx.saved_tensors
        _, gu, gr, gt = ctx.plan.energy_ms(ref, tgt, u, ctx.levels, ctx.lam, ctx.eps, grads=True,
                                           deterministic=True)
        return None, gu * gE, gr * gE, gt * gE, None, None, None


class AsymBlend(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan: Plan, L, R, flow_lr, flow_rl, blend=None, axis: int = 0):
        L, R, flow_lr, flow_rl = (t.contiguous() for t in (L, R, flow_lr, flow_rl))
        F = plan.blend_f32(L, R, flow_lr, flow_rl, blend, axis)
        ctx.plan, ctx.axis, ctx.blend = plan, axis, blend
        ctx.save_for_backward(L, R, flow_lr, flow_rl)
        return F

    @staticmethod
    def backward(ctx, gF):
        L, R, flr, frl = ctx.saved_tensors
        # deterministic scatter for the image gradients: repeatable gradients
        g_lr, g_rl, gL, gR = ctx.plan.blend_backward(L, R, flr, frl, gF.contiguous(), ctx.blend, ctx.axis,
                                                     deterministic=True)
        return None, gL, gR, g_lr, g_rl, None, None


def flow_energy(plan: Plan, u, ref, tgt, lam: float = 0.05, eps: float = 1e-3):
    return FlowEnergy.apply(plan, u, ref, tgt, lam, eps)


def flow_energy_ms(plan: Plan, u, ref, tgt, levels: int, lam: float = 0.05, eps: float = 1e-3):
    return FlowEnergyMS.apply(plan, u, ref, tgt, levels, lam, eps)


def asym_blend(plan: Plan, L, R, flow_lr, flow_rl, blend=None, axis: int = 0):
    return AsymBlend.apply(plan, L, R, flow_lr, flow_rl, blend, axis)


def refine_flow(plan: Plan, ref, tgt, u, steps: int = 50, eta: float = 0.5, lam: float = 0.05, eps: float = 1e-3,
                clip: float = 0.25):
    return plan.refine_flow(ref, tgt, u, steps, eta, lam, eps, clip)
