"""Shared checks of the GPU parity tests: the HIP path's intermediates and
outputs of one strip against the CPU oracle run on the same inputs
(integer stages bit for bit, flows within 1e-2 px, the blend within
0.5/255 on the oracle's flows)."""
import numpy as np
import torch

import oracle

FLOW_TOL = 1e-2
F_TOL = 0.5 / 255.0


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def o_params(p):
    return oracle.Params(**{k: getattr(p, k) for k in oracle.Params.__dataclass_fields__})


def gpu_levels(plan, strip, levels):
    """Host copies of the plan's intermediates of one strip of the last
    flow call: luma, raw search and final integer flow per level and
    direction."""
    out = {}
    for k in range(levels):
        for d in range(2):
            out[(0, k, d)] = plan.view(0, strip, k, d).cpu().numpy()
            out[(1, k, d)] = plan.view(1, strip, k, d).cpu().numpy().astype(np.int32)
            out[(2, k, d)] = plan.view(2, strip, k, d).cpu().numpy().astype(np.int32)
    return out


def check_flows(name, L, R, op, views, g_lr, g_rl):
    o_lr, o_rl, lv = oracle.flow_bidirectional(L, R, op, levels_out=True)
    yl, yr = oracle.luma(L), oracle.luma(R)
    if op.gain_comp:
        yr = oracle.gain_comp(yl, yr)
    pyrL, pyrR = oracle.pyramid(yl, op.levels), oracle.pyramid(yr, op.levels)
    for k in range(op.levels):
        assert np.array_equal(views[(0, k, 0)], pyrL[k]), (name, "luma L", k)
        assert np.array_equal(views[(0, k, 1)], pyrR[k]), (name, "luma R", k)
        for d, tag in ((0, "lr"), (1, "rl")):
            assert np.array_equal(views[(1, k, d)], lv["search_" + tag][k]), (name, "search", tag, k)
            assert np.array_equal(views[(2, k, d)], lv["final_" + tag][k]), (name, "final", tag, k)
    e = max(np.abs(g_lr - o_lr).max(), np.abs(g_rl - o_rl).max())
    print(f"{name}: integer stages equal at {op.levels} levels, max |flow - oracle| {e:.3g} px", flush=True)
    assert e <= FLOW_TOL, (name, e)
    return o_lr, o_rl


def check_blend(plan, name, L, R, axis, op, o_lr, o_rl):
    f_lr, f_rl = o_lr.astype(np.float32), o_rl.astype(np.float32)
    F8, Ff = plan.blend_asymmetric(dev(L), dev(R), dev(f_lr), dev(f_rl), axis=axis, f32=True)
    torch.cuda.synchronize()
    oF, o8 = oracle.blend(L, R, f_lr, f_rl, axis=axis, params=op)
    Ff, F8 = Ff.cpu().numpy(), F8.cpu().numpy()
    e = np.abs(Ff - oF).max()
    assert e <= F_TOL, (name, e)
    safe = np.abs(oF - np.floor(oF) - 0.5) > F_TOL
    assert np.array_equal(F8[safe], o8[safe]), name
    assert np.abs(F8.astype(int) - o8.astype(int)).max() <= 1, name
