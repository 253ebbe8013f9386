"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the 9000x4000 panorama (6 side strips 4000 x 480..960
and the 600 x 9000 top seam, 23 Mpx, 6 pyramid levels) as one batch with
autotuned launch shapes and hipGraph replay, and the single 4000 x 768
strip with the per-strip calls. The oracle runs the whole path on every
strip, so nothing is sampled: every luma level, raw search and
propagated + median flow at every level bit for bit, the refined flows
within 1e-2 px at every pixel, and the blend kernel at these sizes on the
oracle's flows within 0.5/255."""
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


def test_full_panorama_batched(api, tmp_path, monkeypatch):
    monkeypatch.setenv("ABF_TUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = 2
    shapes = synth.strip_shapes(cfg, 0)
    total = sum(h * w for h, w, _ in shapes)
    print(f"[gpu] full panorama: {len(shapes)} strips, {total / 1e6:.2f} Mpx, generating", flush=True)
    strips = synth.make_config(cfg, 0)
    p = api.Params(levels=synth.LEVELS[cfg])
    op = o_params(p)
    plan = api.Plan(p, max_strips=len(shapes), max_pixels=total, max_H=max(h for h, _, _ in shapes),
                    max_W=max(w for _, w, _ in shapes))
    batch = plan.make_batch([(dev(s.L), dev(s.R), s.axis) for s in strips])
    print("[gpu] full panorama: tune + batched graph replay", flush=True)
    plan.tune(batch)
    out = plan.stitch(batch, use_graph=True)
    torch.cuda.synchronize()
    gpu = []
    for i in range(len(strips)):
        gpu.append((gpu_levels(plan, i, p.levels), out[i]["flow_lr"].cpu().numpy(),
                    out[i]["flow_rl"].cpu().numpy(), out[i]["F"].cpu().numpy()))
    for i, s in enumerate(strips):
        views, g_lr, g_rl, g_F = gpu[i]
        name = f"strip {i} {s.L.shape[0]}x{s.L.shape[1]} axis {s.axis}"
        o_lr, o_rl = check_flows(name, s.L, s.R, op, views, g_lr, g_rl)
        # the batch's composite is the blend kernel's on the batch's flows
        F8 = plan.blend_asymmetric(dev(s.L), dev(s.R), dev(g_lr), dev(g_rl), axis=s.axis)
        torch.cuda.synchronize()
        assert np.array_equal(F8.cpu().numpy(), g_F), name
        check_blend(plan, name, s.L, s.R, s.axis, op, o_lr, o_rl)
        gpu[i] = None


def test_full_single_strip(api):
    s = synth.make_config_strip(1, 0, 0)
    H, W = s.L.shape[:2]
    p = api.Params(levels=synth.LEVELS[1])
    op = o_params(p)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W)
    print(f"[gpu] full strip {H}x{W}", flush=True)
    flr, frl = plan.flow_bidirectional(dev(s.L), dev(s.R))
    torch.cuda.synchronize()
    views = gpu_levels(plan, 0, p.levels)
    o_lr, o_rl = check_flows(f"strip {H}x{W}", s.L, s.R, op, views, flr.cpu().numpy(), frl.cpu().numpy())
    check_blend(plan, f"strip {H}x{W}", s.L, s.R, s.axis, op, o_lr, o_rl)
