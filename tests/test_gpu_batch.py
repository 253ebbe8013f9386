"""Batched stitching (one launch per level and stage over all strips,
hipGraph replay, autotuned launch shapes) against the per-strip calls, and
run-to-run determinism."""
import numpy as np
import pytest
import torch

from paper_2006_01201_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_01201_amd import api as _api

    return _api


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_strips():
    # uneven sizes, both seam orientations, one with a user Blend array
    specs = [(1, 96, 130, 0), (2, 57, 61, 0), (3, 40, 210, 1), (4, 128, 77, 0), (5, 9, 33, 0)]
    out = []
    for seed, H, W, axis in specs:
        s = synth.make_random(seed, H, W, axis=axis, max_ux=6, max_uy=2, occluder=(seed == 4))
        out.append((_dev(s.L), _dev(s.R), axis))
    b = synth.rng_for(130, 0, 0).uniform(0, 1, (57, 61)).astype(np.float32)
    out[1] = (*out[1], _dev(b))
    return out


def plain(plan, strips):
    res = []
    for s in strips:
        flr, frl = plan.flow_bidirectional(s[0], s[1])
        F, Ff = plan.blend_asymmetric(s[0], s[1], flr, frl, blend=s[3] if len(s) > 3 else None, axis=s[2], f32=True)
        res.append({"flow_lr": flr, "flow_rl": frl, "F": F, "F_f32": Ff})
    torch.cuda.synchronize()
    return res


def same(a, b):
    for x, y in zip(a, b):
        for k in ("flow_lr", "flow_rl", "F", "F_f32"):
            if x[k] is None or y[k] is None:
                continue
            assert torch.equal(x[k].view(torch.uint8) if x[k].dtype == torch.float32 else x[k],
                               y[k].view(torch.uint8) if y[k].dtype == torch.float32 else y[k]), k


def test_batched_equals_plain(api):
    strips = make_strips()
    p = api.Params(levels=4)
    plan = api.Plan(p, max_strips=8, max_H=256, max_W=256)
    print("[gpu] batched vs plain", flush=True)
    ref = plain(plan, strips)
    for use_graph in (False, True):
        out = plan.stitch_strips(strips, use_graph=use_graph, f32=True)
        torch.cuda.synchronize()
        same(ref, out)


def test_graph_replay_with_new_tensors(api):
    p = api.Params(levels=4)
    plan = api.Plan(p, max_strips=8, max_H=256, max_W=256)
    s1 = make_strips()
    b1 = plan.make_batch(s1, f32=True)
    print("[gpu] graph replay", flush=True)
    first = [{k: (v.clone() if v is not None else None) for k, v in o.items()} for o in plan.stitch(b1, True)]
    eager = plain(plan, s1)
    same(eager, first)
    for rep in range(3):
        # fresh input tensors of the same shapes (different contents) and
        # fresh outputs; plain work between replays
        s2 = [(torch.flip(s[1], [0]).contiguous(), torch.flip(s[0], [0]).contiguous(), *s[2:]) for s in s1]
        b2 = plan.make_batch(s2, f32=True)
        out = plan.stitch(b2, True)
        torch.cuda.synchronize()
        same(plain(plan, s2), out)
        again = plan.stitch(b1, True)
        torch.cuda.synchronize()
        same(first, again)


def test_shape_change_recaptures(api):
    p = api.Params(levels=3)
    plan = api.Plan(p, max_strips=8, max_H=256, max_W=256)
    s1 = make_strips()
    print("[gpu] recapture", flush=True)
    a = plan.stitch_strips(s1[:3], use_graph=True)
    b = plan.stitch_strips(s1[1:], use_graph=True)
    torch.cuda.synchronize()
    same(plain(plan, s1[:3]), a)
    same(plain(plan, s1[1:]), b)


def test_every_launch_shape_gives_identical_results(api):
    strips = make_strips()
    p = api.Params(levels=4)
    plan = api.Plan(p, max_strips=8, max_H=256, max_W=256)
    print("[gpu] launch shape invariance", flush=True)
    ref = plan.stitch_strips(strips, use_graph=False, f32=True)
    torch.cuda.synchronize()
    ths = {2: (1, 2, 4, 8), 3: (8, 10, 12, 16, 32), 4: (2, 4), 5: (1, 2, 4)}
    for stage in range(6):
        for th in ths.get(stage, (4,)):
            for grid in (0, 1, 3):
                for c in range(4):
                    plan.set_launch(stage, c, th, grid)
                out = plan.stitch_strips(strips, use_graph=False, f32=True)
                torch.cuda.synchronize()
                same(ref, out)
        for c in range(4):
            plan.set_launch(stage, c, ths.get(stage, (4,))[0], 0)


def test_autotune_keeps_results(api, tmp_path, monkeypatch):
    monkeypatch.setenv("ABF_TUNE_CACHE", str(tmp_path / "tune.json"))
    strips = make_strips()
    p = api.Params(levels=4)
    plan = api.Plan(p, max_strips=8, max_H=256, max_W=256)
    print("[gpu] autotune", flush=True)
    ref = plan.stitch_strips(strips, use_graph=False, f32=True)
    b = plan.make_batch(strips, f32=True)
    plan.tune(b)
    out = plan.stitch(b, use_graph=True)
    torch.cuda.synchronize()
    same(ref, out)
    text = (tmp_path / "tune.json").read_text()
    assert text.startswith('{"arch": "gfx950')
    # a new plan reads the cache back
    plan2 = api.Plan(p, max_strips=8, max_H=256, max_W=256)
    for st in range(6):
        for c in range(4):
            assert plan2.get_launch(st, c) == plan.get_launch(st, c)


def test_runs_are_bitwise_deterministic(api):
    strips = make_strips()
    p = api.Params(levels=4)
    plan = api.Plan(p, max_strips=8, max_H=256, max_W=256)
    print("[gpu] determinism", flush=True)
    a = plan.stitch_strips(strips, use_graph=False, f32=True)
    b = plan.stitch_strips(strips, use_graph=False, f32=True)
    torch.cuda.synchronize()
    same(a, b)
