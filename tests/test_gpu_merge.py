"""Repeated pairwise merging of a photo set (ring left to right, then the
top photo) on the GPU: the native scheduler equals the same steps issued
one call at a time, bit for bit; and along the oracle's own merge, every
step's box, flows and composite match the oracle's on that step's inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_01201_amd import synth

pytestmark = pytest.mark.gpu

F_TOL = 0.5 / 255.0


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_01201_amd import api as _api

    return _api


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _photos(seed, H, W, n_ring, closed=False):
    return [(dev(i), dev(m), ax, sd)
            for i, m, ax, sd in synth.make_panorama_photos(seed, H, W, n_ring=n_ring, closed=closed)]


def _crop(img, box):
    # the box's crop; on a periodic canvas its columns wrap modulo W
    bx, by, bw, bh = box
    W = img.shape[1]
    if bx + bw <= W:
        return img[by:by + bh, bx:bx + bw]
    cols = (bx + np.arange(bw)) % W
    if isinstance(img, np.ndarray):
        return np.ascontiguousarray(img[by:by + bh][:, cols])
    return img[by:by + bh][:, torch.from_numpy(cols).to(img.device)].contiguous()


def _stepwise(plan, photos, periodic=False):
    """The merge issued call by call: returns the states after every step
    and the flows of every step."""
    img0, m0 = photos[0][0], photos[0][1]
    acc = img0 * (m0 > 0)[..., None]
    cov = (m0 > 0).to(torch.uint8)
    states, flows, boxes = [(acc.clone(), cov.clone())], [None], [(0, 0, 0, 0)]
    for img, m, axis, side in photos[1:]:
        L, R, mL, mR = (acc, img, cov, m) if side == 0 else (img, acc, m, cov)
        box = plan.overlap_box(mL, mR, periodic=periodic)
        bx, by, bw, bh = box
        flr = frl = None
        if bw > 0 and bh > 0:
            flr, frl = plan.flow_bidirectional(_crop(L, box), _crop(R, box))
        acc = plan.composite_canvas(L, R, mL, mR, flr, frl, box, axis=axis, periodic=periodic)
        cov = torch.maximum(cov, (m > 0).to(torch.uint8))
        states.append((acc.clone(), cov.clone()))
        flows.append((flr, frl))
        boxes.append(box)
    torch.cuda.synchronize()
    return states, flows, boxes


@pytest.mark.parametrize("n_ring", [2, 3])
def test_merge_equals_stepwise_calls(api, n_ring):
    H, W = 160, 120 * n_ring
    photos = _photos(n_ring, H, W, n_ring)
    plan = api.Plan(api.Params(levels=3), max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    print(f"[gpu] merge {n_ring} ring photos + top, {H}x{W}", flush=True)
    canvas, cov, boxes = plan.merge_photos(photos)
    torch.cuda.synchronize()
    states, _, sboxes = _stepwise(plan, photos)
    assert boxes == sboxes
    assert torch.equal(canvas, states[-1][0])
    assert torch.equal(cov, states[-1][1])
    assert int(cov.min()) == 1  # the set covers the canvas


def test_merge_steps_match_oracle(api):
    # the oracle merges the set on its own (its boxes, flows and canvases);
    # every GPU step is then checked on the oracle's inputs of that step:
    # box exact, flows within 1e-2 px, the composite of the oracle's flows
    # within 0.5/255, the coverage exact
    H, W, n_ring = 150, 330, 3
    photos_np = synth.make_panorama_photos(7, H, W, n_ring=n_ring)
    p = api.Params(levels=3)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    print("[gpu] merge steps vs oracle", flush=True)
    op = oracle.Params(levels=3)
    acc = photos_np[0][0] * (photos_np[0][1] > 0)[..., None]
    cov = (photos_np[0][1] > 0).astype(np.uint8)
    for i in range(1, len(photos_np)):
        img, m, axis, side = photos_np[i]
        L, R, mL, mR = (acc, img, cov, m) if side == 0 else (img, acc, m, cov)
        box = oracle.overlap_box(mL, mR)
        assert plan.overlap_box(dev(mL), dev(mR)) == box
        bx, by, bw, bh = box
        o_lr, o_rl = oracle.flow_bidirectional(L[by:by + bh, bx:bx + bw], R[by:by + bh, bx:bx + bw], op)
        g_lr, g_rl = plan.flow_bidirectional(dev(L[by:by + bh, bx:bx + bw]), dev(R[by:by + bh, bx:bx + bw]))
        assert np.abs(g_lr.cpu().numpy() - o_lr).max() <= 1e-2 and np.abs(g_rl.cpu().numpy() - o_rl).max() <= 1e-2
        f_lr, f_rl = o_lr.astype(np.float32), o_rl.astype(np.float32)
        F8, Ff = plan.composite_canvas(dev(L), dev(R), dev(mL), dev(mR), dev(f_lr), dev(f_rl), box, axis=axis,
                                       f32=True)
        torch.cuda.synchronize()
        oF, o8 = oracle.composite(L, R, mL, mR, f_lr, f_rl, box, axis=axis, params=op)
        assert np.abs(Ff.cpu().numpy() - oF).max() <= F_TOL
        g8 = F8.cpu().numpy()
        safe = np.abs(oF - np.floor(oF) - 0.5) > F_TOL
        assert np.array_equal(g8[safe], o8[safe]), i
        assert np.abs(g8.astype(int) - o8.astype(int)).max() <= 1
        acc = o8
        cov = np.maximum(cov, (m > 0).astype(np.uint8))


def test_merge_box_beyond_plan_limits(api):
    H, W = 120, 240
    photos = _photos(3, H, W, 2)
    plan = api.Plan(api.Params(levels=3), max_strips=1, max_H=16, max_W=16, canvas=(H, W))
    with pytest.raises(ValueError):
        plan.merge_photos(photos)


def test_merge_is_bitwise_repeatable(api):
    H, W = 140, 300
    photos = _photos(5, H, W, 3)
    plan = api.Plan(api.Params(levels=3), max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    print("[gpu] merge twice", flush=True)
    a, ca, ba = plan.merge_photos(photos)
    a = a.clone()
    ca = ca.clone()
    b, cb, bb = plan.merge_photos(photos)
    torch.cuda.synchronize()
    assert ba == bb and torch.equal(a, b) and torch.equal(ca, cb)


def test_merge_with_a_disjoint_photo(api):
    # photo 1 does not touch the canvas merged so far (empty overlap box:
    # no flows, Area1 and Area2 copied); photo 2 overlaps both
    H, W = 100, 240
    imgs = synth.make_panorama_photos(11, H, W, n_ring=3)
    spans = [(0, 100), (140, 240), (60, 180)]
    photos = []
    for (img, _, _, _), (a, b) in zip(imgs, spans):
        m = np.zeros((H, W), np.uint8)
        m[:, a:b] = 1
        photos.append((dev(img), dev(m), 0, 0))
    plan = api.Plan(api.Params(levels=3), max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    print("[gpu] merge with a disjoint photo", flush=True)
    canvas, cov, boxes = plan.merge_photos(photos)
    torch.cuda.synchronize()
    assert boxes[1] == (0, 0, 0, 0) and boxes[2][2] > 0
    states, _, sboxes = _stepwise(plan, photos)
    assert boxes == sboxes
    assert torch.equal(canvas, states[-1][0]) and torch.equal(cov, states[-1][1])
    # after the disjoint step the canvas is each photo on its own span
    acc1 = states[1][0].cpu().numpy()
    assert np.array_equal(acc1[:, 140:], imgs[1][0][:, 140:]) and np.array_equal(acc1[:, :100], imgs[0][0][:, :100])
    assert (acc1[:, 100:140] == 0).all()


# ----------------------------------------------------------------------------
# A closed 360-degree ring: the last ring photo overlaps the first across the
# canvas wrap and closes the ring in its step


def test_closed_ring_merge_equals_stepwise_calls(api):
    H, W, n_ring = 150, 480, 4
    photos = _photos(2, H, W, n_ring, closed=True)
    plan = api.Plan(api.Params(levels=3), max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    print(f"[gpu] closed ring merge {n_ring} photos + top, {H}x{W}", flush=True)
    canvas, cov, boxes = plan.merge_photos(photos, periodic=True)
    torch.cuda.synchronize()
    states, _, sboxes = _stepwise(plan, photos, periodic=True)
    assert boxes == sboxes
    bx, _, bw, _ = boxes[n_ring - 1]
    assert bx + bw > W  # the closing step's box runs over the wrap
    assert torch.equal(canvas, states[-1][0])
    assert torch.equal(cov, states[-1][1])
    assert int(cov.min()) == 1


def test_closed_ring_steps_match_oracle(api):
    # as test_merge_steps_match_oracle, on the periodic canvas
    H, W, n_ring = 120, 360, 3
    photos_np = synth.make_panorama_photos(5, H, W, n_ring=n_ring, closed=True)
    p = api.Params(levels=3)
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    print("[gpu] closed ring steps vs oracle", flush=True)
    op = oracle.Params(levels=3)
    acc = photos_np[0][0] * (photos_np[0][1] > 0)[..., None]
    cov = (photos_np[0][1] > 0).astype(np.uint8)
    wrapped = 0
    for i in range(1, len(photos_np)):
        img, m, axis, side = photos_np[i]
        L, R, mL, mR = (acc, img, cov, m) if side == 0 else (img, acc, m, cov)
        box = oracle.overlap_box(mL, mR, periodic=True)
        assert plan.overlap_box(dev(mL), dev(mR), periodic=True) == box
        wrapped += box[0] + box[2] > W
        Lc, Rc = _crop(L, box), _crop(R, box)
        o_lr, o_rl = oracle.flow_bidirectional(Lc, Rc, op)
        g_lr, g_rl = plan.flow_bidirectional(dev(Lc), dev(Rc))
        assert np.abs(g_lr.cpu().numpy() - o_lr).max() <= 1e-2 and np.abs(g_rl.cpu().numpy() - o_rl).max() <= 1e-2
        f_lr, f_rl = o_lr.astype(np.float32), o_rl.astype(np.float32)
        F8, Ff = plan.composite_canvas(dev(L), dev(R), dev(mL), dev(mR), dev(f_lr), dev(f_rl), box, axis=axis,
                                       f32=True, periodic=True)
        torch.cuda.synchronize()
        oF, o8 = oracle.composite(L, R, mL, mR, f_lr, f_rl, box, axis=axis, params=op, periodic=True)
        assert np.abs(Ff.cpu().numpy() - oF).max() <= F_TOL
        g8 = F8.cpu().numpy()
        safe = np.abs(oF - np.floor(oF) - 0.5) > F_TOL
        assert np.array_equal(g8[safe], o8[safe]), i
        assert np.abs(g8.astype(int) - o8.astype(int)).max() <= 1
        acc = o8
        cov = np.maximum(cov, (m > 0).astype(np.uint8))
    assert wrapped == 1 and cov.min() == 1


def test_photo_set_stream_through_one_plan(api):
    # several photo sets (plain and closed rings of different sizes) merged
    # one after another through one plan on one stream: each equals its
    # merge through a fresh plan
    H, W = 140, 400
    plan = api.Plan(api.Params(levels=3), max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    sets = [(3, False), (4, True), (5, False), (2, True)]
    outs = []
    print("[gpu] photo-set stream", flush=True)
    for k, (n_ring, closed) in enumerate(sets):
        outs.append(plan.merge_photos(_photos(20 + k, H, W, n_ring, closed=closed), periodic=closed))
    torch.cuda.synchronize()
    for k, (n_ring, closed) in enumerate(sets):
        fresh = api.Plan(api.Params(levels=3), max_strips=1, max_H=H, max_W=W, canvas=(H, W))
        canvas, cov, boxes = fresh.merge_photos(_photos(20 + k, H, W, n_ring, closed=closed), periodic=closed)
        torch.cuda.synchronize()
        assert torch.equal(canvas, outs[k][0]) and torch.equal(cov, outs[k][1]) and boxes == outs[k][2]
