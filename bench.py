#!/usr/bin/env python3
"""Benchmark: overlap Mpix/s and ms per 9000 x 4000 panorama for
bidirectional flow + asymmetric blend, batched vs plain, on one MI355X.

Workload: one synthetic panorama (6 side strips 4000 x U{480..960} plus a
600 x 9000 top seam, 6 pyramid levels, exposure step on: the strips carry
a residual gain), inputs resident in HBM before the timed region. One step
= flow in both directions + Code 1 blend for every strip of the panorama:
  - batched (the reported value): one abf_stitch_strips hipGraph replay;
  - plain: per-strip abf_flow_bidirectional + abf_blend_asymmetric calls.
Also reported: per-replay median and p10/p90, the HBM fraction of the whole
path (algorithmic bytes of the path over the step time), endpoint error
against the generator's ground truth, the "lean" parameter preset, the
per-launch times (HIP events) and the roofline of the dominant kernel, the
2048 x 512 float strip refined by 50 descent steps from the search's flow,
the 32-panorama stream with 20 batched descent steps per strip, the single
strips of 256 x 64 and 4000 x 768, the classic Lucas-Kanade pyramid, canvas
compositing and photo-set merging, and the CPU oracle timed on a bounded
sample of the same workload (plus single-thread and per-strip timings).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "overlap Mpix/s and ms per 9000x4000 panorama (flow+blend), batched vs plain"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 64 lanes x 2.4 GHz = 39.3 T 32-bit lane-ops/s; v_sad_u8 does 4
# byte absolute differences per lane-op
AD_PEAK_TOPS = 256 * 64 * 2.4e9 * 4 / 1e12
FP32_PEAK_TFLOPS = 157.3
STAGES = ("luma", "pyramid", "search", "propagation", "refine", "blend")
KERNELS = ("k_luma", "k_pyr", "k_search", "k_prop", "k_refine", "k_blend")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def level_sizes(H, W, N):
    out = []
    for _ in range(N):
        out.append((H, W))
        H, W = (H + 1) // 2, (W + 1) // 2
    return out


def kernel_name(stage, level, p):
    if stage == 0:
        return "k_luma level 0" if level == 0 else "k_gain_prep + k_gain level 0"
    if stage == 4:
        if level != 0:
            return "k_refine_border level 0"
        return "k_refine_pair level 0" if p.lk_patch <= 2 else "k_refine level 0"
    if stage == 3:
        return f"k_prop ({p.prop_steps} steps + median) level {level}"
    return f"{KERNELS[stage]} level {level}"


def algorithmic(stage, level, shapes, p):
    """(bound, amount per launch, unit, peak) of one launch (of the
    launches of a stage and level, for the propagation)."""
    px = sum(lh * lw for (H, W, _) in shapes for (lh, lw) in [level_sizes(H, W, p.levels)[level]])
    win = (2 * p.patch + 1) ** 2
    if stage == 0 and level == 1:  # exposure step: R's level-0 plane read and written
        px0 = sum(H * W for (H, W, _) in shapes)
        return "hbm", px0 * 2.0, "GB/s", HBM_PEAK_GBS
    if stage == 0:  # RGB of L and R in, two luma planes out
        return "hbm", px * 8.0, "GB/s", HBM_PEAK_GBS
    if stage == 1:  # two finer planes in (4 px per output), two planes out
        return "hbm", px * 2 * 5.0, "GB/s", HBM_PEAK_GBS
    if stage == 2:  # absolute differences: 2 directions x candidates x patch
        r = p.radius_coarse if level == p.levels - 1 else p.radius
        return "alu", 2.0 * px * (2 * r + 1) ** 2 * win, "TOP/s", AD_PEAK_TOPS
    if stage == 3:  # T steps x 4 neighbour candidates x patch, both directions
        return "alu", 2.0 * px * p.prop_steps * 4 * win, "TOP/s", AD_PEAK_TOPS
    if stage == 4:  # per window sample and iteration: 3 lerps (6), residual (1), 2 FMAs (4)
        wn = (2 * p.lk_patch + 1) ** 2
        lp = p.lk_patch
        # level-0 pixels whose window lies inside the strip (interior launch)
        # or not (border launch, reported in the level-1 slot)
        inner = sum(max(H - 2 * lp, 0) * max(W - 2 * lp, 0) for (H, W, _) in shapes)
        px = inner if level == 0 else sum(H * W for (H, W, _) in shapes) - inner
        return "alu", 2.0 * px * p.lk_iters * wn * 11, "TFLOP/s", FP32_PEAK_TFLOPS
    # blend: L, R (6 B) and two float2 flows (16 B) in, F (3 B) out
    return "hbm", px * 25.0, "GB/s", HBM_PEAK_GBS


def run_stream(n_pano, p, timed, log):
    """The cfg4 stream: n_pano panoramas of 7 strips of drawn sizes; flow +
    blend batched per chunk of 4 panoramas (graph replays), then 20
    descent steps on every strip's FlowRtoL, batched per chunk. Inputs
    (uint8 and their float copies) are generated on the GPU beforehand."""
    import torch

    from paper_2006_01201_amd import api, synth

    chunk = 4
    t0 = time.time()
    panos = []
    for k in range(n_pano):
        panos.append([synth.make_config_strip_device(4, k, s) for s in range(7)])
        torch.cuda.synchronize()
        log(f"stream: panorama {k} generated ({time.time() - t0:.1f} s)")
    floats = [[(R.float().div_(255.0), L.float().div_(255.0)) for (L, R, _) in pano] for pano in panos]
    torch.cuda.synchronize()
    total_px = sum(L.shape[0] * L.shape[1] for pano in panos for (L, _, _) in pano)
    log(f"stream: {n_pano} panoramas, {total_px / 1e6:.1f} Mpx generated in {time.time() - t0:.1f} s")
    groups = [sum(panos[i:i + chunk], []) for i in range(0, n_pano, chunk)]
    fgroups = [sum(floats[i:i + chunk], []) for i in range(0, n_pano, chunk)]
    max_px = max(sum(L.shape[0] * L.shape[1] for (L, _, _) in g) for g in groups)
    plan = api.Plan(p, max_strips=7 * chunk, max_pixels=max_px, max_H=4000, max_W=9000)
    batches = [plan.make_batch(g) for g in groups]
    items = [[(ref, tgt, b.outputs[i]["flow_rl"]) for i, (ref, tgt) in enumerate(fg)] for b, fg in zip(batches, fgroups)]

    def flows():
        for b in batches:
            plan.stitch(b, use_graph=True)

    def refine():
        for it in items:
            plan.refine_strips(it, steps=20)

    flows()  # captures one graph per chunk shape
    ms_f, _ = timed(flows, 2)
    ms_r, _ = timed(refine, 1)
    log(f"stream: flow + blend {ms_f:.2f} ms, 20 refinement steps {ms_r:.2f} ms")
    return {"workload": f"{n_pano} panoramas (cfg4) x 7 strips, sizes drawn per panorama, 6 levels",
            "overlap_mpix": round(total_px / 1e6, 2), "ms_flow_blend": round(ms_f, 3),
            "mpix_s_flow_blend": round(total_px / ms_f / 1e3, 1), "ms_refine_20_steps": round(ms_r, 3),
            "mpix_s_with_refine": round(total_px / (ms_f + ms_r) / 1e3, 1)}


def run_canvas(p, timed, log, steps):
    """Canvas compositing of one photo pair: a 4000 x 2400 canvas with two
    side photos (overlap ~0.3 W with slanted, bowed edges, two Area1
    islands inside it). One step = overlap box, both flows on the box
    crops, eq. (1) over the canvas, Code 1 over the canvas."""
    import numpy as np
    import torch

    from paper_2006_01201_amd import api, synth

    t0 = time.time()
    c = synth.make_canvas(0, 4000, 2400, holes=2)
    H, W = c.mask_L.shape
    L, R = torch.from_numpy(c.L).cuda(), torch.from_numpy(c.R).cuda()
    mL, mR = torch.from_numpy(c.mask_L).cuda(), torch.from_numpy(c.mask_R).cuda()
    a = (c.mask_L > 0).astype(np.int64) + 2 * (c.mask_R > 0)
    counts = [int((a == k).sum()) for k in range(4)]
    log(f"canvas: {H} x {W} generated in {time.time() - t0:.1f} s, areas (none, 1, 2, 3) = {counts}")
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W, canvas=(H, W))
    box = plan.overlap_box(mL, mR)
    bx, by, bw, bh = box
    n3 = int((a[by:by + bh, bx:bx + bw] == 3).sum())
    Lc, Rc = L[by:by + bh, bx:bx + bw], R[by:by + bh, bx:bx + bw]
    flr = torch.empty((bh, bw, 2), device="cuda")
    frl = torch.empty((bh, bw, 2), device="cuda")
    B = torch.empty((H, W), device="cuda")
    F = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")
    dbox = torch.empty(4, dtype=torch.int32, device="cuda")
    parts = {
        "overlap_box": lambda: plan.overlap_box(mL, mR, out=dbox),
        "flow_both_ways": lambda: plan.flow_bidirectional(Lc, Rc, out=(flr, frl)),
        "eq1_blend_map": lambda: plan.canvas_blend(mL, mR, out=B),
        "code1_composite": lambda: plan.composite_canvas(L, R, mL, mR, flr, frl, box, blend=B, out=F),
    }
    for fn in parts.values():
        fn()
    ms = {k: timed(fn, steps)[0] for k, fn in parts.items()}
    total = sum(ms.values())
    npx = H * W
    # algorithmic bytes: masks in, row distances out (row pass), row
    # distances in (block minima), masks + row distances in and Blend out
    # (search); masks in, one image in on Area1 / Area2, both images +
    # Blend + two float2 flows on Area3, F out (composite)
    b_map = npx * (2 + 4) + npx * 4 + npx * (2 + 4 + 4)
    b_comp = npx * (2 + 3) + 3 * (counts[1] + counts[2]) + (6 + 4 + 16) * n3
    roof = {k: {"bound": "hbm", "ms": round(ms[k], 4), "bytes": b,
                "achieved": round(b / ms[k] / 1e6, 1), "unit": "GB/s", "frac": round(b / ms[k] / 1e6 / HBM_PEAK_GBS, 4)}
            for k, b in (("eq1_blend_map", b_map), ("code1_composite", b_comp))}
    log(f"canvas: {total:.3f} ms per canvas ({', '.join(f'{k} {v:.3f}' for k, v in ms.items())})")
    return {"workload": f"{H} x {W} pair canvas (two side photos, overlap box {bw} x {bh}, Area3 {counts[3]} px "
                        f"with 2 Area1 islands), box + flows on the box + eq. (1) + Code 1",
            "canvas_mpix": round(npx / 1e6, 3), "ms_per_canvas": round(total, 4),
            "mpix_s": round(npx / total / 1e3, 1), "ms": {k: round(v, 4) for k, v in ms.items()},
            "areas_none_1_2_3": counts, "roofline": roof}


def run_lk_pyramid(dev, shapes, total_px, timed, log, steps, iters=4):
    """The panorama workload with the classic coarse-to-fine Lucas-Kanade
    (flow method 1, `iters` Gauss-Newton steps per level, double
    arithmetic) instead of the integer search, batched and replayed from a
    graph like the reported value, plus its level-0 launch against the FP64
    vector peak (per window sample and step: bilinear sample 6, residual 1,
    two products into the sums 4 flops; the normal matrix 6 per sample),
    counted over the level-0 interior pixels."""
    from paper_2006_01201_amd import api

    p = api.Params(levels=6, flow_method=1, lk_iters=iters, gain_comp=1)
    plan = api.Plan(p, max_strips=len(shapes), max_pixels=total_px, max_H=max(h for h, _, _ in shapes),
                    max_W=max(w for _, w, _ in shapes))
    batch = plan.make_batch(dev)
    plan.stitch(batch, use_graph=True)
    ms, _ = timed(lambda: plan.stitch(batch, use_graph=True), steps)
    prof = plan.profile(batch, reps=3)
    # per level: the interior launch (refinement slot) and the border
    # launch (search slot)
    lvl = [prof[2][k] + prof[4][k] for k in range(6)]
    l0 = prof[4][0]
    win = (2 * p.lk_patch + 1) ** 2
    inner = sum(max(h - 2 * p.lk_patch, 0) * max(w - 2 * p.lk_patch, 0) for h, w, _ in shapes)
    flops = 2.0 * inner * win * (6 + iters * 11)
    log(f"classic LK pyramid: {ms:.3f} ms per panorama, level 0 interior {l0:.3f} ms, border {prof[2][0]:.3f} ms")
    return {"workload": "the same panorama, flow by the classic coarse-to-fine Lucas-Kanade (6 levels, "
                        f"{iters} Gauss-Newton steps per level, 5x5 window, double) + blend, batched graph replay",
            "ms_per_panorama": round(ms, 4), "mpix_s": round(total_px / ms / 1e3, 1),
            "level_ms": [round(v, 4) for v in lvl],
            "level0_interior": {"bound": "alu", "ms": round(l0, 4), "achieved": round(flops / l0 / 1e9, 2),
                       "peak": 78.6, "unit": "TFLOP/s", "frac": round(flops / l0 / 1e9 / 78.6, 4)}}


def run_merge(p, log, reps, n_stream=3):
    """Repeated pairwise merging of photo sets on a 4000 x 9000 canvas, 6
    ring photos left to right, then the top photo (7 photos, seams of the
    ring with overlaps U[480, 960] px and a ~600-row top band), images
    generated on the GPU. One step = one whole merge (abf_merge_photos,
    which reads every overlap box back to size the flows):
      - planar: the ring does not close (the canvas does not wrap);
      - closed ring: a 360-degree panorama (periodic canvas), whose last
        ring photo closes the ring across the wrap in its step;
      - stream: n_stream closed photo sets merged one after another
        through one plan on one stream."""
    import torch

    from paper_2006_01201_amd import api, synth

    H, W = 4000, 9000
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W, max_pixels=10 << 20, canvas=(H, W))
    out = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")

    def timed_merge(photos, periodic):
        _, _, boxes = plan.merge_photos(photos, out=out, periodic=periodic)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            plan.merge_photos(photos, out=out, periodic=periodic)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, (time.perf_counter() - w0) * 1e3 / reps, boxes

    res = {}
    for closed in (False, True):
        t0 = time.time()
        photos = synth.make_panorama_photos(0, H, W, n_ring=6, device="cuda", closed=closed)
        torch.cuda.synchronize()
        log(f"merge: 7 photos on {H} x {W} generated in {time.time() - t0:.1f} s (closed ring {closed})")
        ms, wall, boxes = timed_merge(photos, closed)
        log(f"merge: {ms:.3f} ms per panorama (wall {wall:.3f}), closed ring {closed}")
        res["closed_ring" if closed else "planar"] = {
            "workload": f"{H} x {W} canvas, 7 photos (6 ring left to right + top"
                        f"{', the ring closing across the 360-degree wrap' if closed else ''}), overlap boxes "
                        f"{[list(b) for b in boxes[1:]]}, each step box + flows + eq. (1) + Code 1 over the canvas",
            "ms_per_panorama": round(ms, 3), "wall_ms_per_panorama": round(wall, 3),
            "canvas_mpix_s": round(H * W / ms / 1e3, 1)}
        del photos
    if n_stream:
        sets = []
        for k in range(n_stream):
            sets.append(synth.make_panorama_photos(1 + k, H, W, n_ring=6, device="cuda", closed=True))
        torch.cuda.synchronize()
        for ph in sets:  # warm-up: graph-free, but the first call of a shape sets up buffers
            plan.merge_photos(ph, out=out, periodic=True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record()
        for ph in sets:
            plan.merge_photos(ph, out=out, periodic=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n_stream
        wall = (time.perf_counter() - w0) * 1e3 / n_stream
        log(f"merge stream: {n_stream} closed photo sets, {ms:.3f} ms per panorama (wall {wall:.3f})")
        res["stream"] = {"workload": f"{n_stream} closed 360-degree photo sets of 7 photos on {H} x {W}, merged one "
                                     "after another through one plan on one stream",
                         "ms_per_panorama": round(ms, 3), "wall_ms_per_panorama": round(wall, 3)}
    return res


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.txt")
CSRC = os.path.join(ROOT, "paper_2006_01201_amd", "csrc")
# the sources whose change invalidates the recorded counters (kernels and
# the runtime that shapes their launches)
TRAFFIC_SOURCES = ("abf_kernels.hip", "abf_prop.hip", "abf_runtime.hip", "abf_internal.h", "abf_device.h", "abf_tiles.h")


def source_digest():
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def traffic_records():
    """Entries of the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for a copy of known
    size) whose source digest matches the sources this run uses."""
    if not os.path.exists(TRAFFIC_FILE):
        return []
    digest = source_digest()
    out = []
    for line in open(TRAFFIC_FILE):
        if line.startswith("#") or "=" not in line:
            continue
        f = dict(kv.strip().split("=", 1) for kv in line.strip().split(";") if "=" in kv)
        if f.get("source_sha256") == digest:
            out.append(f)
    return out


def measured_traffic(kernel, records):
    """HBM bytes per launch of `kernel` (None when not recorded for these
    sources)."""
    for f in records:
        if f.get("kernel") == kernel:
            return int(float(f["fetch_kib"]) * 1024 * float(f["fetch_scale"]) +
                       float(f["write_kib"]) * 1024 * float(f["write_scale"]))
    return None


def measured_step_traffic(records, workload):
    for f in records:
        if f.get("step_total") == workload:
            return int(float(f["bytes"]))
    return None


def rate(amount, ms, unit):
    s = ms / 1e3
    return amount / s / (1e9 if unit == "GB/s" else 1e12)


def path_bytes(shapes, levels):
    """Algorithmic HBM bytes of one pass of the path (flow both ways +
    blend) over strips of `shapes`: per level-0 pixel, RGB of L and R in
    (6 B), level-0 luma written and read back (4 B), two float2 flows out
    (16 B) and the blend (L, R, both flows in, F out: 25 B); per pixel of
    the coarser levels, both luma planes written and read (4 B) and both
    directions' int16x2 flows written and read (16 B). Level-0 search and
    refinement are counted as fused on chip."""
    px0 = sum(H * W for H, W, _ in shapes)
    pxc = sum(h * w for H, W, _ in shapes for (h, w) in level_sizes(H, W, levels)[1:])
    return px0 * (6 + 4 + 16 + 25) + pxc * (2 * 2 * 1 + 2 * 2 * 4)


def hbm_frac(nbytes, ms):
    return nbytes / (ms / 1e3) / (HBM_PEAK_GBS * 1e9)


def epe_stats(strips, flows, margin=8):
    """Endpoint error of both flows against the generator's ground truth
    over visible correspondences, `margin` px from the strip edges."""
    import numpy as np

    errs = []
    for s, (flr, frl) in zip(strips, flows):
        sl = (slice(margin, s.H - margin), slice(margin, s.W - margin))
        for f, gt, valid in ((frl, s.flow_rl_gt, s.valid_rl), (flr, s.flow_lr_gt, s.valid_lr)):
            e = np.hypot(f[..., 0] - gt[..., 0], f[..., 1] - gt[..., 1])[sl][valid[sl]]
            errs.append(e)
    e = np.concatenate(errs)
    return {"median_px": round(float(np.median(e)), 4), "mean_px": round(float(e.mean()), 4),
            "p90_px": round(float(np.percentile(e, 90)), 4), "frac_within_1px": round(float((e <= 1).mean()), 4),
            "pixels": int(e.size)}


def make_timers(stream):
    import torch

    def timed(fn, k):
        """Mean ms per call over k calls between one event pair (and the
        wall clock)."""
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        return e0.elapsed_time(e1) / k, (w1 - w0) * 1e3 / k

    def timed_each(fn, k):
        """Median, p10 and p90 of k calls, each between its own event pair."""
        import numpy as np

        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        t = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
        return {"median": round(float(np.median(t)), 4), "p10": round(float(np.percentile(t, 10)), 4),
                "p90": round(float(np.percentile(t, 90)), 4), "runs": k}

    return timed, timed_each


def run_lean(strips, dev, shapes, total_px, timed, timed_each, log, args):
    """The same panorama with the lean preset (3x3 patches, radius 1 (3 at
    the coarsest level), one propagation step, 3x3 refinement window, one
    Gauss-Newton step), batched graph replay."""
    from paper_2006_01201_amd import api

    p = api.Params.lean(levels=6, gain_comp=1)
    plan = api.Plan(p, max_strips=len(shapes), max_pixels=total_px, max_H=max(h for h, _, _ in shapes),
                    max_W=max(w for _, w, _ in shapes))
    batch = plan.make_batch(dev)
    if not args.no_tune:
        plan.tune(batch)
    for _ in range(args.warmup):
        plan.stitch(batch, use_graph=True)
    ms, _ = timed(lambda: plan.stitch(batch, use_graph=True), args.steps)
    dist = timed_each(lambda: plan.stitch(batch, use_graph=True), 50)
    out = plan.stitch(batch, use_graph=True)
    import torch

    torch.cuda.synchronize()
    epe = epe_stats(strips, [(o["flow_lr"].cpu().numpy(), o["flow_rl"].cpu().numpy()) for o in out])
    nb = path_bytes(shapes, p.levels)
    log(f"lean preset: {ms:.3f} ms / panorama, HBM fraction {hbm_frac(nb, ms):.3f}, EPE median {epe['median_px']}")
    plan.close()
    return {"params": {k: getattr(p, k) for k in ("patch", "radius", "radius_coarse", "prop_steps", "median",
                                                   "lk_patch", "lk_iters", "lk_eps")},
            "ms_per_panorama": round(ms, 4), "ms_dist": dist, "mpix_s": round(total_px / ms / 1e3, 1),
            "hbm_frac_path": round(hbm_frac(nb, ms), 4), "epe": epe}


def run_cfg3(p6, timed, timed_each, log):
    """cfg3: the 2048 x 512 float strip. Its images quantised to uint8 go
    through the search path (6 levels, both directions); FlowRtoL then takes
    50 gradient-descent steps on the float images (Ref = R, Tgt = L).
    Endpoint error against the ground truth before and after."""
    import numpy as np
    import torch

    from paper_2006_01201_amd import api, synth

    st = synth.make_config_strip(3, 0, 0)
    H, W = st.H, st.W
    q = lambda a: np.clip(np.rint(a.astype(np.float64) * 255.0), 0, 255).astype(np.uint8)
    L8, R8 = torch.from_numpy(q(st.L)).cuda(), torch.from_numpy(q(st.R)).cuda()
    ref, tgt = torch.from_numpy(st.R).cuda(), torch.from_numpy(st.L).cuda()
    plan = api.Plan(p6, max_strips=1, max_H=H, max_W=W)
    flr, frl = plan.flow_bidirectional(L8, R8)
    ms_flow = timed_each(lambda: plan.flow_bidirectional(L8, R8, out=(flr, frl)), 20)
    u0 = frl.clone()
    u = u0.clone()
    plan.refine_flow(ref, tgt, u, steps=50)
    torch.cuda.synchronize()
    u_after = u.cpu().numpy()

    def ref50():
        u.copy_(u0)
        plan.refine_flow(ref, tgt, u, steps=50)

    ms_ref = timed_each(ref50, 10)
    strip = [st]
    before = epe_stats(strip, [(flr.cpu().numpy(), u0.cpu().numpy())])
    # FlowRtoL only (the refined direction)
    m = 8
    sl = (slice(m, H - m), slice(m, W - m))
    e0 = np.hypot(*(u0.cpu().numpy() - st.flow_rl_gt).transpose(2, 0, 1))[sl][st.valid_rl[sl]]
    e1 = np.hypot(*(u_after - st.flow_rl_gt).transpose(2, 0, 1))[sl][st.valid_rl[sl]]
    E0 = float(plan.energy(ref, tgt, u0, grads=False).item())
    E1 = float(plan.energy(ref, tgt, torch.from_numpy(u_after).cuda(), grads=False).item())
    # the multi-level energy (6 levels of a float pyramid of the images and
    # the flow): energy with all three gradients, and 20 descent steps on it
    plan.energy_ms(ref, tgt, u0, 6, grads=True)
    ms_ems = timed_each(lambda: plan.energy_ms(ref, tgt, u0, 6, grads=True), 20)

    def ms20():
        u.copy_(u0)
        plan.refine_flow_ms(ref, tgt, u, 6, steps=20)

    ms_ms20 = timed_each(ms20, 10)
    e2 = np.hypot(*(u.cpu().numpy() - st.flow_rl_gt).transpose(2, 0, 1))[sl][st.valid_rl[sl]]
    log(f"cfg3 multi-level energy: E + gradients {ms_ems['median']:.3f} ms, 20 steps {ms_ms20['median']:.3f} ms, "
        f"EPE(RtoL) median {np.median(e0):.4f} -> {np.median(e2):.4f} px")
    log(f"cfg3: search {ms_flow['median']:.3f} ms, 50 steps {ms_ref['median']:.3f} ms, EPE(RtoL) median "
        f"{np.median(e0):.4f} -> {np.median(e1):.4f} px")
    plan.close()
    return {"workload": "2048 x 512 float RGB strip (cfg3): search path on its uint8 quantisation (6 levels, both "
                        "directions), then 50 gradient-descent steps on FlowRtoL over the float images",
            "ms_search": ms_flow, "ms_50_steps": ms_ref,
            "mpix_steps_s": round(H * W * 50 / ms_ref["median"] / 1e3, 1),
            "energy_before_after": [round(E0, 3), round(E1, 3)],
            "multi_level": {"levels": 6, "ms_energy_and_gradients": ms_ems, "ms_20_steps": ms_ms20,
                            "epe_rtol_after_median_px": round(float(np.median(e2)), 4)},
            "epe_rtol_before": {"median_px": round(float(np.median(e0)), 4), "mean_px": round(float(e0.mean()), 4)},
            "epe_rtol_after": {"median_px": round(float(np.median(e1)), 4), "mean_px": round(float(e1.mean()), 4)},
            "epe_both_search": before}


def run_single_strips(timed_each, log):
    """cfg0 (256 x 64, 3 levels) and cfg1 (4000 x 768, 6 levels): one strip
    each, plain calls (flow both ways + blend), per-call events."""
    import torch

    from paper_2006_01201_amd import api, synth

    out = {}
    for cfg in (0, 1):
        st = synth.make_config_strip(cfg, 0, 0)
        p = api.Params(levels=synth.LEVELS[cfg])
        plan = api.Plan(p, max_strips=1, max_H=st.H, max_W=st.W)
        L, R = torch.from_numpy(st.L).cuda(), torch.from_numpy(st.R).cuda()
        flr, frl = plan.flow_bidirectional(L, R)
        F = plan.blend_asymmetric(L, R, flr, frl, axis=st.axis)

        def step():
            plan.flow_bidirectional(L, R, out=(flr, frl))
            plan.blend_asymmetric(L, R, flr, frl, axis=st.axis, out=F)

        for _ in range(3):
            step()
        d = timed_each(step, 50)
        torch.cuda.synchronize()
        epe = epe_stats([st], [(flr.cpu().numpy(), frl.cpu().numpy())], margin=4 if cfg == 0 else 8)
        out[f"cfg{cfg}"] = {"strip": [st.H, st.W], "levels": p.levels, "ms_per_strip": d,
                            "mpix_s": round(st.H * st.W / d["median"] / 1e3, 2), "epe": epe}
        log(f"cfg{cfg} strip: {d['median']:.4f} ms, EPE median {epe['median_px']}")
        plan.close()
    return out


def run_cpu(strips, args, log):
    """The oracle on the host: the bounded sample of the panorama's side
    strips (the reported cpu_baseline), and, unless skipped, per-strip
    timings of cfg0 and cfg1 with one thread and with all, the whole
    panorama with all threads, and descent steps on the cfg3 strip."""
    import numpy as np

    import oracle

    op = oracle.Params(levels=6, gain_comp=1)
    n_all = oracle.num_threads()
    used, px_done, t_cpu = [], 0, 0.0
    while t_cpu < args.cpu_seconds:
        for i, s in enumerate(strips[:-1]):
            t0 = time.perf_counter()
            o_lr, o_rl = oracle.flow_bidirectional(s.L, s.R, op)
            oracle.blend(s.L, s.R, o_lr, o_rl, axis=s.axis, params=op)
            t_cpu += time.perf_counter() - t0
            px_done += s.H * s.W
            used.append(i)
            log(f"cpu oracle strip {i}: {t_cpu:.1f} s so far")
            if t_cpu >= args.cpu_seconds:
                break
    base = {"value": round(px_done / t_cpu / 1e6, 4), "unit": "Mpix/s", "cores": n_all, "kind": "oracle",
            "sample": f"side strips {used} of the same panorama, in turn ({px_done / 1e6:.2f} Mpx): flow "
                      f"both directions + Code 1 blend, C/OpenMP oracle (int32 search, FP64 refine and "
                      f"blend), {t_cpu:.1f} s"}
    if args.no_cpu_detail:
        return base, None
    from paper_2006_01201_amd import synth

    detail = {"threads_all": n_all, "host_cpu": host_cpu()}
    for cfg in (0, 1):
        st = synth.make_config_strip(cfg, 0, 0)
        o = oracle.Params(levels=synth.LEVELS[cfg])
        row = {}
        for th in (1, n_all):
            oracle.set_num_threads(th)
            t0 = time.perf_counter()
            a, b = oracle.flow_bidirectional(st.L, st.R, o)
            oracle.blend(st.L, st.R, a, b, axis=st.axis, params=o)
            row[f"ms_{th}_threads"] = round((time.perf_counter() - t0) * 1e3, 1)
        oracle.set_num_threads(n_all)
        detail[f"cfg{cfg}_strip"] = row
        log(f"cpu oracle cfg{cfg}: {row}")
    t0 = time.perf_counter()
    for s in strips:
        a, b = oracle.flow_bidirectional(s.L, s.R, op)
        oracle.blend(s.L, s.R, a, b, axis=s.axis, params=op)
    t = time.perf_counter() - t0
    px = sum(s.H * s.W for s in strips)
    detail["cfg2_panorama"] = {"ms": round(t * 1e3, 1), "mpix_s": round(px / t / 1e6, 3), "threads": n_all}
    log(f"cpu oracle panorama: {t:.1f} s")
    st = synth.make_config_strip(3, 0, 0)
    u0 = np.rint(st.flow_rl_gt).astype(np.float64)
    t0 = time.perf_counter()
    oracle.refine_gd(st.R, st.L, u0, steps=5)
    t = time.perf_counter() - t0
    detail["cfg3_descent"] = {"ms_per_step": round(t * 1e3 / 5, 1), "threads": 1,
                              "ms_50_steps_extrapolated": round(t * 1e3 * 10, 1)}
    return base, detail


def host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pano", type=int, default=0, help="panorama seed index of the workload")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-detail", action="store_true",
                    help="skip the oracle's per-strip, single-thread, whole-panorama and descent timings")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the workload, copy a MIB-mebibyte device buffer once (a kernel of known "
                         "traffic, for scaling hardware byte counters)")
    ap.add_argument("--traffic-pass", action="store_true",
                    help="run exactly one eager pass of the batched path (for hardware counters) and exit")
    ap.add_argument("--no-refine", action="store_true", help="skip the cfg3 leg (search + 50 descent steps)")
    ap.add_argument("--no-lean", action="store_true", help="skip the lean-preset leg")
    ap.add_argument("--no-strips", action="store_true", help="skip the single-strip legs (cfg0, cfg1)")
    ap.add_argument("--no-canvas", action="store_true", help="skip the canvas-compositing leg")
    ap.add_argument("--no-merge", action="store_true", help="skip the photo-set merging leg")
    ap.add_argument("--no-lk-pyramid", action="store_true", help="skip the classic Lucas-Kanade leg")
    ap.add_argument("--stream", type=int, default=32, metavar="PANORAMAS",
                    help="panoramas of the cfg4 stream (7 strips of drawn sizes each; flow + blend batched per "
                         "4 panoramas, then 20 batched refinement steps); 0 skips it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(strips shard across GPUs by design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2006_01201_amd import _abi, api, synth

    _abi.load()  # the HIP library must be there; no fallback
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        src = torch.empty(args.copy_calibration << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = src.clone()
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calibration} MiB done")
        del src, dst

    cfg = 2
    shapes = synth.strip_shapes(cfg, args.pano)
    total_px = sum(h * w for h, w, _ in shapes)
    log(f"generating workload cfg{cfg} pano {args.pano}: {len(shapes)} strips, {total_px / 1e6:.2f} Mpx")
    t0 = time.time()
    strips = synth.make_config(cfg, args.pano)
    log(f"generated in {time.time() - t0:.1f} s")
    dev = [(torch.from_numpy(s.L).cuda(), torch.from_numpy(s.R).cuda(), s.axis) for s in strips]
    torch.cuda.synchronize()

    # the panorama's strips carry an exposure gain U[0.9, 1.1]: exposure step on
    p = api.Params(levels=synth.LEVELS[cfg], gain_comp=1)
    plan = api.Plan(p, max_strips=len(shapes), max_pixels=total_px, max_H=max(h for h, _, _ in shapes),
                    max_W=max(w for _, w, _ in shapes))
    batch = plan.make_batch(dev)
    if args.traffic_pass:
        plan.stitch(batch, use_graph=False)
        torch.cuda.synchronize()
        log("traffic pass: one eager pass of the batched path done")
        return
    if not args.no_tune:
        t0 = time.time()
        plan.tune(batch)
        log(f"autotuned launch shapes in {time.time() - t0:.1f} s")

    stream = torch.cuda.current_stream()
    timed, timed_each = make_timers(stream)
    nbytes = path_bytes(shapes, p.levels)

    # batched: one graph replay per panorama
    for _ in range(args.warmup):
        plan.stitch(batch, use_graph=True)
    ms_b, wall_b = timed(lambda: plan.stitch(batch, use_graph=True), args.steps)
    dist_b = timed_each(lambda: plan.stitch(batch, use_graph=True), 50)
    log(f"batched: {ms_b:.3f} ms / panorama (wall {wall_b:.3f}); per replay median {dist_b['median']:.3f} "
        f"p10 {dist_b['p10']:.3f} p90 {dist_b['p90']:.3f}")
    out_b = plan.stitch(batch, use_graph=True)
    torch.cuda.synchronize()
    flows_b = [(o["flow_lr"].cpu().numpy(), o["flow_rl"].cpu().numpy()) for o in out_b]
    epe_b = epe_stats(strips, flows_b)
    log(f"batched EPE: {epe_b}")

    plain = None
    if not args.no_plain:
        outs = [(torch.empty((h, w, 2), device="cuda"), torch.empty((h, w, 2), device="cuda"),
                 torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")) for h, w, _ in shapes]

        def plain_step():
            for (L, R, axis), (flr, frl, F) in zip(dev, outs):
                plan.flow_bidirectional(L, R, out=(flr, frl))
                plan.blend_asymmetric(L, R, flr, frl, axis=axis, out=F)

        for _ in range(args.warmup):
            plain_step()
        ms_p, wall_p = timed(plain_step, args.steps)
        dist_p = timed_each(plain_step, 50)
        torch.cuda.synchronize()
        epe_p = epe_stats(strips, [(a.cpu().numpy(), b.cpu().numpy()) for a, b, _ in outs])
        same = all(np.array_equal(a.cpu().numpy(), fb[0]) and np.array_equal(b.cpu().numpy(), fb[1])
                   for (a, b, _), fb in zip(outs, flows_b))
        plain = {"ms_per_panorama": round(ms_p, 4), "ms_dist": dist_p, "mpix_s": round(total_px / ms_p / 1e3, 2),
                 "wall_ms_per_panorama": round(wall_p, 4), "hbm_frac_path": round(hbm_frac(nbytes, ms_p), 4),
                 "epe": epe_p, "flows_equal_batched": bool(same)}
        log(f"plain: {ms_p:.3f} ms / panorama")

    # per-launch times (eager launches bracketed by HIP events on this stream)
    prof = plan.profile(batch, reps=max(3, args.steps))
    launches = []
    for st in range(6):
        for k in range(p.levels):
            if prof[st][k] > 0:
                launches.append((prof[st][k], st, k))
    stage_ms = {STAGES[st]: round(sum(prof[st]), 4) for st in range(6)}
    dom_ms, dom_st, dom_k = max(launches)
    bound, amount, unit, peak = algorithmic(dom_st, dom_k, shapes, p)
    achieved = rate(amount, dom_ms, unit)
    records = traffic_records()
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(kernel_name(dom_st, dom_k, p), records),
                "kernel": kernel_name(dom_st, dom_k, p), "launch_ms": round(dom_ms, 4),
                "work_per_launch": amount}
    per_launch = []
    for ms, st, k in sorted(launches, reverse=True)[:8]:
        b, a, u, pk = algorithmic(st, k, shapes, p)
        per_launch.append({"kernel": kernel_name(st, k, p), "ms": round(ms, 4), "bound": b,
                           "achieved": round(rate(a, ms, u), 3), "unit": u, "frac": round(rate(a, ms, u) / pk, 4),
                           "traffic": measured_traffic(kernel_name(st, k, p), records)})
    log(f"dominant launch {roofline['kernel']}: {dom_ms:.4f} ms, {achieved:.2f} {unit} of {peak:.1f}")
    step_traffic = measured_step_traffic(records, "cfg2 panorama, one batched pass")
    path = {"bytes_alg": nbytes, "bytes_alg_per_px": round(nbytes / total_px, 2),
            "hbm_frac_path": round(hbm_frac(nbytes, ms_b), 4),
            "achieved_GBs_alg": round(nbytes / (ms_b / 1e3) / 1e9, 1),
            "counter_bytes_per_step": step_traffic,
            "counter_over_alg": round(step_traffic / nbytes, 3) if step_traffic else None}
    log(f"path: {nbytes / total_px:.2f} B/px algorithmic, HBM fraction {path['hbm_frac_path']:.4f}")

    lean = None if args.no_lean else run_lean(strips, dev, shapes, total_px, timed, timed_each, log, args)
    refine = None if args.no_refine else run_cfg3(api.Params(levels=6), timed, timed_each, log)
    single = None if args.no_strips else run_single_strips(timed_each, log)
    lkp = None
    if not args.no_lk_pyramid:
        lkp = run_lk_pyramid(dev, shapes, total_px, timed, log, max(3, args.steps // 2))
    canvas = None if args.no_canvas else run_canvas(api.Params(levels=6), timed, log, args.steps)
    merge = None if args.no_merge else run_merge(api.Params(levels=6, gain_comp=1), log, max(2, args.steps // 4))
    stream_leg = run_stream(args.stream, p, timed, log) if args.stream else None

    cpu, cpu_detail = (None, None) if args.no_cpu_baseline else run_cpu(strips, args, log)

    out = {
        "metric": METRIC,
        "value": round(total_px / ms_b / 1e3, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_b, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8+f32",
        "data": "synthetic",
        "config": {"workload": f"9000x4000 panorama (cfg2, pano {args.pano}): 6 side strips 4000 x U{{480..960}} "
                               f"+ top seam 600 x 9000, {p.levels} pyramid levels, flow both directions + blend, "
                               "exposure step on (strips carry a gain U[0.9, 1.1])",
                   "overlap_mpix": round(total_px / 1e6, 3), "strips": len(shapes),
                   "strip_shapes": [[h, w, a] for h, w, a in shapes], "mode": "batched hipGraph replay",
                   "generator": "analytic texture: 128 + 24 oriented sinusoids (amplitude U[6, 14], frequency "
                                "log-uniform [1/400, 1/5] cycles/px) + 60 additive rectangles; smooth disparity "
                                "(blurred white noise, |u_x| <= 40, |u_y| <= 8 px) with an occluding band; "
                                "noise sigma 2; seed SeedSequence([2006, 1201, 2, pano, strip])",
                   "params": "defaults: P=2 (5x5 patch), R=2, R_c=4, T=2, M=1, LK 5x5 window, 2 iterations, "
                             "eps 25, kS=10, kF=20, gain_comp=1"},
        "ms_per_panorama": {"batched": round(ms_b, 4), "plain": plain["ms_per_panorama"] if plain else None},
        "ms_dist_batched": dist_b,
        "plain": plain,
        "wall_ms_per_panorama_batched": round(wall_b, 4),
        "path": path,
        "epe": epe_b,
        "lean": lean,
        "stage_ms": stage_ms,
        "top_launches": per_launch,
        "roofline": roofline,
        "refine_flow": refine,
        "single_strips": single,
        "stream": stream_leg,
        "lk_pyramid": lkp,
        "canvas": canvas,
        "merge": merge,
        "cpu_baseline": cpu,
        "cpu_detail": cpu_detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
