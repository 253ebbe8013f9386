#!/usr/bin/env python3
"""Benchmark: overlap Mpix/s and ms per 9000 x 4000 panorama for
bidirectional flow + asymmetric blend, batched vs plain, on one MI355X.

Workload: one synthetic panorama (6 side strips 4000 x U{480..960} plus a
600 x 9000 top seam, 6 pyramid levels), inputs resident in HBM before the
timed region. One step = flow in both directions + Code 1 blend for every
strip of the panorama:
  - batched (the reported value): one abf_stitch_strips hipGraph replay;
  - plain: per-strip abf_flow_bidirectional + abf_blend_asymmetric calls.
Also reported: per-launch times (HIP events), the roofline of the dominant
kernel, and the CPU oracle timed on a bounded sample of the same workload.
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

    p = api.Params(levels=6, flow_method=1, lk_iters=iters)
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


def run_merge(p, log, reps):
    """Repeated pairwise merging of one photo set on a 4000 x 9000 canvas:
    6 ring photos left to right, then the top photo (7 photos, 6 seams of
    the ring with overlaps U[480, 960] px and a ~600-row top band), images
    generated on the GPU. One step = one whole merge (abf_merge_photos,
    which reads every overlap box back to size the flows)."""
    import torch

    from paper_2006_01201_amd import api, synth

    t0 = time.time()
    H, W = 4000, 9000
    photos = synth.make_panorama_photos(0, H, W, n_ring=6, device="cuda")
    torch.cuda.synchronize()
    log(f"merge: 7 photos on {H} x {W} generated in {time.time() - t0:.1f} s")
    plan = api.Plan(p, max_strips=1, max_H=H, max_W=W, max_pixels=8 << 20, canvas=(H, W))
    out = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")
    _, _, boxes = plan.merge_photos(photos, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(reps):
        plan.merge_photos(photos, out=out)
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) * 1e3 / reps
    ms = e0.elapsed_time(e1) / reps
    log(f"merge: {ms:.3f} ms per panorama (wall {wall:.3f})")
    return {"workload": f"{H} x {W} canvas, 7 photos (6 ring left to right + top), overlap boxes "
                        f"{[list(b) for b in boxes[1:]]}, each step box + flows + eq. (1) + Code 1 over the canvas",
            "ms_per_panorama": round(ms, 3), "wall_ms_per_panorama": round(wall, 3),
            "canvas_mpix_s": round(H * W / ms / 1e3, 1)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2006_01201_amd", "csrc", "abf_kernels.hip")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a copy of known size), or None when there is no entry or the
    kernel source has changed since the counters were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    for line in open(TRAFFIC_FILE):
        if not line.startswith("kernel="):
            continue
        f = dict(kv.strip().split("=", 1) for kv in line.strip().split(";"))
        if f["kernel"] == kernel and f["source_sha256"] == digest:
            return int(float(f["fetch_kib"]) * 1024 * float(f["fetch_scale"]) +
                       float(f["write_kib"]) * 1024 * float(f["write_scale"]))
    return None


def rate(amount, ms, unit):
    s = ms / 1e3
    return amount / s / (1e9 if unit == "GB/s" else 1e12)


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
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the workload, copy a MIB-mebibyte device buffer once (a kernel of known "
                         "traffic, for scaling hardware byte counters)")
    ap.add_argument("--refine", action="store_true",
                    help="also time 50 gradient-descent refinement steps on the 2048 x 512 float strip")
    ap.add_argument("--no-canvas", action="store_true", help="skip the canvas-compositing leg")
    ap.add_argument("--no-merge", action="store_true", help="skip the photo-set merging leg")
    ap.add_argument("--no-lk-pyramid", action="store_true", help="skip the classic Lucas-Kanade leg")
    ap.add_argument("--stream", type=int, default=0, metavar="PANORAMAS",
                    help="also time a stream of this many panoramas of the cfg4 workload (7 strips of drawn "
                         "sizes each; flow + blend batched per 4 panoramas, then 20 batched refinement steps)")
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

    p = api.Params(levels=synth.LEVELS[cfg])
    plan = api.Plan(p, max_strips=len(shapes), max_pixels=total_px, max_H=max(h for h, _, _ in shapes),
                    max_W=max(w for _, w, _ in shapes))
    batch = plan.make_batch(dev)
    if not args.no_tune:
        t0 = time.time()
        plan.tune(batch)
        log(f"autotuned launch shapes in {time.time() - t0:.1f} s")

    stream = torch.cuda.current_stream()

    def timed(fn, k):
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

    # batched: one graph replay per panorama
    for _ in range(args.warmup):
        plan.stitch(batch, use_graph=True)
    ms_b, wall_b = timed(lambda: plan.stitch(batch, use_graph=True), args.steps)
    log(f"batched: {ms_b:.3f} ms / panorama (wall {wall_b:.3f})")

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
        plain = {"ms_per_panorama": round(ms_p, 4), "mpix_s": round(total_px / ms_p / 1e3, 2),
                 "wall_ms_per_panorama": round(wall_p, 4)}
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
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(kernel_name(dom_st, dom_k, p)),
                "kernel": kernel_name(dom_st, dom_k, p), "launch_ms": round(dom_ms, 4),
                "work_per_launch": amount}
    per_launch = []
    for ms, st, k in sorted(launches, reverse=True)[:8]:
        b, a, u, pk = algorithmic(st, k, shapes, p)
        per_launch.append({"kernel": kernel_name(st, k, p), "ms": round(ms, 4), "bound": b,
                           "achieved": round(rate(a, ms, u), 3), "unit": u, "frac": round(rate(a, ms, u) / pk, 4)})
    log(f"dominant launch {roofline['kernel']}: {dom_ms:.4f} ms, {achieved:.2f} {unit} of {peak:.1f}")

    refine = None
    if args.refine:
        st3 = synth.make_config_strip(3, 0, 0)
        H3, W3 = st3.H, st3.W
        plan3 = api.Plan(p, max_strips=1, max_H=H3, max_W=W3)
        ref3 = torch.from_numpy(st3.R).cuda()
        tgt3 = torch.from_numpy(st3.L).cuda()
        u0 = torch.from_numpy(np.rint(st3.flow_rl_gt)).float().cuda()
        u = u0.clone()
        plan3.refine_flow(ref3, tgt3, u, steps=5)
        ms_r, _ = timed(lambda: (u.copy_(u0), plan3.refine_flow(ref3, tgt3, u, steps=50)), 3)
        refine = {"workload": "2048 x 512 float RGB strip, 50 gradient-descent steps (energy gradient + step, "
                              "fused per step)", "ms": round(ms_r, 4),
                  "mpix_steps_s": round(H3 * W3 * 50 / ms_r / 1e3, 1)}
        log(f"refine 50 steps: {ms_r:.3f} ms")

    lkp = None if args.no_lk_pyramid else run_lk_pyramid(dev, shapes, total_px, timed, log, max(3, args.steps // 2))
    canvas = None if args.no_canvas else run_canvas(p, timed, log, args.steps)
    merge = None if args.no_merge else run_merge(p, log, max(2, args.steps // 4))

    stream = None
    if args.stream:
        stream = run_stream(args.stream, p, timed, log)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        op = oracle.Params(levels=p.levels)
        used, px_done, t_cpu = [], 0, 0.0
        # side strips of the panorama in turn (the top seam is the one shape
        # left out), repeated until the time budget is spent
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
        cpu = {"value": round(px_done / t_cpu / 1e6, 4), "unit": "Mpix/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"side strips {used} of the same panorama, in turn ({px_done / 1e6:.2f} Mpx): flow "
                         f"both directions + Code 1 blend, C/OpenMP oracle (int32 search, FP64 refine and "
                         f"blend), {t_cpu:.1f} s"}

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
                               f"+ top seam 600 x 9000, {p.levels} pyramid levels, flow both directions + blend",
                   "overlap_mpix": round(total_px / 1e6, 3), "strips": len(shapes),
                   "strip_shapes": [[h, w, a] for h, w, a in shapes], "mode": "batched hipGraph replay"},
        "ms_per_panorama": {"batched": round(ms_b, 4), "plain": plain["ms_per_panorama"] if plain else None},
        "plain": plain,
        "wall_ms_per_panorama_batched": round(wall_b, 4),
        "stage_ms": stage_ms,
        "top_launches": per_launch,
        "roofline": roofline,
        "refine_flow": refine,
        "lk_pyramid": lkp,
        "canvas": canvas,
        "merge": merge,
        "stream": stream,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
