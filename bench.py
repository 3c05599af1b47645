#!/usr/bin/env python
"""Benchmark of the PatchMatch depth-map estimation step on one MI355X.

A step is one whole depth map: random initialisation plus 8 iterations of red/black
propagation and refinement, with outputs (depth, normal, cost) in device memory.  The
default workload is the 3200x2130 reference with 10 sources, a 31x31 window at
dilation 3 (11x11 taps), top-5 aggregation and 8 iterations, on a seeded synthetic
piecewise-planar scene; images are resident in HBM before the timed region.

Printed: one JSON line with the metric, the evaluate-and-select kernel's roofline
figures (live HIP-event timing of every launch in the timed region, algorithmic flops
from the exact number of hypotheses scored) and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per 3200×2130 depth map (10 src, 8 it); learned vs random init at equal cost"
FLOPS_PER_TAP_VIEW = 23            # algorithmic flops per (tap, view), FMA = 2
PEAK_FP32_VECTOR_TFLOPS = 157.3    # MI355X FP32 vector peak: 256 CU x 2.4 GHz x 256 flop/clk
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # the same without packed FP32: 256 CU x 2.4 GHz x 128 flop/clk


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel_file: str, profile: str):
    """HBM bytes per launch of the evaluate kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a plain-copy calibration), or None
    when the kernel source has changed since those counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        src = open(os.path.join(ROOT, "paper_2104_06165_amd", "csrc", kernel_file), "rb").read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith(" "))
    digest = fields.get("kernel_source_sha256", "").split()[0] if fields.get("kernel_source_sha256") else ""
    if digest != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse_tuning(pm, text):
    """ROWS,PERSISTENT,WGS[,ORDER_BY_DEPTH] -> the library's launch configuration (the order
    a mask: 1 initialisation, 2 propagation, 4 refinement)."""
    v = [int(x) for x in text.split(",")]
    if len(v) not in (3, 4):
        raise SystemExit("--tuning takes ROWS,PERSISTENT,WGS[,ORDER_BY_DEPTH]")
    return pm.Tuning(v[0], bool(v[1]), v[2], order_by_depth=v[3] if len(v) == 4 else 0)


def nominal_tap_views(valid_px, n_src, taps, iters):
    # 1 initial hypothesis + per iteration 8 propagation + 3 refinement candidates
    return valid_px * (1 + 11 * iters) * n_src * taps


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ctx, scene_full, solver, single_iters=1, crop=(320, 213)):
    """The oracle on the centre crop of the reference (its own problem instance, sources
    whole) at the workload's iterations: the OpenMP build of the same source on every host
    thread this process may use (at most 16; bitwise the single-threaded results), FP32 and
    FP64, plus the single-threaded FP32 build on init + `single_iters` iterations for the
    per-core rate.  `value` scales the all-thread FP32 time to one full depth map by
    nominal tap-views (extrapolated: the full map would take minutes even on every core).
    The GPU's time on the same crop problem is given beside it."""
    import torch

    import oracle
    import paper_2104_06165_amd as pm
    import scenegen as sg

    sc = sg.crop_reference(scene_full, *crop)
    pb = oracle.Problem.from_scene(sc, solver["window"], solver["dilation"], top_k=solver["top_k"],
                                   bilateral=True, sigma_s=(solver["window"] - 1) / 2.0, sigma_c=12.0,
                                   seed=sg.PM_SEED)
    iters = solver["iters"]
    R = (solver["window"] - 1) // (2 * solver["dilation"])
    taps = (2 * R + 1) ** 2
    n_src = len(sc.images) - 1
    valid = int(pb.valid_mask().sum())
    crop_tv = nominal_tap_views(valid, n_src, taps, iters)
    threads = oracle.default_threads()
    used = oracle.threads_in_effect(threads)

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    dt32 = timed(lambda: oracle.patchmatch(pb, iters, threads=threads))
    dt64 = timed(lambda: oracle.patchmatch(pb, iters, fp64=True, threads=threads))
    dt1 = timed(lambda: oracle.patchmatch(pb, single_iters))
    single_tv = nominal_tap_views(valid, n_src, taps, single_iters)
    # the GPU on the same crop problem (sources whole), outputs in device memory
    ctx.set_scene(sc)
    params = pm.Params(top_k=solver["top_k"], bilateral=True, sigma_spatial_px=(solver["window"] - 1) / 2.0,
                       seed=sg.PM_SEED)
    srcs = list(range(1, n_src + 1))
    run = lambda: ctx.patchmatch(0, srcs, solver["window"], solver["dilation"], iters, params)  # noqa: E731
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        run()
    torch.cuda.synchronize()
    gpu_crop_ms = (time.perf_counter() - t0) * 1e3 / 5
    H, W = scene_full.images[0].shape
    r = solver["dilation"] * R
    full_tv = nominal_tap_views(max(0, H - 2 * r) * max(0, W - 2 * r), n_src, taps, iters)
    return {
        "value": dt32 * 1e3 * full_tv / crop_tv,
        "unit": "ms per depth map (extrapolated from the crop)",
        "cores": used,
        "kind": "oracle",
        "sample": f"{crop[0]}x{crop[1]} centre crop of the reference (sources whole), init + {iters} iterations "
                  f"({crop_tv:.3e} nominal tap-views), FP32 oracle (OpenMP build, {used} threads): {dt32:.2f} s; "
                  f"scaled by nominal tap-views to the full {W}x{H} depth map ({full_tv:.3e})",
        "cpu_model": cpu_model(),
        "crop_seconds_fp32": dt32,
        "crop_seconds_fp64": dt64,
        "crop_tap_views_per_s_fp32": crop_tv / dt32,
        "crop_tap_views_per_s_fp64": crop_tv / dt64,
        "single_thread": {"iterations": single_iters, "seconds": dt1, "ns_per_tap_view": dt1 * 1e9 / single_tv},
        "gpu_crop_ms": gpu_crop_ms,
        "gpu_vs_cpu_on_crop": dt32 * 1e3 / gpu_crop_ms,
    }


def bench_batched(args):
    """24 references of three sizes (8 x 3200x2130, 8 x 1600x1066, 8 x 960x640), 6-12 sources
    each, from a 40-camera scene of 30 planes; all in shared launches replayed from a hipGraph,
    launch configuration picked by the autotuner; beside the same 24 depth maps run one by one."""
    import torch

    import paper_2104_06165_amd as pm
    import scenegen as sg

    log("[bench] rendering the 40-camera scene (30 planes)")
    t0 = time.time()
    mv = sg.make_multiview_scene(seed=sg.SCENE_SEEDS["batched"], device="cuda")
    log(f"[bench] scene ready in {time.time() - t0:.1f} s")
    ctx = pm.Context(0)
    ctx.set_views(mv.images, mv.K, mv.R, mv.t, mv.depth_ranges)
    iters = 8
    jobs = []
    for i, (ref, srcs, (win, dil)) in enumerate(zip(mv.refs, mv.sources, mv.windows)):
        jobs.append(dict(ref=ref, srcs=srcs, window=win, dilation=dil,
                         params=pm.Params(top_k=min(5, len(srcs)), seed=sg.PM_SEED + i)))
    if args.tuning:
        ctx.set_tuning(parse_tuning(pm, args.tuning))
        best, allr = ctx.get_tuning(), []
        log(f"[bench] launch configuration fixed: rows{best.tile_rows}/p{int(best.persistent)}/{best.wgs_per_cu}"
            f"{f'/depth{best.order_by_depth}' if best.order_by_depth else ''}")
    else:
        best, allr = ctx.autotune(jobs, iters=args.autotune_iters)
        log("[bench] autotune: " + ", ".join(
            f"rows{r.tile_rows}/p{int(r.persistent)}/{r.wgs_per_cu}{f'/depth{r.order_by_depth}' if r.order_by_depth else ''}={r.ms:.1f}ms"
            for r in allr))
    outs = [dict(depth=torch.empty(mv.images[j["ref"]].shape, dtype=torch.float32, device="cuda"),
                 normal=torch.empty(mv.images[j["ref"]].shape + (3,), dtype=torch.float32, device="cuda"),
                 cost=torch.empty(mv.images[j["ref"]].shape, dtype=torch.float32, device="cuda")) for j in jobs]
    gjobs = [dict(j, **o) for j, o in zip(jobs, outs)]
    for i in range(args.warmup):
        ctx.patchmatch_batch(gjobs, iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.patchmatch_batch(gjobs, iters)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"[bench] batch of {len(jobs)}: {ms_batch:.1f} ms")
    # the same depth maps one at a time through the single-view entry point
    t0 = time.perf_counter()
    for j in jobs:
        ctx.patchmatch(j["ref"], j["srcs"], j["window"], j["dilation"], iters, j["params"])
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
    tap_views = 0.0
    pixels = 0
    for j in jobs:
        H, W = mv.images[j["ref"]].shape
        R = (j["window"] - 1) // (2 * j["dilation"])
        r = R * j["dilation"]
        valid = max(0, H - 2 * r) * max(0, W - 2 * r)
        pixels += H * W
        tap_views += nominal_tap_views(valid, len(j["srcs"]), (2 * R + 1) ** 2, iters)
    achieved = tap_views * FLOPS_PER_TAP_VIEW / (ms_batch * 1e-3) / 1e12
    filt = bench_filter(ctx, mv, jobs, outs)
    phi = bench_phi(ctx, mv, jobs, outs)
    line = {
        "metric": "ms per batch of 24 mixed-size depth maps (8 it)", "value": ms_batch, "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": f"synthetic (seeded 40-camera scene, seed {sg.SCENE_SEEDS['batched']})",
        "config": {"workload": "batched: 24 references (8 x 3200x2130 at 31x31/s3, 8 x 1600x1066 at 21x21/s2, "
                               "8 x 960x640 at 11x11/s1; 11x11 taps), 6-12 sources, top-min(5,N), 8 iterations, "
                               "shared launches replayed from a hipGraph",
                   "pixels": pixels, "tuning": best.__dict__},
        "sequential_ms": ms_seq, "speedup_vs_sequential": ms_seq / ms_batch,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "note": "whole-sequence time; nominal tap-views (all 11 candidates per iteration)"},
        "autotune": [r.__dict__ for r in allr],
        "consistency_filter": filt,
        "plane_hypothesis_inference": phi,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def bench_batched_refs(args):
    """The batched workload's references one at a time through the single-view entry point
    (one warm-up run each, then one run with the exact hypothesis count and the evaluate
    kernel's time): scored tap-views per second of evaluate time, per reference and per
    size class.  --job K runs only the K-th reference (e.g. under a counter profiler)."""
    import torch

    import paper_2104_06165_amd as pm
    import scenegen as sg

    mv = sg.make_multiview_scene(seed=sg.SCENE_SEEDS["batched"], device="cuda")
    ctx = pm.Context(0)
    ctx.set_views(mv.images, mv.K, mv.R, mv.t, mv.depth_ranges)
    if args.tuning:
        ctx.set_tuning(parse_tuning(pm, args.tuning))
    iters = 8
    refs = []
    for i, (ref, srcs, (win, dil)) in enumerate(zip(mv.refs, mv.sources, mv.windows)):
        if args.job >= 0 and i != args.job:
            continue
        p = pm.Params(top_k=min(5, len(srcs)), seed=sg.PM_SEED + i)
        if args.job < 0:
            ctx.patchmatch(ref, srcs, win, dil, iters, p)  # warm-up
        ctx.diag_enable(pm.DIAG_COUNT | pm.DIAG_TIME)
        ctx.patchmatch(ref, srcs, win, dil, iters, p)
        torch.cuda.synchronize()
        n_hyp, launches, ms = ctx.diag_read()
        ctx.diag_enable(0)
        R = (win - 1) // (2 * dil)
        H, W = mv.images[ref].shape
        tv = n_hyp * len(srcs) * (2 * R + 1) ** 2
        refs.append({"job": i, "width": W, "height": H, "n_src": len(srcs),
                     "larger_sources": sum(1 for s in srcs if mv.images[s].size > mv.images[ref].size),
                     "hypotheses": n_hyp, "evaluate_ms": ms, "launches": launches,
                     "tap_views_per_s": tv / (ms * 1e-3)})
        log(f"[bench] job {i}: {W}x{H}, {len(srcs)} sources: {tv / (ms * 1e-3) / 1e12:.3f}e12 tap-views/s")
    classes = {}
    for r in refs:
        classes.setdefault(f"{r['width']}x{r['height']}", []).append(r["tap_views_per_s"])
    line = {"metric": "scored tap-views per second of evaluate time, batched workload's references one by one",
            "value": float(np.mean([r["tap_views_per_s"] for r in refs])), "unit": "tap-views/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic (seeded 40-camera scene, seed 4)",
            "config": {"workload": "batched_refs: each reference of the batched workload alone, 8 iterations",
                       "tuning": ctx.get_tuning().__dict__},
            "by_size": {k: {"min": min(v), "max": max(v)} for k, v in classes.items()}, "references": refs}
    print(json.dumps(line), flush=True)


def bench_filter(ctx, mv, jobs, outs, reps=5):
    """Geometric-consistency filter of the batch's 24 depth maps, each against the other
    references among its sources (Sec. III-D).  Algorithmic HBM bytes per reference pixel:
    its depth, normal and the three outputs (4 + 12 + 4 + 12 + 1), plus per neighbour the
    four depth texels and one normal (16 + 12)."""
    import torch

    import paper_2104_06165_amd as pm

    maps = [(j["ref"], o["depth"], o["normal"]) for j, o in zip(jobs, outs)]
    index = {j["ref"]: i for i, j in enumerate(jobs)}
    plan = [(i, [index[v] for v in j["srcs"] if v in index]) for i, j in enumerate(jobs)]
    params = pm.FilterParams()

    def run():
        return [ctx.filter(maps, i, nb, params) for i, nb in plan]

    res = run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    pixels = sum(int(mv.images[j["ref"]].size) for j in jobs)
    nbr_pixels = sum(int(mv.images[jobs[i]["ref"]].size) * len(nb) for i, nb in plan)
    algo_bytes = pixels * 33 + nbr_pixels * 28
    kept = sum(int((r[0] > 0).sum()) for r in res)
    return {"ms_per_batch": ms, "references": len(plan), "neighbour_maps_per_reference": nbr_pixels / max(pixels, 1),
            "kept_fraction": kept / pixels,
            "roofline": {"bound": "hbm", "achieved": algo_bytes / (ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": algo_bytes / (ms * 1e-3) / 1e9 / 8000.0, "traffic": None,
                         "note": "whole-batch time over 24 launches (host launch gaps included)"}}


def bench_phi(ctx, mv, jobs, outs, size=None):
    """Plane hypothesis inference (Sec. III-E) on the references (of one size class if
    given): each depth map is filtered by geometric consistency against the other
    references among its sources, its empty pixels get hypotheses, costs, a selection (graph
    model decoded on the host) and normals, and the filled maps are filtered again against
    each other.  Reported: completeness (pixels with depth) and accuracy against the
    rendered depth at each stage, the GPU time of hypotheses + costs + normals and the host
    time of the selection."""
    import torch

    import paper_2104_06165_amd as pm

    maps = [(j["ref"], o["depth"], o["normal"]) for j, o in zip(jobs, outs)]
    index = {j["ref"]: i for i, j in enumerate(jobs)}
    sel = [i for i, j in enumerate(jobs) if size is None or mv.images[j["ref"]].shape[::-1] == tuple(size)]
    fparams = pm.FilterParams()
    filtered = {}
    for i, j in enumerate(jobs):
        nb = [index[v] for v in j["srcs"] if v in index]
        d, n, _ = ctx.filter(maps, i, nb, fparams)
        filtered[i] = (d, n)
    torch.cuda.synchronize()
    gpu_ms = host_ms = 0.0
    filled = {}
    for i in sel:
        j = jobs[i]
        d, n = filtered[i]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.prepare(j["ref"], j["srcs"], j["window"], j["dilation"], j["params"])
        hyp = ctx.phi_hypotheses(d)
        cost = ctx.phi_costs(hyp)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dp = ctx.phi_select(d, hyp, cost)
        t2 = time.perf_counter()
        npn = ctx.phi_normals(j["ref"], dp)
        new = (d <= 0) & (dp > 0)
        nf = torch.where(new[..., None], npn, n).contiguous()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        gpu_ms += (t1 - t0 + t3 - t2) * 1e3
        host_ms += (t2 - t1) * 1e3
        filled[i] = (dp, nf)
    # second filter pass over the filled maps (the others keep their filtered maps)
    maps2 = [(j["ref"],) + (filled[i] if i in filled else filtered[i]) for i, j in enumerate(jobs)]
    final = {}
    for i in sel:
        nb = [index[v] for v in jobs[i]["srcs"] if v in index]
        final[i] = ctx.filter(maps2, i, nb, fparams)[0]
    torch.cuda.synchronize()

    def stats(get):
        n_px = hit = good1 = good5 = 0
        for i in sel:
            gt = mv.gt_depths[jobs[i]["ref"]]
            d = get(i).cpu().numpy()
            m = d > 0
            rel = np.abs(d[m] - gt[m]) / gt[m]
            n_px += d.size
            hit += int(m.sum())
            good1 += int((rel < 0.01).sum())
            good5 += int((rel < 0.05).sum())
        return {"completeness": hit / n_px, "within_1pct_of_filled": good1 / max(hit, 1),
                "within_5pct_of_filled": good5 / max(hit, 1)}

    return {"references": len(sel), "pixels": int(sum(mv.images[jobs[i]["ref"]].size for i in sel)),
            "raw": stats(lambda i: outs[i]["depth"]), "filtered": stats(lambda i: filtered[i][0]),
            "phi_filled": stats(lambda i: filled[i][0]), "phi_filtered_again": stats(lambda i: final[i]),
            "gpu_ms": gpu_ms, "host_selection_ms": host_ms,
            "fusion": bench_fusion(ctx, mv, [(jobs[i]["ref"], final[i]) for i in sel])}


def bench_fusion(ctx, mv, maps, tau=0.01, reps=3):
    """Depth-map fusion (Sec. III-F) of the final maps in reference order: GPU time (best of
    reps), points, support, and against the rendered depth: accuracy (points whose depth in
    the camera of the pixel they started from is within 1% of that pixel's true depth) and
    completeness (pixels of all maps that ended in an accurate point)."""
    import torch

    ms = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pts, sup, own = ctx.fuse(maps, tau)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    dev = pts.device
    sizes = [d.numel() for _, d in maps]
    gt = torch.cat([torch.from_numpy(np.ascontiguousarray(mv.gt_depths[v], np.float32)).reshape(-1) for v, _ in maps])
    gt = gt.to(dev).double()
    mapid = torch.repeat_interleave(torch.arange(len(maps), device=dev), torch.tensor(sizes, device=dev))
    Rz = torch.from_numpy(np.stack([mv.R[v][2] for v, _ in maps])).to(dev)
    tz = torch.from_numpy(np.array([mv.t[v][2] for v, _ in maps])).to(dev)
    g = torch.nonzero(sup > 0)[:, 0]
    m = mapid[g]
    z = (Rz[m] * pts[g].double()).sum(-1) + tz[m]
    acc = (z - gt[g]).abs() < 0.01 * gt[g]
    good = torch.zeros_like(sup, dtype=torch.bool)
    good[g] = acc
    has = own >= 0
    covered = has & good[own.clamp(min=0)]
    n_pts = int(g.numel())
    return {"ms": min(ms), "maps": len(maps), "pixels": int(sum(sizes)), "pixels_with_depth": int(has.sum()),
            "points": n_pts, "mean_support": float(sup[g].double().mean()) if n_pts else 0.0,
            "accuracy_1pct": float(acc.double().mean()) if n_pts else 0.0,
            "completeness_1pct": float(covered.double().mean()), "max_rel_dist": tau}


def bench_resize(args):
    """The paper's window-resize study (Table III) on the 1600x1066 scene (9 sources, top-4,
    8 iterations): r_now taps per side over the original radius r_orig, for r_orig = 5..10,
    against the dense window (r_now = r_orig).  Reported per configuration: ms per depth map,
    depth accuracy against the ground truth and the evaluate kernel's rate."""
    import torch

    import paper_2104_06165_amd as pm
    import scenegen as sg

    scene = sg.workload_scene("mid", device="cuda")
    ctx = pm.Context(0)
    ctx.set_scene(scene)
    srcs = list(range(1, len(scene.images)))
    H, W = scene.images[0].shape
    textured = scene.textured[scene.gt_plane]
    rows = []
    for r_orig in range(5, 11):
        for r_now in sorted({5, r_orig}):
            window = 2 * r_orig + 1
            params = pm.Params(top_k=4, sigma_spatial_px=float(r_orig), seed=sg.PM_SEED,
                               tap_radius=r_now if r_now != r_orig else 0)
            run = lambda: ctx.patchmatch(0, srcs, window, 1, 8, params)  # noqa: E731
            for _ in range(args.warmup):
                run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                d, n, c = run()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            dd = d.cpu().numpy()
            valid = np.zeros((H, W), bool)
            valid[r_orig:H - r_orig, r_orig:W - r_orig] = True
            rel = np.abs(dd - scene.gt_depth) / scene.gt_depth
            rows.append({"r_now": r_now, "r_orig": r_orig, "taps": (2 * r_now + 1) ** 2, "ms": ms,
                         "depth_within_1pct": float((rel[valid] < 0.01).mean()),
                         "depth_within_1pct_textured": float((rel[valid & textured] < 0.01).mean())})
            log(f"[bench] {r_now}/{r_orig}: {ms:.1f} ms, within 1% {rows[-1]['depth_within_1pct']:.4f}")
    line = {"metric": "ms per 1600x1066 depth map by matching-window configuration (r_now/r_orig)",
            "value": rows[0]["ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": rows[0]["ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": f"synthetic (seeded piecewise-planar scene, seed {sg.SCENE_SEEDS['mid']})",
            "config": {"workload": "resize: 1 reference + 9 sources at 1600x1066, top-4, 8 iterations, windows "
                                   "r_orig = 5..10 with r_now = 5 (window-resize scheme) or r_now = r_orig"},
            "table": rows}
    ctx.close()
    print(json.dumps(line), flush=True)


def learned_vs_random(ctx, net, scene, srcs, solver, params, valid, textured, random_ms, reps=3):
    """Learned-proposal initialisation against random initialisation at equal final cost:
    the mean cost (valid pixels) after k = 0..iters iterations of both, the fewest
    iterations at which the learned run reaches the random run's final mean cost within
    1%, and the end-to-end time of that run (proposal network included) against the
    random run's full time."""
    import torch

    iters = solver["iters"]
    win, dil = solver["window"], solver["dilation"]
    gt = scene.gt_depth

    def stats(d, c):
        d = d.cpu().numpy()
        c = c.cpu().numpy()
        rel = np.abs(d - gt) / gt
        return {"mean_cost": float(c[valid].mean()),
                "depth_within_1pct": float((rel[valid] < 0.01).mean()),
                "depth_within_1pct_textured": float((rel[valid & textured] < 0.01).mean()),
                "mean_abs_rel_depth_error": float(rel[valid].mean())}

    rand, learned = [], []
    for k in range(iters + 1):
        d, n, c = ctx.patchmatch(0, srcs, win, dil, k, params)
        rand.append(stats(d, c))
    proposal = ctx.propose(net, 0, srcs)
    for k in range(iters + 1):
        d, n, c = ctx.patchmatch_proposal(0, srcs, win, dil, k, proposal, params)
        learned.append(stats(d, c))
    # pixels whose initial plane is the proposal: the gated initial cost is below the random one's
    c_rand0 = ctx.patchmatch(0, srcs, win, dil, 0, params)[2]
    c_learn0 = ctx.patchmatch_proposal(0, srcs, win, dil, 0, proposal, params)[2]
    vt = torch.from_numpy(valid).to(c_rand0.device)
    kept = float(((c_learn0 < c_rand0) & vt).sum().item() / max(int(vt.sum().item()), 1))
    target = 1.01 * rand[iters]["mean_cost"]
    k_rand = next(k for k in range(iters + 1) if rand[k]["mean_cost"] <= target)
    k_learned = next((k for k in range(iters + 1) if learned[k]["mean_cost"] <= target), None)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    out = {"target_mean_cost": target, "random_iters_to_target": k_rand, "learned_iters_to_target": k_learned,
           "random_ms": random_ms, "proposal_kept_fraction": kept,
           "per_iteration": {"random": rand, "learned": learned}}
    out["proposal_ms"] = timed(lambda: ctx.propose(net, 0, srcs, out=proposal))
    if k_learned is not None:
        def run():
            ctx.propose(net, 0, srcs, out=proposal)
            ctx.patchmatch_proposal(0, srcs, win, dil, k_learned, proposal, params)
        out["learned_ms"] = timed(run)
        # the end-to-end speed-up at equal cost: the random run stopped as soon as it reaches
        # the same target, against the learned run (proposal network and gate included)
        out["random_ms_at_target"] = timed(lambda: ctx.patchmatch(0, srcs, win, dil, k_rand, params))
        out["speedup_at_equal_cost"] = out["random_ms_at_target"] / out["learned_ms"]
        # against the full 8-iteration random run: this measures the 1% margin as much as the network
        out["speedup_vs_full_random_run"] = random_ms / out["learned_ms"]
        out["learned_at_target"] = learned[k_learned]
        out["random_final"] = rand[iters]
    # the ceiling of any initialisation under this metric: the scene's true planes as the
    # proposal (the search converges below their cost, so they too need iterations)
    true_p = np.concatenate([scene.gt_normal, scene.gt_depth[..., None]], -1).astype(np.float32)
    gt_planes = torch.from_numpy(np.ascontiguousarray(true_p)).to(proposal.device)
    k_gt = None
    for k in range(iters + 1):
        if stats(*ctx.patchmatch_proposal(0, srcs, win, dil, k, gt_planes, params)[::2])["mean_cost"] <= target:
            k_gt = k
            break
    out["true_planes_iters_to_target"] = k_gt
    return out


def bench_ceiling(args):
    """How much any initialisation could gain under the equal-cost metric on the 3200x2130
    workload: synthetic proposals handed to the same gated initialisation (true planes;
    true depth with 2% and 5% multiplicative noise, true or perturbed normals; the 4x4
    block mean of the true depth as fronto-parallel planes, plain and quantised to 32
    inverse-depth levels), each run for k = 0..iters iterations, against the random run's
    final mean cost + 1%.  Seeded noise (numpy, seed 7)."""
    import torch

    import paper_2104_06165_amd as pm
    import scenegen as sg

    scene = sg.workload_scene("highres", device="cuda")
    sol = sg.SOLVER["highres"]
    srcs = list(range(1, len(scene.images)))
    win, dil, iters = sol["window"], sol["dilation"], sol["iters"]
    params = pm.Params(top_k=sol["top_k"], bilateral=True, sigma_spatial_px=(win - 1) / 2.0, seed=sg.PM_SEED)
    ctx = pm.Context(0)
    ctx.set_scene(scene)
    H, W = scene.images[0].shape
    r = dil * ((win - 1) // (2 * dil))
    valid = np.zeros((H, W), bool)
    valid[r:H - r, r:W - r] = True
    K = scene.cams[0].K
    ys, xs = np.mgrid[0:H, 0:W]
    rays = np.stack([xs, ys, np.ones_like(xs)], -1).astype(np.float64) @ np.linalg.inv(K).T
    rng = np.random.default_rng(7)

    def facing(n):
        n = n / np.linalg.norm(n, axis=-1, keepdims=True)
        flip = (n * rays).sum(-1) > 0
        n[flip] = -n[flip]
        return n

    lo, hi = scene.depth_range
    gt_d, gt_n = scene.gt_depth.astype(np.float64), scene.gt_normal.astype(np.float64)
    bm = gt_d[:H - H % 4, :W - W % 4].reshape(H // 4, 4, W // 4, 4).mean(axis=(1, 3))
    block = np.pad(np.repeat(np.repeat(bm, 4, 0), 4, 1), ((0, H % 4), (0, W % 4)), mode="edge")
    inv = 1.0 / block
    q = np.round((inv - 1.0 / hi) / ((1.0 / lo - 1.0 / hi) / 31)) * ((1.0 / lo - 1.0 / hi) / 31) + 1.0 / hi
    fronto = facing(np.broadcast_to(np.array([0.0, 0.0, -1.0]), (H, W, 3)).copy())
    kinds = {
        "true planes": (gt_n, gt_d),
        "true depth x (1 + 2% noise), true normals": (gt_n, gt_d * (1 + 0.02 * rng.standard_normal((H, W)))),
        "true depth x (1 + 5% noise), normals +-0.2": (facing(gt_n + rng.uniform(-0.2, 0.2, (H, W, 3))),
                                                     gt_d * (1 + 0.05 * rng.standard_normal((H, W)))),
        "4x4-block mean depth, fronto-parallel": (fronto, block),
        "the same quantised to 32 inverse-depth levels": (fronto, 1.0 / q),
    }

    def mean_cost(c):
        return float(c.cpu().numpy()[valid].mean())

    rand = [mean_cost(ctx.patchmatch(0, srcs, win, dil, k, params)[2]) for k in range(iters + 1)]
    target = 1.01 * rand[-1]
    rows = [{"proposal": "random (the method's own initialisation)", "mean_cost": rand,
             "iters_to_target": next(k for k in range(iters + 1) if rand[k] <= target)}]
    for name, (n, d) in kinds.items():
        planes = np.concatenate([n, np.clip(d, lo, hi)[..., None]], -1).astype(np.float32)
        prop = torch.from_numpy(np.ascontiguousarray(planes)).cuda()
        mc = []
        for k in range(iters + 1):
            mc.append(mean_cost(ctx.patchmatch_proposal(0, srcs, win, dil, k, prop, params)[2]))
            if mc[-1] <= target:
                break
        rows.append({"proposal": name, "mean_cost": mc,
                     "iters_to_target": len(mc) - 1 if mc[-1] <= target else None})
        log(f"[bench] {name}: {rows[-1]['iters_to_target']} iterations ({', '.join(f'{v:.4f}' for v in mc)})")
    ctx.close()
    line = {"metric": "iterations to the random run's final mean cost + 1% from synthetic initial proposals",
            "value": min(r["iters_to_target"] for r in rows if r["iters_to_target"] is not None),
            "unit": "iterations", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": f"synthetic (seeded piecewise-planar scene, seed {sg.SCENE_SEEDS['highres']}; noise seed 7)",
            "config": {"workload": "ceiling: 1 reference + 10 sources at 3200x2130, 31x31 at dilation 3, top-5, "
                                   "8 iterations, gated initialisation from synthetic proposals"},
            "target_mean_cost": target, "table": rows}
    print(json.dumps(line), flush=True)


def bench_taps(args):
    """Split of the evaluate kernel's time on the 3200x2130 workload (10 sources, top-5, 8
    iterations) into a part per window tap and a fixed part per (pixel, hypothesis, view):
    the same depth map at 3x3 to 19x19 taps (window and dilation varied), every candidate
    scored (score_all = 2, so each configuration scores about the same hypotheses), and a
    least-squares line through the evaluate time per hypothesis against the tap count."""
    import torch

    import paper_2104_06165_amd as pm
    import scenegen as sg

    scene = sg.workload_scene("highres", device="cuda")
    sol = sg.SOLVER["highres"]
    srcs = list(range(1, len(scene.images)))
    params = pm.Params(top_k=sol["top_k"], bilateral=True, sigma_spatial_px=(sol["window"] - 1) / 2.0,
                       seed=sg.PM_SEED, score_all=2)
    ctx = pm.Context(0)
    ctx.set_scene(scene)
    rows = []
    for window, dilation in [(31, 15), (31, 5), (25, 3), (31, 3), (25, 2), (29, 2), (37, 2)]:
        n = (window - 1) // dilation + 1
        for _ in range(args.warmup):
            ctx.patchmatch(0, srcs, window, dilation, sol["iters"], params)
        torch.cuda.synchronize()
        ctx.diag_enable(pm.DIAG_TIME | pm.DIAG_COUNT)
        for _ in range(args.steps):
            ctx.patchmatch(0, srcs, window, dilation, sol["iters"], params)
        torch.cuda.synchronize()
        hyp, launches, kms = ctx.diag_read()
        ctx.diag_enable(0)
        rows.append({"window": window, "dilation": dilation, "taps": n * n, "eval_ms": kms / args.steps,
                     "hypotheses": hyp // args.steps})
        log(f"[bench] {n}x{n} taps: evaluate {rows[-1]['eval_ms']:.1f} ms per depth map")
    ctx.close()
    t = np.array([r["taps"] for r in rows], np.float64)
    hyp = np.array([r["hypotheses"] for r in rows], np.float64)
    # evaluate time scaled to the mean hypothesis count (the counts differ by under 1%)
    ms = np.array([r["eval_ms"] for r in rows], np.float64) * hyp.mean() / hyp
    slope, fixed = np.polyfit(t, ms, 1)
    # wave64 VALU issue: 4 SIMDs per CU, one wave instruction per 4 cycles each
    wave_instr_per_s = 256 * 4 * 2.4e9 / 4
    wave_views = hyp.mean() * len(srcs) / 64
    line = {"metric": "evaluate-kernel ms per 3200x2130 depth map against window taps",
            "value": float(ms[t == 121][0]), "unit": "ms", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": float(ms[t == 121][0]), "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": f"synthetic (seeded piecewise-planar scene, seed {sg.SCENE_SEEDS['highres']})",
            "config": {"workload": "taps: 1 reference + 10 sources at 3200x2130, top-5, 8 iterations, "
                                   "3x3 to 19x19 taps, every candidate scored"},
            "fit": {"ms_per_tap": float(slope), "fixed_ms": float(fixed),
                    "fixed_share_at_121_taps": float(fixed / (fixed + 121 * slope)),
                    "wave_instr_time_per_tap_view": float(slope * 1e-3 * wave_instr_per_s / wave_views),
                    "wave_instr_time_fixed_per_view": float(fixed * 1e-3 * wave_instr_per_s / wave_views)},
            "table": rows}
    print(json.dumps(line), flush=True)


def bench_train(args):
    """One training step of the proposal network at the training shape: a minibatch of 8
    samples at 267x400 (1/4 of 1600x1066), 5 input channels, masked loss, gradient of
    every layer and an Adam step, on seeded synthetic inputs and targets."""
    import torch

    import paper_2104_06165_amd as pm

    B, h, w = 8, 267, 400
    g = torch.Generator(device="cuda").manual_seed(1)
    x = torch.rand((B, h, w, 5), generator=g, device="cuda")
    nrm = torch.nn.functional.normalize(torch.randn((B, h, w, 3), generator=g, device="cuda"), dim=-1)
    nrm[..., 2] = -nrm[..., 2].abs()
    rng = torch.tensor([1.0, 20.0], device="cuda").repeat(B, 1).contiguous()
    dep = 1.0 + 19.0 * torch.rand((B, h, w, 1), generator=g, device="cuda")
    target = torch.cat([dep, nrm], -1).contiguous()
    mask = (torch.rand((B, h, w), generator=g, device="cuda") < 0.7).float().contiguous()
    net = pm.Net(0, np.load(args.weights) if os.path.exists(args.weights) else None)
    step = lambda: (net.loss_grad(x, target, mask, rng, 1.0, want_loss=True), net.adam(1e-3))  # noqa: E731
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    net.close()
    # flops per pixel: forward, weight gradient and data gradient (none for the input layer)
    fwd = sum(2 * 9 * ci * co for ci, co in pm.Net.SHAPES)
    per_px = 2 * fwd + (fwd - 2 * 9 * pm.Net.SHAPES[0][0] * pm.Net.SHAPES[0][1])
    flops = per_px * B * h * w
    line = {"metric": "ms per proposal-network training step (minibatch 8 at 267x400)", "value": ms, "unit": "ms",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic (seeded random inputs and targets)",
            "config": {"workload": "train: 5-layer 3x3 network (5-32-32-32-32-4), bf16 MFMA, minibatch 8 at "
                                   "267x400, masked loss, all gradients, Adam"},
            "samples_per_s": B / (ms * 1e-3),
            "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": flops / (ms * 1e-3) / 1e12 / 2500.0, "traffic": None,
                         "note": "whole step (loss read back to the host each step, as in training)"}}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="highres",
                    choices=["highres", "mid", "mid_dense", "tiny", "batched", "batched_refs", "resize", "taps", "train",
                             "ceiling"])
    ap.add_argument("--cpu-iters", type=int, default=1,
                    help="iterations of the single-threaded oracle's sample (the all-thread runs take the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2104_06165_amd", "weights", "proposal_net.npy"),
                    help="parameters of the proposal network for the learned-versus-random comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-versus-random comparison")
    ap.add_argument("--score-all", type=int, default=0, choices=(0, 1, 2),
                    help="0: leave out every propagation candidate that cannot win (default); 1: not those "
                         "offered by the previous propagation of the colour; 2: score every candidate")
    ap.add_argument("--autotune-iters", type=int, default=3,
                    help="batched workload: iterations per autotuner trial (from the second on, the "
                         "propagation launches leave out candidates offered before, as in a full run)")
    ap.add_argument("--no-skip-counts", action="store_true",
                    help="do not count the hypotheses of the other score_all settings (extra untimed runs)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes sharing each pixel (2..16: split tap sums, for small references); 0: one lane")
    ap.add_argument("--tuning", default="", metavar="ROWS,PERSISTENT,WGS[,ORDER_BY_DEPTH]",
                    help="evaluate-kernel launch configuration (batched workload: instead of autotuning)")
    ap.add_argument("--job", type=int, default=-1,
                    help="batched_refs workload: only this reference (index in the batch); -1: all 24")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM-counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the depth-map estimation runs on one GPU; --gpus above 1 is not supported "
              "(the depth maps of a scene would shard by reference view, one process per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2104_06165_amd as pm
    import scenegen as sg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        # one elementwise kernel that reads and writes exactly n bytes each
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)
        return
    wl = args.workload
    if wl == "batched":
        return bench_batched(args)
    if wl == "batched_refs":
        return bench_batched_refs(args)
    if wl == "resize":
        return bench_resize(args)
    if wl == "taps":
        return bench_taps(args)
    if wl == "train":
        return bench_train(args)
    if wl == "ceiling":
        return bench_ceiling(args)
    scene_name = "mid" if wl.startswith("mid") else wl
    solver = sg.SOLVER[wl]
    cfg = sg.CONFIGS[scene_name]
    log(f"[bench] rendering the {wl} scene ({cfg.width}x{cfg.height}, {cfg.n_src} sources, {cfg.n_planes} planes)")
    t0 = time.time()
    scene = sg.workload_scene(scene_name, device="cuda")
    log(f"[bench] scene ready in {time.time() - t0:.1f} s")

    ctx = pm.Context(0)
    ctx.set_scene(scene)
    if args.tuning:
        ctx.set_tuning(parse_tuning(pm, args.tuning))
    n_src = len(scene.images) - 1
    srcs = list(range(1, n_src + 1))
    params = pm.Params(top_k=solver["top_k"], bilateral=True, sigma_spatial_px=(solver["window"] - 1) / 2.0,
                       seed=sg.PM_SEED, lanes=args.lanes, score_all=args.score_all)
    H, W = scene.images[0].shape
    out = (torch.empty((H, W), dtype=torch.float32, device="cuda"),
           torch.empty((H, W, 3), dtype=torch.float32, device="cuda"),
           torch.empty((H, W), dtype=torch.float32, device="cuda"))

    def run():
        return ctx.patchmatch(0, srcs, solver["window"], solver["dilation"], solver["iters"], params, out=out)

    # exact number of hypotheses scored per depth map (deterministic: counter-based RNG), also
    # with fewer of the candidates that cannot win left out (same results, more work)
    ctx.diag_enable(pm.DIAG_COUNT)
    run()
    n_hyp, _, _ = ctx.diag_read()
    hyp_by_level = {}
    for level in (0, 1, 2):
        if level == args.score_all or args.no_skip_counts:
            hyp_by_level[level] = n_hyp
            continue
        ctx.diag_enable(pm.DIAG_COUNT)  # resets the count
        ctx.patchmatch(0, srcs, solver["window"], solver["dilation"], solver["iters"],
                       dataclasses.replace(params, score_all=level), out=out)
        hyp_by_level[level], _, _ = ctx.diag_read()
    ctx.diag_enable(0)
    for i in range(args.warmup):
        run()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    ctx.diag_enable(pm.DIAG_TIME)
    # per-step times from events between the steps (recorded on the stream the library uses)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record()
    for i in range(args.steps):
        run()
        marks[i + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = [marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)]
    _, launches, kernel_ms = ctx.diag_read()
    ctx.diag_enable(0)
    ms_per_step = elapsed * 1e3 / args.steps
    log(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms per depth map")

    R = (solver["window"] - 1) // (2 * solver["dilation"])
    taps = (2 * R + 1) ** 2
    launches_per_step = launches / args.steps
    flops_per_step = float(n_hyp) * n_src * taps * FLOPS_PER_TAP_VIEW
    avg_launch_ms = kernel_ms / launches
    achieved = flops_per_step / launches_per_step / (avg_launch_ms * 1e-3) / 1e12
    # the same depth map with the 8-bit images handed over from host memory (upload included)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_scene(scene)
    run()
    torch.cuda.synchronize()
    pcie_ms = (time.perf_counter() - t0) * 1e3
    traffic = measured_traffic("phimvs_kernels.hip", "eval_kernel_highres_hbm.md") if wl == "highres" else None
    depth, normal, cost = out
    d = depth.cpu().numpy()
    c = cost.cpu().numpy()
    r = solver["dilation"] * R
    valid = np.zeros_like(d, dtype=bool)
    valid[r:H - r, r:W - r] = True
    rel = np.abs(d - scene.gt_depth) / scene.gt_depth
    textured = scene.textured[scene.gt_plane]

    line = {
        "metric": METRIC,
        "value": ms_per_step,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": f"synthetic (seeded piecewise-planar scene, seed {sg.SCENE_SEEDS[scene_name]}); random init",
        "config": {"workload": f"{wl}: 1 reference + {n_src} sources at {W}x{H}, {solver['window']}x{solver['window']} "
                               f"window at dilation {solver['dilation']} ({2 * R + 1}x{2 * R + 1} taps), "
                               f"top-{solver['top_k']}, {solver['iters']} iterations",
                   "width": W, "height": H, "n_src": n_src, "window": solver["window"],
                   "dilation": solver["dilation"], "top_k": solver["top_k"], "iters": solver["iters"],
                   "planes": cfg.n_planes, "images": "8-bit texel quads (sources), fp16 copy (reference) in HBM",
                   "cost": "fp32", "lanes_per_pixel": max(1, args.lanes),
                   "tuning": ctx.get_tuning().__dict__},
        "ms_per_step_min": min(step_ms),
        "ms_per_step_median": float(np.median(step_ms)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                     "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "eval_kernel (evaluate-and-select)", "avg_launch_ms": avg_launch_ms,
                     "launches_per_step": launches_per_step,
                     "kernel_share_of_step": kernel_ms / (elapsed * 1e3),
                     # every candidate the method offers counted as scored (score_all = 2), over the
                     # same kernel time: the rate of the method's nominal work that leaving out the
                     # candidates that cannot win gives; achieved and frac count only those scored
                     "achieved_nominal": (achieved * hyp_by_level[2] / n_hyp) if 2 in hyp_by_level else None,
                     "frac_nominal": (achieved * hyp_by_level[2] / n_hyp / PEAK_FP32_VECTOR_TFLOPS)
                     if 2 in hyp_by_level else None},
        "pcie_inclusive_ms": pcie_ms,
        "hypotheses_per_step": n_hyp,
        "hypotheses_per_step_by_score_all": {str(k): v for k, v in sorted(hyp_by_level.items())},
        "cost_evals_per_s": n_hyp * n_src / (ms_per_step * 1e-3),
        "tap_views_per_s": n_hyp * n_src * taps / (ms_per_step * 1e-3),
        "quality": {"mean_cost": float(c[valid].mean()),
                    "depth_within_1pct": float((rel[valid] < 0.01).mean()),
                    "depth_within_1pct_textured": float((rel[valid & textured] < 0.01).mean())},
    }
    if not args.no_learned and wl == "highres" and os.path.exists(args.weights):
        log("[bench] learned proposal versus random initialisation")
        net = pm.Net(0, np.load(args.weights))
        lv = learned_vs_random(ctx, net, scene, srcs, solver, params, valid, textured, ms_per_step)
        line["learned_vs_random"] = {k: v for k, v in lv.items() if k != "per_iteration"}
        line["learned_vs_random"]["weights"] = os.path.relpath(args.weights, ROOT)
        for key in ("mean_cost", "depth_within_1pct", "mean_abs_rel_depth_error"):
            line["learned_vs_random"][key + "_per_iteration"] = {
                "random": [r[key] for r in lv["per_iteration"]["random"]],
                "learned": [r[key] for r in lv["per_iteration"]["learned"]]}
        log("[bench] " + json.dumps(line["learned_vs_random"]))
        net.close()
    if not args.no_cpu_baseline and wl == "highres":
        log("[bench] timing the CPU oracle on its bounded sample")
        line["cpu_baseline"] = cpu_baseline(ctx, scene, solver, args.cpu_iters)
        log(f"[bench] cpu baseline: {line['cpu_baseline']['sample']}")
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
