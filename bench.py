#!/usr/bin/env python3
"""Benchmark of the sliding-window Gaussian-splatting hot path on one MI355X.

Workload of `value` (config 2): the paper-scale window step -- 200k
optimisable Gaussians plus their 200k-slot frozen store, SH degree 3, a
window of 10 frames x 4 cameras at 1352x1014, every frame with exactly 200k
live slots (10% retire and 10% are born per frame), 2% of the Gaussians
near-transparent at the start (so relocation has work from the first step).
One step = forward of all 40 views, the image term 0.8 L1 + 0.2 D-SSIM and
its gradient, backward, Adam + SGLD, relocation.

The step runs in three launch structures on the same inputs, from the same
initial state with the same seeds: GRAPH (chosen form: the batched sequence
captured once in a hipGraph), BATCHED (one launch per kernel over all views;
its timed runs also yield the per-kernel HIP-event breakdown) and PLAIN (one
launch sequence per view with a host read-back of each view's pair count,
the per-frame baseline).  Each form does `--warmup` untimed steps, then
`--reps` timed runs of `--steps` steps (device synchronised around each
run); ms/step is the median run.  `value` is GRAPH window steps/s.  After
`--psnr-steps` steps in total the PSNR of each form shows they train
equally.  The other configurations -- the tiny window (1), the uneven
180-view window (3) and the 1M-Gaussian long video (5) -- are timed the same
way under `configs`; serving (4) under `serving`.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--num-gs", type=int, default=200_000)
    ap.add_argument("--swin", type=int, default=10)
    ap.add_argument("--cams", type=int, default=4)
    ap.add_argument("--width", type=int, default=1352)
    ap.add_argument("--height", type=int, default=1014)
    ap.add_argument("--sh-degree", type=int, default=3)
    ap.add_argument("--tile", default="auto", help="auto (autotuner) or WxH")
    ap.add_argument("--lds-batch", type=int, default=0)
    ap.add_argument("--modes", default="graph,batched,plain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=1536)
    ap.add_argument("--serve-rates", default="200,500,1000,4000",
                    help="Poisson request rates (req/s); empty: no serving")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="measured seconds per rate (after 1 s warm-up)")
    ap.add_argument("--serve-active", type=int, default=300_000)
    ap.add_argument("--serve-frames", type=int, default=300)
    ap.add_argument("--serve-lanes", type=int, default=3)
    ap.add_argument("--serve-max-batch", type=int, default=16)
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--stream-frames", type=int, default=10, help="frames of the update-stream run; 0: skip it")
    ap.add_argument("--literal-iters", type=int, default=200,
                    help="timed iterations of the paper's one-view-per-iteration loop; 0: skip it")
    ap.add_argument("--reps", type=int, default=5, help="timed runs of --steps steps per form (median reported)")
    ap.add_argument("--psnr-steps", type=int, default=200, help="steps (in total) before the PSNR comparison")
    ap.add_argument("--dead-fraction", type=float, default=0.02,
                    help="fraction of the student's Gaussians made near-transparent at the start (seeded)")
    ap.add_argument("--c1", type=int, default=1, help="time the tiny window (config 1)")
    ap.add_argument("--c1-steps", type=int, default=100)
    ap.add_argument("--c3", type=int, default=1, help="time the uneven 180-view window (config 3)")
    ap.add_argument("--c3-steps", type=int, default=10)
    ap.add_argument("--c3-tile", default="auto", help="auto (autotuner) or WxH/LDS, e.g. 16x16/256")
    ap.add_argument("--c3-forms", default="graph,plain")
    ap.add_argument("--c5-advances", type=int, default=300, help="window advances of the 1M long video; 0: skip")
    ap.add_argument("--cpu-threads", type=int, default=0, help="threads of the oracle's all-core leg (0: the host's)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run 3 device-to-device copies of this many MiB (HBM counter calibration) and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is a design "
              "described in DESIGN.md, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 18
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 3}), flush=True)
        return

    from paper_2409_07759_amd import swgs
    from paper_2409_07759_amd import synth as S

    from paper_2409_07759_amd import autotune

    dev = torch.device("cuda", 0)
    st0 = args.swin
    frames = list(range(st0, st0 + args.swin))
    t0 = time.time()
    student = S.steady_window_pool(args.num_gs, args.swin, args.sh_degree, st0, seed=0)
    teacher = S.steady_window_pool(args.num_gs, args.swin, args.sh_degree, st0, seed=1)
    views = S.ring_views(frames, args.cams, args.width, args.height, phase_deg=10.0)
    log(f"inputs built in {time.time() - t0:.1f}s: {student.slots} slots, {len(views)} views")

    ctx = swgs.Context(0)
    # targets: teacher renders (forward only)
    tpool = swgs.Pool.from_synth(teacher, train=False)
    tplan = swgs.Plan(ctx, tpool, views)
    targets = tplan.forward()
    torch.cuda.synchronize()
    tplan.close()
    del tpool
    log("targets rendered")

    tune_table = None
    if args.tile == "auto":
        dp = swgs.Pool.from_synth(student)
        (tw, th), lds, tune_table = autotune.tune(ctx, dp, views, use_cache=False, log=log)
        del dp
        if args.lds_batch == 0:
            args.lds_batch = lds
        log(f"autotuned: {tw}x{th}, lds batch {args.lds_batch}")
    else:
        tw, th = (int(x) for x in args.tile.split("x"))
    S.add_faint_gaussians(student, args.dead_fraction, seed=5)
    cfg_base = dict(window_start=st0, relocate_period=1)
    results = run_forms(ctx, student, views, targets, (tw, th), args.lds_batch, cfg_base,
                        [m.strip() for m in args.modes.split(",")], args.steps, args.warmup, args.reps,
                        args.psnr_steps, breakdown=True, label="c2")

    chosen = "graph" if "graph" in results else list(results)[0]
    out = {
        "metric": "window train steps/s (batched hipGraph step vs plain per-frame launches, same PSNR)",
        "value": round(results[chosen]["steps_per_s"], 4),
        "unit": "window steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(results[chosen]["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; DyNeRF-shaped window: 300-frame clip scale, 1352x1014, 200k live Gaussians)",
        "config": {
            "workload": f"paper-scale window step: {args.num_gs} optimisable + {args.num_gs} frozen Gaussians, "
                        f"SH degree {args.sh_degree}, W={args.swin} frames x {args.cams} cameras at "
                        f"{args.width}x{args.height}, image term 0.8 L1 + 0.2 D-SSIM, Adam+SGLD+relocation "
                        f"every step, {args.dead_fraction:g} of the Gaussians near-transparent at the start",
            "views": len(views), "tile": f"{tw}x{th}", "lds_batch": args.lds_batch, "form": chosen,
            "repetitions": args.reps, "statistic": f"median of {args.reps} timed runs of {args.steps} steps",
        },
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()
                      if kk not in ("timing", "counts", "timed_steps")}
                  for k, v in results.items()},
    }
    if "plain" in results:
        out["speedup_vs_plain"] = round(results[chosen]["steps_per_s"] / results["plain"]["steps_per_s"], 3)
        out["psnr_delta_vs_plain_db"] = round(results[chosen]["psnr"] - results["plain"]["psnr"], 4)
        out["psnr_steps"] = results[chosen]["psnr_steps"]
    if tune_table:
        out["autotune_ms_fwd_bwd"] = {f"{t[0]}x{t[1]}/lds{l}": ms for t, l, ms in tune_table}
    if "batched" in results and results["batched"]["timing"]:
        out.update(roofline_report(results["batched"], (tw, th), args.lds_batch))
    configs = {}
    if args.c1:
        configs["c1"] = run_c1(args, ctx)
    if args.c3:
        configs["c3"] = run_c3(args, ctx)
    if args.c5_advances > 0:
        configs["c5"] = run_c5(args, ctx)
    if configs:
        out["configs"] = configs
    if args.literal_iters > 0:
        out["literal_loop"] = run_literal(args, ctx, student, views, targets, (tw, th), results)
    if args.stream_frames > 0:
        out["stream"] = run_stream(args, ctx)
    if args.serve_rates.strip():
        del student, teacher, targets
        torch.cuda.empty_cache()
        out["serving"] = run_serving(args, ctx, (tw, th), args.lds_batch)
        out["metric"] = ("window train steps/s (batched hipGraph step vs plain per-frame launches, same PSNR); "
                         "served frames/s at p99 ms (continuous batching vs plain FIFO, identical images)")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(S.steady_window_pool(args.num_gs, args.swin, args.sh_degree, st0, seed=0),
                                           views, args)
    print(json.dumps(out), flush=True)


MODES = {"graph": 2, "batched": 1, "plain": 0}


def run_forms(ctx, synth_pool, views, targets, tile, lds, cfg_base, forms, steps, warmup, reps, psnr_steps,
              breakdown=False, label="", headroom=1.5, inspect=False):
    """Train `synth_pool` on `views` in each launch structure of `forms` from
    the same initial state with the same seeds: `warmup` untimed steps, then
    `reps` timed runs of `steps` steps each (device synchronised around each
    run; the median run gives ms/step), then untimed steps up to `psnr_steps`
    in total, and the PSNR of the result over all views.  Every step writes
    its own stats row (relocated count, pairs, loss).  With `breakdown` the
    batched form also records per-kernel-class HIP-event times over its
    timed runs and counts the blend pairs in its last warm-up step."""
    import numpy as np
    import torch

    from paper_2409_07759_amd import swgs
    results = {}
    for name in forms:
        dp = swgs.Pool.from_synth(synth_pool)
        plan = swgs.Plan(ctx, dp, views, tile=tile, lds_batch=lds, headroom=headroom)
        cfg = swgs.step_cfg(mode=MODES[name], **cfg_base)
        n_rows = max(warmup + reps * steps, psnr_steps)
        st_all = torch.zeros((n_rows, 8), dtype=torch.float64, device="cuda")
        step = 0
        counts = None
        for w in range(warmup):
            count = breakdown and name == "batched" and w == warmup - 1
            if count:
                plan.set_timing(swgs.SWGS_TIMING_COUNT)
            plan.window_step(cfg, targets, step + 1, step, 2, stats=st_all[step])
            if count:
                counts = plan.timing()[1]
                plan.set_timing(0)
            step += 1
        torch.cuda.synchronize()
        if breakdown and name == "batched":
            plan.set_timing(swgs.SWGS_TIMING_EVENTS)
        rep_ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                plan.window_step(cfg, targets, step + 1, step, 2, stats=st_all[step])
                step += 1
            torch.cuda.synchronize()
            rep_ms.append(1e3 * (time.perf_counter() - t) / steps)
        timing = None
        if breakdown and name == "batched":
            timing = plan.timing()[0]
            plan.set_timing(0)
        timed = slice(warmup, step)
        while step < psnr_steps:
            plan.window_step(cfg, targets, step + 1, step, 2, stats=st_all[step])
            step += 1
        st = st_all[:step].cpu().numpy()
        if (st[:, 6] != 0).any():
            raise RuntimeError(f"{label} {name}: pair capacity overflow or stale plan (flags {st[:, 6].max()})")
        img = plan.forward()
        torch.cuda.synchronize()
        mse = torch.mean((img - targets) ** 2).item()
        psnr = 10 * math.log10(1.0 / mse)
        ms = float(np.median(rep_ms))
        rel = st[timed, 5]
        r = dict(ms=ms, steps_per_s=1e3 / ms, rep_ms=[round(x, 4) for x in rep_ms], psnr=psnr, psnr_steps=step,
                 loss=float(st[-1, 3]), pairs=int(st[-1, 4]), relocated_per_step=float(rel.mean()),
                 relocated_steps_nonzero=int((rel > 0).sum()), relocated_first_step=int(st[0, 5]),
                 records=plan.n_records, pixels=plan.n_pixels, ws_gb=plan.ws_bytes / 1e9, timing=timing,
                 counts=counts, timed_steps=reps * steps)
        if inspect and not results:
            cnt = plan.buffer(swgs.SWGS_BUF_ACTIVE_COUNT).cpu().numpy()
            rng = plan.buffer(swgs.SWGS_BUF_TILE_RANGE).cpu().numpy().reshape(-1, 2).astype(np.int64)
            ln = rng[:, 1] - rng[:, 0]
            r["inspect"] = {"live_per_frame": [int(x) for x in cnt[:plan.n_groups]], "window_set": int(cnt[plan.n_groups]),
                            "tile_list_len": {"mean": round(float(ln.mean()), 1),
                                              "p99": int(np.percentile(ln, 99)), "max": int(ln.max())}}
        results[name] = r
        log(f"{label} {name}: {ms:.3f} ms/step (median of {reps} x {steps}), PSNR {psnr:.3f} dB after {step} "
            f"steps, pairs {r['pairs']}, relocated {r['relocated_per_step']:.1f}/step")
        plan.close()
        del dp, plan
        torch.cuda.empty_cache()
    return results


# Algorithmic work of the blend kernels per contributing (pixel, Gaussian)
# pair -- alpha >= 1/255 before the pixel stops -- in VALU lane operations
# (an FMA, a compare, a select, v_exp_f32, v_rcp_f32 each count one):
#  forward: offsets 2, quadratic form 4, exp 1, o*g 1, clamp 1, skip test 1,
#    1 - alpha 1, T (1 - alpha) 1, stop test 1, weight alpha T 1, colour 3 = 17
#  backward: the forward's first 10 (alpha recomputed), 1 - alpha and its
#    reciprocal 2, T recovery 1, g.c - g.W 4, dL/dalpha 1, weight 1, colour
#    terms 3, clamp select 1, opacity term 1, dL/dQ 1, offset products 2,
#    conic products 3, g.W update 1, T update 1, and one add per gradient
#    term into the Gaussian's sums 9 = 41
LANE_OPS_FWD, LANE_OPS_BWD = 17.0, 41.0
PEAK_LANE_OPS = 256 * 64 * 2.4e9 / 1e12   # T lane-ops/s: 256 CUs x 4 SIMD x 16 lanes, one op per lane per clock


def roofline_report(res, tile, lds):
    """Per-kernel-class ms per step, blend pair counts, and the roofline of
    the dominant kernel: contributing pairs x lane-ops per pair per launch
    over its average launch time, against the FP32 vector rate."""
    tm, counts = res["timing"], res["counts"]
    n_steps = max(1, res["timed_steps"])
    out = {"kernel_ms_per_step": {k: round(v[0] / n_steps, 4) for k, v in tm.items()}}
    dom = max(tm, key=lambda k: tm[k][0])
    avg_s = tm[dom][0] / max(1, tm[dom][1]) / 1e3
    if counts is None:
        return out
    ev_f, ev_b, n_bl = counts
    out["blend_pairs_per_step"] = {"fwd_evaluated": ev_f, "bwd_evaluated": ev_b, "contributing": n_bl}
    work = {"blend_fwd": n_bl * LANE_OPS_FWD, "blend_bwd": n_bl * LANE_OPS_BWD}
    per_kernel = {}
    for k, w in work.items():
        a = w / (tm[k][0] / max(1, tm[k][1]) / 1e3) / 1e12
        per_kernel[k] = {"achieved": round(a, 3), "frac": round(a / PEAK_LANE_OPS, 4),
                         "avg_launch_ms": round(tm[k][0] / max(1, tm[k][1]), 4)}
    out["blend_roofline"] = per_kernel
    if dom in work:
        ach = work[dom] / avg_s / 1e12
        ev = ev_b if dom == "blend_bwd" else ev_f
        out["roofline"] = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": round(PEAK_LANE_OPS, 2),
                           "unit": "T lane-ops/s", "frac": round(ach / PEAK_LANE_OPS, 4),
                           "traffic": measured_traffic(dom, tile[0], tile[1], lds),
                           "work_per_launch": int(work[dom]),
                           "work": f"contributing pairs x {int(LANE_OPS_BWD if dom == 'blend_bwd' else LANE_OPS_FWD)} "
                                   f"lane-ops (FMA = 1; peak 256 CU x 64 lanes x 2.4 GHz, packed FP32 off)",
                           "avg_launch_ms": round(avg_s * 1e3, 4),
                           "tiling_overhead": {"evaluated_per_contributing": round(ev / max(1, n_bl), 3),
                                               "evaluated_pairs": int(ev)}}
    else:
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": None, "traffic": None, "avg_launch_ms": round(avg_s * 1e3, 4)}
    return out


def summarize_forms(res, chosen, base="plain"):
    d = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()
             if kk not in ("timing", "counts", "timed_steps")} for k, v in res.items()}
    if chosen in res and base in res:
        d["speedup_vs_plain"] = round(res[chosen]["steps_per_s"] / res[base]["steps_per_s"], 3)
        d["psnr_delta_vs_plain_db"] = round(res[chosen]["psnr"] - res[base]["psnr"], 4)
    return d


def run_c1(args, ctx):
    """The tiny plain-method window: 2,000 Gaussians, SH degree 0, W = 3
    frames x 3 cameras at 128x96; targets rendered from a second seeded set.
    Captured graph against one launch sequence per view."""
    import torch

    from paper_2409_07759_amd import swgs
    from paper_2409_07759_amd import synth as S
    n = 2000
    birth, start, expire = S.lifespans_tiny(n, 0)
    student = S.Pool(n, 3, 0, S.make_gaussians(n, 0, 0), birth, start, expire)
    teacher = S.Pool(n, 3, 0, S.make_gaussians(n, 0, 1), birth, start, expire)
    views = S.ring_views([0, 1, 2], 3, 128, 96)
    tp = swgs.Pool.from_synth(teacher, train=False)
    tpl = swgs.Plan(ctx, tp, views)
    targets = tpl.forward()
    torch.cuda.synchronize()
    tpl.close()
    res = run_forms(ctx, student, views, targets, (16, 16), 0, dict(window_start=0, relocate_period=1),
                    ["graph", "plain"], args.c1_steps, 5, args.reps, 5 + args.reps * args.c1_steps, label="c1")
    out = summarize_forms(res, "graph")
    out["workload"] = "2000 Gaussians, SH degree 0, W=3 frames x 3 cameras at 128x96, relocation every step"
    return out


def run_c3(args, ctx):
    """The uneven window: a 500k-slot pool over 30 frames (40k Gaussians live
    in every frame, 460k start at U{0..29} and live U{1..27} frames), SH
    degree 3, 6 cameras per frame (960x720 and 1352x1014 alternating): 180
    views per step, tile shape and LDS batch autotuned over {8x8, 16x16,
    32x8} x {128, 256}; captured graph against one launch sequence per view,
    PSNR after the same 50-odd steps."""
    import torch

    from paper_2409_07759_amd import autotune, swgs
    from paper_2409_07759_amd import synth as S
    sizes = [(960, 720), (1352, 1014)] * 3
    student = S.uneven_window_pool(500_000, 40_000, 30, 3, 5)
    teacher = S.uneven_window_pool(500_000, 40_000, 30, 3, 6)
    views = S.ring_views(list(range(30)), 6, 0, 0, sizes=sizes)
    tp = swgs.Pool.from_synth(teacher, train=False)
    tpl = swgs.Plan(ctx, tp, views)
    targets = tpl.forward()
    torch.cuda.synchronize()
    tpl.close()
    del tp
    if args.c3_tile == "auto":
        dp = swgs.Pool.from_synth(student)
        cands = [((8, 8), 128), ((8, 8), 256), ((16, 16), 128), ((16, 16), 256), ((32, 8), 128), ((32, 8), 256)]
        tile, lds, table = autotune.tune(ctx, dp, views, reps=1, use_cache=False, candidates=cands, log=log)
        del dp
        torch.cuda.empty_cache()
    else:
        ts, ls = args.c3_tile.split("/")
        tile, lds, table = tuple(int(x) for x in ts.split("x")), int(ls), []
    res = run_forms(ctx, student, views, targets, tile, lds, dict(window_start=0, relocate_period=1),
                    [f.strip() for f in args.c3_forms.split(",")], args.c3_steps, 3, args.reps,
                    3 + args.reps * args.c3_steps, label="c3", inspect=True, breakdown=True)
    out = summarize_forms(res, "graph")
    if "batched" in res and res["batched"]["timing"]:
        out["kernel_ms_per_step_batched"] = {k: round(v[0] / max(1, res["batched"]["timed_steps"]), 4)
                                             for k, v in res["batched"]["timing"].items()}
    first = res[list(res)[0]]
    live = first.get("inspect", {}).get("live_per_frame", [])
    out["workload"] = ("500k-slot pool, 30 frames x 6 cameras (960x720 / 1352x1014), uneven live sets, SH degree 3, "
                       "relocation every step")
    out["tile"], out["lds_batch"] = f"{tile[0]}x{tile[1]}", lds
    out["autotune_ms_fwd_bwd"] = {f"{t[0]}x{t[1]}/lds{l}": ms for t, l, ms in table}
    if live:
        out["live_min_max"] = [min(live), max(live)]
    return out


def run_c5(args, ctx):
    """The long video: a constant pool of 1M optimisable Gaussians (plus the
    1M-slot frozen store), SH degree 3, window W = 10 x 4 cameras at
    1352x1014.  Each advance runs one window step (I = 1), then mature(st+1)
    emits the packed per-frame update of the slice born at st and the next
    window's plan is made.  Device memory is sampled after every advance.
    The batched form (one launch per kernel over the window; a graph would
    be captured for a single replay per window) against one launch sequence
    per view.  The teacher is static (every Gaussian live in every frame),
    so its renders of the 4 cameras are every frame's targets, resident as
    one W x C buffer."""
    import numpy as np
    import torch

    from paper_2409_07759_amd import swgs
    from paper_2409_07759_amd import synth as S
    num_gs, swin, deg, cams, W, H, st0 = 1_000_000, 10, 3, 4, 1352, 1014, 10
    n_adv = args.c5_advances
    base = S.steady_window_pool(num_gs, swin, deg, st0, seed=21)
    S.add_faint_gaussians(base, args.dead_fraction, seed=22)
    tpar = S.make_gaussians(num_gs, deg, 23)
    big = np.int32(1 << 30)
    tp = swgs.Pool(tpar, np.zeros(num_gs, np.int32), np.zeros(num_gs, np.int32), np.full(num_gs, big, np.int32),
                   0, swin, deg, "cuda", train=False)
    cam_views = S.ring_views([st0], cams, W, H, phase_deg=10.0)
    tpl = swgs.Plan(ctx, tp, cam_views)
    t4 = tpl.forward()
    torch.cuda.synchronize()
    tpl.close()
    del tp, tpar
    targets = t4.repeat(swin)
    del t4
    res = {}
    for name in ("batched", "plain"):
        dp = swgs.Pool.from_synth(base)
        cfg = swgs.step_cfg(mode=MODES[name], relocate_period=1)
        stats = torch.zeros((n_adv, 8), dtype=torch.float64, device="cuda")
        views0 = S.ring_views(list(range(st0, st0 + swin)), cams, W, H, phase_deg=10.0)
        probe = swgs.Plan(ctx, dp, views0)
        cap = int(probe.measure() * 1.5) + 65536
        probe.close()
        del probe
        torch.cuda.empty_cache()
        used, t_step, t_adv, rec_bytes = [], [], [], []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for k in range(n_adv):
            t0 = time.perf_counter()
            st = st0 + k
            views = S.ring_views(list(range(st, st + swin)), cams, W, H, phase_deg=10.0)
            plan = swgs.Plan(ctx, dp, views, pair_capacity=cap)
            cfg.window_start = st
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            plan.window_step(cfg, targets, k + 1, k, 5, stats=stats[k])
            torch.cuda.synchronize()
            t_step.append(time.perf_counter() - t1)
            if k == n_adv - 1:
                # the PSNR render (its image buffer is not part of the loop)
                img = plan.forward()
                mse = torch.mean((img - targets) ** 2).item()
                del img
            plan.close()
            del plan
            rec, cnt = swgs.mature(ctx, dp, st + 1)
            rec_bytes.append(rec.numel())
            del rec
            torch.cuda.synchronize()
            t_adv.append(time.perf_counter() - t0)
            if k < n_adv - 1:
                free, total = torch.cuda.mem_get_info()
                used.append(total - free)
            if k % 50 == 0:
                log(f"c5 {name}: advance {k}, step {1e3 * t_step[-1]:.1f} ms, advance {1e3 * t_adv[-1]:.1f} ms")
        wall = time.perf_counter() - t_all
        s = stats.cpu().numpy()
        if (s[:, 6] != 0).any():
            raise RuntimeError(f"c5 {name}: pair capacity overflow or stale plan")
        u = np.array(used[1:], np.float64)        # after the first advance (first-use allocations)
        res[name] = {"ms": float(np.median(t_step)) * 1e3, "steps_per_s": 1.0 / float(np.median(t_step)),
                     "advance_ms": float(np.median(t_adv)) * 1e3, "sustained_advances_per_s": n_adv / wall,
                     "psnr": 10 * math.log10(1.0 / mse), "psnr_steps": n_adv,
                     "record_bytes": int(np.median(rec_bytes)), "relocated_per_step": float(s[:, 5].mean()),
                     "device_bytes_min_max": [int(u.min()), int(u.max())],
                     "device_bytes_spread": float((u.max() - u.min()) / u.max())}
        log(f"c5 {name}: {res[name]}")
        del dp
        torch.cuda.empty_cache()
    out = summarize_forms(res, "batched")
    out["workload"] = (f"1M optimisable + 1M frozen Gaussians, SH degree 3, W=10 x 4 cameras at 1352x1014; "
                       f"{n_adv} advances measured (each: plan, window step, mature/emit), a 3,000-frame run is "
                       f"3000/{n_adv} times longer at the same per-advance cost")
    return out


def measured_traffic(kernel, tw, th, lds):
    """HBM bytes per launch of `kernel` measured by rocprofv3 counters
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size), as
    recorded in profiles/hbm_traffic.json for this workload -- or None when
    the kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        src = os.path.join(ROOT, "paper_2409_07759_amd", "csrc", "kernels_blend.hip")
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        e = rec["kernels"].get(f"{kernel}@{lds}")
        if e is None or rec["source_sha256"] != digest or e["config"] != f"{tw}x{th}/lds{lds}":
            return None
        return round(e["bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


RESOLUTIONS = [(640, 480), (1280, 720), (1920, 1080)]


def serving_trace(rate, seconds, n_frames, seed):
    """Poisson arrivals at `rate` req/s over 1 s of warm-up plus `seconds`;
    each request: frame U{0..n_frames-1}, camera uniform on a sphere of
    radius U[3, 5] looking at the origin, resolution uniform over
    RESOLUTIONS."""
    import numpy as np

    from paper_2409_07759_amd import synth as S
    rng = np.random.default_rng(seed)
    arr = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > 1.0 + seconds:
            break
        arr.append(t)
    views = []
    for _ in arr:
        W, H = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
        views.append(S.random_pose_view(rng, int(rng.integers(0, n_frames)), W, H))
    return np.array(arr), views


def latency_summary(arr, ready, status, t_lo):
    import numpy as np
    m = (arr >= t_lo) & (status == 0)
    lat = (ready[m] - arr[m]) * 1e3
    if lat.size == 0:
        return dict(p50_ms=None, p99_ms=None, frames_per_s=0.0, completed=0)
    span = ready[m].max() - arr[m].min()
    return dict(p50_ms=round(float(np.percentile(lat, 50)), 3), p99_ms=round(float(np.percentile(lat, 99)), 3),
                mean_ms=round(float(lat.mean()), 3), frames_per_s=round(float(m.sum() / span), 2),
                completed=int(m.sum()), failed=int(((arr >= t_lo) & (status != 0)).sum()))


def run_literal(args, ctx, student, views, targets, tile, results):
    """The paper's own loop (Algorithm 1's train_swin) on the same window:
    one sampled (frame, camera) per iteration (Adam + SGLD + relocation at
    its cadence), against the window step that takes all views at once."""
    import torch

    from paper_2409_07759_amd import swgs
    dp = swgs.Pool.from_synth(student)
    t0 = time.time()
    tr = swgs.Trainer(ctx, dp, views, tile=tile, lds_batch=args.lds_batch)
    t_setup = time.time() - t0
    HW = [3 * v.width * v.height for v in views]
    offs = [0]
    for n in HW:
        offs.append(offs[-1] + n)
    tgts = [targets[offs[i]:offs[i + 1]] for i in range(len(views))]
    cfg = swgs.step_cfg(window_start=views[0].frame, relocate_period=100)
    tr.run(cfg, tgts, 10, 0, 5)
    torch.cuda.synchronize()
    n = args.literal_iters
    stats = torch.zeros(8 * n, dtype=torch.float64, device="cuda")
    t = time.perf_counter()
    tr.run(cfg, tgts, n, 10, 5, stats=stats)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    tr.close()
    ips = n / el
    st = stats.view(n, 8).cpu()
    res = {"iterations_per_s": round(ips, 2), "ms_per_iteration": round(1e3 * el / n, 3),
           "views": len(views), "setup_s": round(t_setup, 2),
           "paper_window_2000_iterations_s": round(2000 / ips, 3),
           "views_per_s": round(ips, 1),
           "window_step_views_per_s": round(len(views) * results.get("graph", results[list(results)[0]])["steps_per_s"], 1),
           "loss_first_last": [round(float(st[0, 3]), 5), round(float(st[-1, 3]), 5)],
           "overflow": bool(st[:, 6].max() > 0)}
    log(f"literal loop: {res}")
    del dp
    torch.cuda.empty_cache()
    return res


def run_stream(args, ctx):
    """The update stream of a 200K-Gaussian model with swin 5 (Sec. 5.2's
    configuration: 40K Gaussians per frame): record sizes per frame (full,
    FP32 DC-only, Table 6), GPU encode and decode times, client playback
    (Algorithm 2) with the next record's transfer overlapped with rendering
    against a serialized client, and the rate-distortion of Table 6's
    quantisation and Sec. 5.5's tail-drop (PSNR of the client render against
    the FP32 DC-only client)."""
    import numpy as np
    import torch

    from paper_2409_07759_amd import swgs
    from paper_2409_07759_amd import synth as S
    num_gs, swin, deg, st0, n = 200_000, 5, args.sh_degree, 7, args.stream_frames
    pool = S.steady_window_pool(num_gs, swin, deg, st0, seed=11)
    dp = swgs.Pool.from_synth(pool)
    W, H = args.width, args.height

    def client():
        # the client's first read: the live window at st0 (DC-only buffer)
        return swgs.Pool(np.ascontiguousarray(pool.params[:14, :num_gs]), pool.birth[:num_gs].copy(),
                         pool.start[:num_gs].copy(), pool.expire[:num_gs].copy(), 0, swin, 0, "cuda", train=False)

    encs = {"fp32": (swgs.SWGS_ENC_FP32, -1), "table6": (swgs.SWGS_ENC_Q, -1)}
    for f in (0.75, 0.5, 0.25):
        encs[f"table6_keep{f}"] = (swgs.SWGS_ENC_Q, f)
    recs = {k: [] for k in encs}
    full_bytes, t_enc = [], {k: 0.0 for k in encs}
    for st in range(st0 + 1, st0 + 1 + n):
        rec, cnt = swgs.mature(ctx, dp, st)
        full_bytes.append(rec.numel())
        for k, (e, kf) in encs.items():
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = swgs.encode_update(ctx, rec, e, -1 if kf < 0 else int(cnt * kf))
            torch.cuda.synchronize()
            t_enc[k] += time.perf_counter() - t
            recs[k].append(out)
    frames = list(range(st0, st0 + n))          # record i is due at frame st0 + i
    cap = 4 * num_gs * 8
    view = lambda fr: S.ring_views([fr], 1, W, H)[0]

    def render(buf, fr):
        pl = swgs.Plan(ctx, buf, [view(fr)], pair_capacity=cap)
        img = pl.forward()
        pl.close()
        return img

    # client playback: push the next record (transfer on the copy stream) and render the current frame
    host_recs = [r.cpu().numpy() for r in recs["table6"]]
    buf = client()
    player = swgs.Player(ctx, buf, queue_depth=4, max_record_bytes=max(h.nbytes for h in host_recs))
    player.push(host_recs[0])
    render(buf, frames[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i, fr in enumerate(frames):
        if i + 1 < n:
            player.push(host_recs[i + 1])
        player.advance(fr)
        render(buf, fr)
    torch.cuda.synchronize()
    t_play = (time.perf_counter() - t) / n
    player.close()
    # serialized client: synchronous transfer, apply, render
    buf2 = client()
    torch.cuda.synchronize()
    t = time.perf_counter()
    t_h2d = t_dec = 0.0
    for i, fr in enumerate(frames):
        a = time.perf_counter()
        d = torch.from_numpy(host_recs[i]).cuda()
        torch.cuda.synchronize()
        b = time.perf_counter()
        swgs.apply_update(ctx, buf2, d)
        c = time.perf_counter()
        render(buf2, fr)
        t_h2d += b - a
        t_dec += c - b
    torch.cuda.synchronize()
    t_ser = (time.perf_counter() - t) / n
    same = bool(torch.equal(render(buf, frames[-1]), render(buf2, frames[-1])))
    # rate-distortion at the last frame (every slice replaced once n >= swin)
    imgs = {}
    for k in encs:
        b = client()
        for r in recs[k]:
            swgs.apply_update(ctx, b, r)
        imgs[k] = render(b, frames[-1])
    ref = imgs["fp32"]
    rd = {}
    for k, img in imgs.items():
        mse = float(torch.mean((img - ref) ** 2))
        rd[k] = {"mb_per_frame": round(float(np.mean([r.numel() for r in recs[k]])) / 1e6, 4),
                 "psnr_vs_fp32_db": None if mse == 0 else round(10 * math.log10(1.0 / mse), 2)}
    res = {"workload": f"{num_gs} Gaussians, swin {swin} ({num_gs // swin} per frame), trainer SH degree {deg}, "
                       f"DC-only client; {n} frames from frame {st0}; client renders one {W}x{H} view per frame",
           "bytes_per_frame": {"full_record": int(np.mean(full_bytes)),
                               "fp32_dc": int(np.mean([r.numel() for r in recs["fp32"]])),
                               "table6": int(np.mean([r.numel() for r in recs["table6"]]))},
           "paper_mb_per_frame": {"fp32_dc": 2.1, "table6": 1.2},
           "encode_ms": {k: round(1e3 * v / n, 3) for k, v in t_enc.items()},
           "playback_ms_per_frame": {"player_overlapped": round(1e3 * t_play, 3), "serialized": round(1e3 * t_ser, 3),
                                     "serialized_transfer": round(1e3 * t_h2d / n, 3),
                                     "serialized_apply": round(1e3 * t_dec / n, 3)},
           "player_equals_serialized": same,
           "rate_distortion": rd}
    log(f"stream: {res['bytes_per_frame']}, playback {res['playback_ms_per_frame']}, rd {rd}")
    del dp
    torch.cuda.empty_cache()
    return res


def run_serving(args, ctx, tile, lds):
    """Serving of a 300-frame clip from a resident pool (300k live per frame,
    1-2% replaced per frame): continuous batching (lanes x batches of mixed
    resolutions, admission by memory budget) against the plain form (FIFO,
    one request per launch sequence, one in flight)."""
    import numpy as np
    import torch

    from paper_2409_07759_amd import swgs
    from paper_2409_07759_amd import synth as S
    t0 = time.time()
    pool = S.serving_pool(args.serve_active, args.serve_frames, args.sh_degree, seed=3)
    dp = swgs.Pool.from_synth(pool, train=False)
    n_slots = pool.params.shape[1]
    del pool
    log(f"serving pool: {n_slots} resident slots, {args.serve_frames} frames, built in {time.time() - t0:.1f}s")
    budget = int(args.serve_budget_gb * (1 << 30))
    forms = {"served": dict(lanes=args.serve_lanes, max_batch=args.serve_max_batch),
             "plain": dict(lanes=1, max_batch=1)}
    servers = {k: swgs.Server(ctx, dp, args.serve_frames, budget + (512 << 20), tile=tile, lds_batch=lds, **v)
               for k, v in forms.items()}
    # same images from both forms (sampled requests)
    _, views = serving_trace(100.0, 0.1, args.serve_frames, seed=99)
    views = views[:8]
    imgs = {k: [torch.empty((3, v.height, v.width), device="cuda") for v in views] for k in forms}
    for k, srv in servers.items():
        srv.run(views, images=imgs[k])
    diff = max(float((a - b).abs().max()) for a, b in zip(imgs["served"], imgs["plain"]))
    del imgs
    res = {"workload": f"{args.serve_frames}-frame clip, {args.serve_active} live Gaussians per frame, 1-2% "
                       f"replaced per frame ({n_slots} resident slots), SH degree {args.sh_degree}; Poisson "
                       f"arrivals, frame U{{0..{args.serve_frames - 1}}}, pose on a sphere of radius U[3,5], "
                       f"resolution uniform over 640x480/1280x720/1920x1080; forward only, FP32",
           "served_form": f"continuous batching: {args.serve_lanes} lanes, <= {args.serve_max_batch} requests per "
                          f"batch, memory budget {args.serve_budget_gb} GB",
           "plain_form": "FIFO, one request per launch sequence, one in flight",
           "measured_seconds_per_rate": args.serve_seconds, "warmup_seconds": 1.0,
           "served_vs_plain_max_abs_diff": diff, "rates": {}}
    for rate in [float(r) for r in args.serve_rates.split(",") if r.strip()]:
        arr, views = serving_trace(rate, args.serve_seconds, args.serve_frames, seed=int(rate))
        row = {}
        for k, srv in servers.items():
            (a, ready, status, batch), st = srv.run(views, arrivals=arr, realtime=True)
            summ = latency_summary(a, ready, status, 1.0)
            summ.update(batches=st["batches"], mean_batch=round(st["mean_batch"], 2), redone=st["redone"],
                        peak_gb=round(st["peak_bytes"] / 1e9, 3))
            row[k] = summ
            log(f"serve {rate:.0f} req/s {k}: p50 {summ['p50_ms']} ms, p99 {summ['p99_ms']} ms, "
                f"{summ['frames_per_s']} frames/s, mean batch {summ['mean_batch']}, redone {st['redone']}")
        if row["served"]["p99_ms"] and row["plain"]["p99_ms"]:
            row["p99_speedup_vs_plain"] = round(row["plain"]["p99_ms"] / row["served"]["p99_ms"], 3)
        res["rates"][str(int(rate))] = row
    # saturation: every request queued at once (capacity of each form)
    _, views = serving_trace(2000.0, 0.5, args.serve_frames, seed=7)
    sat = {}
    for k, srv in servers.items():
        (a, ready, status, batch), st = srv.run(views)
        ok = int((status == 0).sum())
        sat[k] = dict(requests=len(views), completed=ok, frames_per_s=round(ok / st["wall_s"], 2),
                      mean_batch=round(st["mean_batch"], 2), redone=st["redone"])
        log(f"serve saturation {k}: {sat[k]['frames_per_s']} frames/s over {len(views)} requests, "
            f"mean batch {sat[k]['mean_batch']}")
    sat["speedup_vs_plain"] = round(sat["served"]["frames_per_s"] / sat["plain"]["frames_per_s"], 3)
    res["saturation"] = sat
    for srv in servers.values():
        srv.close()
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads(args):
    if args.cpu_threads > 0:
        return args.cpu_threads
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_c2_sample(O, student, views, pixels, seed):
    """One view of the paper-scale window in the FP64 oracle: preprocess of
    every slot, forward and adjoint of `pixels` random pixels (brute force
    over every visible Gaussian in depth order), adjoint preprocess of every
    visible optimisable slot; returns seconds per part."""
    import numpy as np
    v = views[0]
    rng = np.random.default_rng(seed)
    P = v.width * v.height
    pix = rng.choice(P, size=min(pixels, P), replace=False)
    t = time.perf_counter()
    vis, rec, _ = O.preprocess(student.params, student.sh_degree, student.start, student.expire, v)
    t_pre = time.perf_counter() - t
    t = time.perf_counter()
    O.render_records(vis, rec, v, pixels=pix)
    t_fwd = time.perf_counter() - t
    t = time.perf_counter()
    drec = O.blend_backward_pixels(vis, rec, v, pix, rng.uniform(-1, 1, size=(3, len(pix))))
    t_bwd = time.perf_counter() - t
    t = time.perf_counter()
    O.preprocess_backward_visible(student.params, student.sh_degree, v, drec, vis, student.num_gs)
    t_pb = time.perf_counter() - t
    return dict(pre=t_pre, fwd=t_fwd, bwd=t_bwd, pb=t_pb, pixels=len(pix), P=P)


def cpu_c1_full(O):
    """The tiny window in full in the FP64 oracle: 9 views of 128x96 from
    2,000 Gaussians -- render, L1 + D-SSIM loss and gradient, adjoint, the
    adjoint preprocess, Adam + SGLD and relocation; seconds."""
    import numpy as np

    from paper_2409_07759_amd import synth as S
    n = 2000
    params = S.make_gaussians(n, 0, 0)
    birth, start, expire = S.lifespans_tiny(n, 0)
    views = S.ring_views([0, 1, 2], 3, 128, 96)
    tgt = S.random_images(views, 1)
    t = time.perf_counter()
    img, _ = O.window_render(params, 0, start, expire, views)
    A = O.window_set(start, expire, n, [0, 1, 2])
    L, _, g, dreg = O.loss_and_grad(img, tgt, views, params, A, lam_dssim=0.2)
    grads = dreg.copy()
    o = 0
    for v in views:
        m = 3 * v.width * v.height
        vis, rec, _ = O.preprocess(params, 0, start, expire, v)
        drec = O.blend_backward(vis, rec, v, g[o:o + m].reshape(3, -1))
        grads += O.preprocess_backward_visible(params, 0, v, drec, vis, n)
        o += m
    Z = np.zeros_like(grads)
    P2, M2, V2 = O.adam_sgld_step(params, grads, Z, Z, A, 1, 0, seed=2, step=0)
    O.relocate(P2, M2, V2, A, 2, 0)
    return time.perf_counter() - t


def cpu_baseline(student, views, args):
    """The FP64 oracle on the host cores: the paper-scale step from a
    bounded sample (one view's preprocess of every slot, forward and adjoint
    of random pixels, adjoint preprocess of the visible slots; scaled to all
    40 views x 1.37M pixels, plus the numpy Adam step), single-threaded and
    with every host core (OpenMP over slots and pixels); and the tiny window
    (config 1) timed in full both ways."""
    import numpy as np

    import oracle as O
    nt = host_threads(args)
    F = student.params.shape[0]
    rng = np.random.default_rng(0)
    g = rng.normal(size=(F, student.num_gs)) * 1e-3
    A = np.ones(student.num_gs, bool)
    t = time.perf_counter()
    O.adam_sgld_step(student.params[:, :student.num_gs], g, np.zeros_like(g), np.zeros_like(g), A, 1,
                     student.sh_degree, 0, 0, noise_lr=0.0)
    t_adam = time.perf_counter() - t
    legs = {}
    for threads, px in ((1, args.cpu_pixels), (nt, args.cpu_pixels * max(1, nt // 2))):
        O.set_threads(threads)
        try:
            smp = cpu_c2_sample(O, student, views, px, 0)
            c1 = cpu_c1_full(O)
        finally:
            O.set_threads(1)
        per_view = smp["pre"] + (smp["P"] / smp["pixels"]) * (smp["fwd"] + smp["bwd"]) + smp["pb"]
        step_s = len(views) * per_view + t_adam
        legs[threads] = dict(step_s=step_s, sample_s=smp["pre"] + smp["fwd"] + smp["bwd"] + smp["pb"],
                             pixels=smp["pixels"], c1_s=c1)
        log(f"cpu oracle, {threads} thread(s): c2 sample {legs[threads]['sample_s']:.1f}s "
            f"({smp['pixels']} px) -> {step_s:.0f} s/step; c1 window step in full {c1:.2f}s")
        if nt == 1:
            break
    best = legs[nt]
    return {"value": 1.0 / best["step_s"], "unit": "window steps/s", "cores": nt, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"1 of {len(views)} views: preprocess of all {student.slots} slots, forward+adjoint of "
                      f"{best['pixels']} random pixels of {views[0].width * views[0].height} (brute force over "
                      f"every visible Gaussian), adjoint preprocess of the visible slots, dense numpy Adam step; "
                      f"scaled to {len(views)} views x all pixels",
            "sample_seconds": round(best["sample_s"] + t_adam, 2),
            "single_thread": {"value": 1.0 / legs[1]["step_s"], "sample_seconds": round(legs[1]["sample_s"], 2),
                              "pixels": legs[1]["pixels"]},
            "c1_full_step_s": {"1": round(legs[1]["c1_s"], 3), str(nt): round(best["c1_s"], 3)},
            "c1_steps_per_s": {"1": round(1.0 / legs[1]["c1_s"], 4), str(nt): round(1.0 / best["c1_s"], 4)}}


if __name__ == "__main__":
    main()
