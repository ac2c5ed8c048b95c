#!/usr/bin/env python3
"""Benchmark of the sliding-window Gaussian-splatting hot path on one MI355X.

Workload (default): the paper-scale window step -- 200k optimisable
Gaussians plus their 200k-slot frozen store, SH degree 3, a window of 10
frames x 4 cameras at 1352x1014, every frame with exactly 200k live slots
(10% retire and 10% are born per frame).  One step = forward of all 40
views with the fused L1 gradient, backward, Adam + SGLD, relocation.

The step runs in three launch structures on the same inputs and the same
number of steps from the same initial state: GRAPH (chosen form: the batched
sequence captured once in a hipGraph), BATCHED (one launch per kernel over
all views; its timed region also yields the per-kernel HIP-event breakdown)
and PLAIN (one launch sequence per view with a host read-back of each
view's pair count, the per-frame baseline).  `value` is GRAPH window
steps/s.  The PSNR of each form after the run shows they train equally.

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
PEAK_FP32_NONPACKED = 78.6     # TFLOP/s: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, no packed FP32
# Algorithmic FP32 work of the blend kernels, counted from the math (FMA = 2):
#  every evaluated (pixel, splat) pair: offsets 4, quadratic form 7, exp 1,
#    o*g 1, min 1, alpha test 1                                        = 15
#  forward, per blended pair: 1-alpha 1, T(1-alpha) 1, stop test 1,
#    w = alpha T 1, colour 3 FMA 6                                     = 10
#  backward, per blended pair: T recovery (rcp, mul) 2, dC/dalpha 3 x 5,
#    colour grads 4, U update 3 x 3, prod 1, dQ 2, opacity 1, conic and
#    offset terms 5                                                    = 40
FLOPS_EVAL, FLOPS_FWD_BLEND, FLOPS_BWD_BLEND = 15.0, 10.0, 40.0


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
    ap.add_argument("--serve-rates", default="200,500,1000", help="Poisson request rates (req/s); empty: no serving")
    ap.add_argument("--serve-seconds", type=float, default=5.0, help="measured seconds per rate (after 1 s warm-up)")
    ap.add_argument("--serve-active", type=int, default=300_000)
    ap.add_argument("--serve-frames", type=int, default=300)
    ap.add_argument("--serve-lanes", type=int, default=3)
    ap.add_argument("--serve-max-batch", type=int, default=16)
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--stream-frames", type=int, default=10, help="frames of the update-stream run; 0: skip it")
    ap.add_argument("--literal-iters", type=int, default=200,
                    help="timed iterations of the paper's one-view-per-iteration loop; 0: skip it")
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
    cfg_base = dict(window_start=st0, relocate_period=1)
    results = {}
    pool_for = {}

    def run_mode(mode_name):
        mode = {"graph": swgs.SWGS_MODE_GRAPH, "batched": swgs.SWGS_MODE_BATCHED, "plain": swgs.SWGS_MODE_PLAIN}[mode_name]
        dp = swgs.Pool.from_synth(student)
        plan = swgs.Plan(ctx, dp, views, tile=(tw, th), lds_batch=args.lds_batch, headroom=1.5)
        cfg = swgs.step_cfg(mode=mode, **cfg_base)
        stats = torch.zeros(8, dtype=torch.float64, device=dev)
        step = 0
        counts = None
        for w in range(args.warmup):
            # the batched form's last warm-up step counts the blend pairs (in
            # the forward's counting build); the timed steps run uncounted
            count = mode_name == "batched" and w == args.warmup - 1
            if count:
                plan.set_timing(swgs.SWGS_TIMING_COUNT)
            plan.window_step(cfg, targets, step + 1, step, 2, stats=stats)
            if count:
                counts = plan.timing()[1]
                plan.set_timing(0)
            step += 1
        torch.cuda.synchronize()
        timing = None
        if mode_name == "batched":
            plan.set_timing(swgs.SWGS_TIMING_EVENTS)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            plan.window_step(cfg, targets, step + 1, step, 2, stats=stats)
            step += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        if mode_name == "batched":
            timing = (plan.timing()[0], counts)
            plan.set_timing(0)
        st = stats.cpu().numpy()
        if st[6] != 0:
            raise RuntimeError(f"{mode_name}: pair capacity overflow")
        # PSNR of the trained state over all window views
        img = plan.forward()
        torch.cuda.synchronize()
        mse = torch.mean((img - targets) ** 2).item()
        psnr = 10 * math.log10(1.0 / mse)
        results[mode_name] = dict(ms=1e3 * el / args.steps, steps_per_s=args.steps / el, psnr=psnr,
                                  loss=float(st[3]), pairs=int(st[4]), relocated=int(st[5]), timing=timing,
                                  records=plan.n_records, pixels=plan.n_pixels, ws_gb=plan.ws_bytes / 1e9)
        log(f"{mode_name}: {1e3 * el / args.steps:.2f} ms/step, {args.steps / el:.2f} steps/s, PSNR {psnr:.3f} dB, "
            f"pairs {int(st[4])}, relocated {int(st[5])}")
        plan.close()
        del dp

    for m in args.modes.split(","):
        run_mode(m.strip())

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
                        f"{args.width}x{args.height}, Adam+SGLD+relocation every step",
            "views": len(views), "tile": f"{tw}x{th}", "lds_batch": args.lds_batch, "form": chosen,
        },
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items() if kk != "timing"}
                  for k, v in results.items()},
    }
    if "plain" in results:
        out["speedup_vs_plain"] = round(results[chosen]["steps_per_s"] / results["plain"]["steps_per_s"], 3)
        out["psnr_delta_vs_plain_db"] = round(results[chosen]["psnr"] - results["plain"]["psnr"], 4)
    if tune_table:
        out["autotune_ms_fwd_bwd"] = {f"{t[0]}x{t[1]}/lds{l}": ms for t, l, ms in tune_table}
    if "batched" in results and results["batched"]["timing"]:
        tm, counts = results["batched"]["timing"]
        per_step = {k: round(v[0] / max(1, args.steps), 4) for k, v in tm.items()}
        out["kernel_ms_per_step"] = per_step
        dom = max(tm, key=lambda k: tm[k][0])
        n_launch = max(1, tm[dom][1])
        avg_s = tm[dom][0] / n_launch / 1e3
        blend_work = {}
        if counts is not None:
            # pairs of one step; launches per step from the timed run
            ev_f, ev_b, n_bl = counts
            per = lambda k: max(1, tm[k][1]) / max(1, args.steps)
            blend_work = {"blend_fwd": (ev_f * FLOPS_EVAL + n_bl * FLOPS_FWD_BLEND) / per("blend_fwd"),
                          "blend_bwd": (ev_b * FLOPS_EVAL + n_bl * FLOPS_BWD_BLEND) / per("blend_bwd")}
            out["blend_pairs_per_step"] = {"fwd_evaluated": ev_f, "bwd_evaluated": ev_b, "blended": n_bl}
        if dom in blend_work:
            ach = blend_work[dom] / avg_s / 1e12
            out["roofline"] = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": PEAK_FP32_NONPACKED,
                               "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_NONPACKED, 4),
                               "traffic": measured_traffic(dom, tw, th, args.lds_batch),
                               "flops_per_launch": int(blend_work[dom]), "avg_launch_ms": round(avg_s * 1e3, 4)}
        else:
            out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": None, "traffic": None, "avg_launch_ms": round(avg_s * 1e3, 4)}
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


def cpu_baseline(student, views, args):
    """The FP64 oracle, single-threaded, on a bounded sample of the same step:
    one view's preprocess of every slot, forward and adjoint of `cpu_pixels`
    random pixels, the adjoint preprocess of every visible slot; scaled to a
    full window step (all views, all pixels) plus the numpy Adam step."""
    import numpy as np

    import oracle as O

    v = views[0]
    rng = np.random.default_rng(0)
    P = v.width * v.height
    pix = rng.choice(P, size=min(args.cpu_pixels, P), replace=False)
    t = time.perf_counter()
    vis, rec, _ = O.preprocess(student.params, student.sh_degree, student.start, student.expire, v)
    t_pre = time.perf_counter() - t
    t = time.perf_counter()
    O.render_records(vis, rec, v, pixels=pix)
    t_fwd = time.perf_counter() - t
    t = time.perf_counter()
    drec = O.blend_backward_pixels(vis, rec, v, pix, rng.uniform(-1, 1, size=(3, len(pix))))
    t_bwd = time.perf_counter() - t
    slots = np.nonzero(vis[:student.num_gs])[0]
    sub = slots[: min(len(slots), 20000)]
    t = time.perf_counter()
    O.preprocess_backward(student.params, student.sh_degree, v, drec, sub)
    t_pb = (time.perf_counter() - t) * (len(slots) / max(1, len(sub)))
    F = student.params.shape[0]
    g = rng.normal(size=(F, student.num_gs)) * 1e-3
    A = np.ones(student.num_gs, bool)
    t = time.perf_counter()
    O.adam_sgld_step(student.params[:, :student.num_gs], g, np.zeros_like(g), np.zeros_like(g), A, 1,
                     student.sh_degree, 0, 0, noise_lr=0.0)
    t_adam = time.perf_counter() - t
    per_view = t_pre + (P / len(pix)) * (t_fwd + t_bwd) + t_pb
    step_s = len(views) * per_view + t_adam
    sample_s = t_pre + t_fwd + t_bwd + t_pb * len(sub) / max(1, len(slots)) + t_adam
    log(f"cpu oracle: preprocess {t_pre:.2f}s, fwd {t_fwd:.2f}s + bwd {t_bwd:.2f}s for {len(pix)} px, "
        f"adjoint preprocess {t_pb:.2f}s (extrapolated), adam {t_adam:.2f}s -> {step_s:.0f} s/step")
    return {"value": 1.0 / step_s, "unit": "window steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 of {len(views)} views: preprocess of all {student.slots} slots, forward+adjoint of "
                      f"{len(pix)} random pixels of {P}, adjoint preprocess of {len(sub)} of {len(slots)} visible "
                      f"slots, dense Adam step; scaled to {len(views)} views x {P} pixels",
            "sample_seconds": round(sample_s, 2)}


if __name__ == "__main__":
    main()
