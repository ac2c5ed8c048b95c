"""Autotuner for the blend kernels: tile shape x Gaussians staged per LDS batch.

For a pool and a set of views it builds one plan per candidate, times the
forward + backward of the whole view set (no parameter update, so every
candidate sees the same scene) with device-side synchronisation, and returns
the fastest (the default, first candidate unless another beats it by more
than 1%).  Results are cached in a JSON file keyed by the workload shape
(view resolutions, view count, live-slot count, SH degree).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import torch

from . import swgs

TIE_BAND = 0.01
CANDIDATES = [((16, 16), 256), ((16, 16), 128), ((8, 8), 64), ((8, 8), 128), ((32, 8), 256), ((32, 8), 128)]
CACHE = os.environ.get("SWGS_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "swgs_autotune.json"))


def workload_key(pool: "swgs.Pool", views) -> str:
    res = sorted((int(v.width), int(v.height)) for v in views)
    desc = dict(res=res, n_views=len(views), slots=int(pool.params.shape[1]), num_gs=int(pool.num_gs),
                sh=int(pool.sh_degree), frames=len(set(int(v.frame) for v in views)))
    return hashlib.sha1(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:16]


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def tune(ctx: "swgs.Context", pool: "swgs.Pool", views, reps: int = 3, use_cache: bool = True,
         candidates=CANDIDATES, log=None):
    """Returns (tile, lds_batch, table) with table = [(tile, lds, ms), ...]."""
    key = workload_key(pool, views)
    cache = _load() if use_cache else {}
    if key in cache:
        e = cache[key]
        return tuple(e["tile"]), int(e["lds_batch"]), e["table"]
    table = []
    for tile, lds in candidates:
        plan = swgs.Plan(ctx, pool, views, tile=tile, lds_batch=lds, headroom=1.2)
        dl = torch.randn(3 * plan.n_pixels, device=ctx.device) * 1e-6
        plan.forward()
        plan.backward(dl)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            plan.forward()
            plan.backward(dl)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t) / reps
        table.append((list(tile), lds, round(ms, 3)))
        if log:
            # one more pass with per-kernel events for the log
            plan.set_timing(swgs.SWGS_TIMING_EVENTS | swgs.SWGS_TIMING_COUNT)
            plan.forward()
            plan.backward(dl)
            tm, ev = plan.timing()
            plan.set_timing(0)
            per = " ".join(f"{k}={v[0]:.2f}" for k, v in tm.items() if v[1])
            log(f"autotune {tile[0]}x{tile[1]} lds {lds}: {ms:.2f} ms fwd+bwd [{per}] evals {ev[0]:.3g}/{ev[1]:.3g} "
                f"blended {ev[2]:.3g}")
        plan.close()
        del dl
    # the first candidate (the default shape) is kept unless another is
    # faster by more than TIE_BAND: differences inside run-to-run noise do
    # not flip the choice
    best = min(table, key=lambda r: r[2])
    if best is not table[0] and best[2] > table[0][2] * (1.0 - TIE_BAND):
        best = table[0]
    if use_cache:
        cache = _load()
        cache[key] = dict(tile=best[0], lds_batch=best[1], table=table)
        _store(cache)
    return tuple(best[0]), int(best[1]), table
