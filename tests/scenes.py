"""Scene builders and comparison helpers shared by the GPU parity tests.
Only seeded inputs (paper_2409_07759_amd.synth) and the oracle are used."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2409_07759_amd import synth as S

MARGIN_INT = 1e-12      # integer decisions closer than this (relative) are reported, not asserted
MARGIN_PIX = 1e-4       # pixel skip/stop decisions closer than this are excluded from image parity
IMG_TOL = 1e-5          # spec image tolerance (absolute)
GRAD_RTOL = 1e-3        # spec gradient tolerance (relative)


def tiny(seed=0, n=2000, width=128, height=96, deg=0, frames=(0, 1, 2), cams=3):
    """The 2000-Gaussian, 3-frame x 3-camera window at 128x96."""
    params = S.make_gaussians(n, deg, seed)
    birth, start, expire = S.lifespans_tiny(n, seed)
    views = S.ring_views(list(frames), cams, width, height)
    return S.Pool(n, 3, deg, params, birth, start, expire), views


def steady(num_gs=600, swin=5, st=7, deg=1, seed=3, width=96, height=72, cams=2):
    pool = S.steady_window_pool(num_gs, swin, deg, st, seed)
    views = S.ring_views(list(range(st, st + swin)), cams, width, height, phase_deg=20.0)
    return pool, views


def oracle_records(pool, view, tw, th):
    vis, rec, rect = O.preprocess(pool.params, pool.sh_degree, pool.start, pool.expire, view, tw, th)
    return vis, rec, rect


def grad_close(g, ref, rtol=GRAD_RTOL, floor=1e-2):
    """|g - ref| <= rtol * max(|ref|, floor * ||ref||_inf), per tensor."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), floor * (np.abs(ref).max() if ref.size else 0.0))
    bad = np.abs(g - ref) > rtol * scale + 1e-30
    return ~bad


def split_views(flat, views):
    return O.split_images(flat, views)
