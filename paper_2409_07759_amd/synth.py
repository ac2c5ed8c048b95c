"""Seeded synthetic inputs shared by the HIP path, the oracle and the benches.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic (no projection, blending, optimisation or relocation).
Everything is float32/int32 numpy on the host so either side can consume it.

Parameter layout ("planar rows", slot-major inside a row): a pool of S slots
is a float32 array of shape [F, S] with
    rows 0..2   mean (x, y, z)
    rows 3..5   log-scale per axis
    rows 6..9   rotation quaternion (w, x, y, z), not necessarily unit
    row  10     opacity logit
    rows 11..   SH coefficients, row 11 + 3*k + ch for basis k < (d+1)^2,
                colour channel ch in (r, g, b)
so F = 11 + 3*(d+1)^2 (14 at degree 0, 59 at degree 3).

Distributions follow the tiny-scene recipe of the paper-shaped workloads:
mean U[-1,1]^3, log-scale N(-3, 0.5) (shifted by -0.5*ln(N/2000) for pools
above 2000 so the on-screen footprint stays that of the 2000-Gaussian scene),
uniform random unit quaternion, opacity logit N(0,1), SH DC N(0, 0.5),
higher SH N(0, 0.05).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROW_MEAN = 0
ROW_SCALE = 3
ROW_QUAT = 6
ROW_LOGIT = 10
ROW_SH = 11


def n_rows(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def log_scale_shift(n: int) -> float:
    return -0.5 * math.log(n / 2000.0) if n > 2000 else 0.0


def make_gaussians(n: int, sh_degree: int, seed: int, shift: float | None = None) -> np.ndarray:
    """Planar [F, n] float32 parameters drawn from the recipe above."""
    rng = np.random.default_rng(seed)
    F = n_rows(sh_degree)
    p = np.zeros((F, n), dtype=np.float64)
    p[0:3] = rng.uniform(-1.0, 1.0, size=(3, n))
    s = log_scale_shift(n) if shift is None else shift
    p[3:6] = rng.normal(-3.0 + s, 0.5, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    p[6:10] = q
    p[10] = rng.normal(0.0, 1.0, size=n)
    p[11:14] = rng.normal(0.0, 0.5, size=(3, n))
    if sh_degree > 0:
        p[14:] = rng.normal(0.0, 0.05, size=(F - 14, n))
    return p.astype(np.float32)


@dataclass
class View:
    """One (frame, camera) view. R, t map world to camera (x right, y down,
    z forward); fx, fy, cx, cy are pinhole intrinsics in pixels."""
    frame: int
    width: int
    height: int
    R: np.ndarray  # (3,3) float64
    t: np.ndarray  # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    bg: tuple = (0.0, 0.0, 0.0)

    def cam16(self) -> np.ndarray:
        """R row-major (9), t (3), fx, fy, cx, cy as float64[16]."""
        return np.concatenate([self.R.reshape(-1), self.t,
                               [self.fx, self.fy, self.cx, self.cy]]).astype(np.float64)


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World->camera rotation and translation for a camera at `eye` looking at
    `target`, OpenCV axes: +z forward, +x right, +y down on screen."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, dtype=np.float64)
    right = np.cross(fwd, upv)
    if np.linalg.norm(right) < 1e-9:
        right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])  # rows: camera axes in world coords
    t = -R @ eye
    return R, t


def ring_views(frames, n_cams: int, width: int, height: int, radius: float = 4.0,
               hfov_deg: float = 60.0, phase_deg: float = 0.0, sizes=None):
    """Cameras on a horizontal ring (x-z plane, y=0) looking at the origin,
    camera k at angle 2*pi*k/C; f_y = f_x from the horizontal FoV.  `sizes`
    optionally gives (width, height) per camera (mixed resolutions)."""
    views = []
    for f in frames:
        for k in range(n_cams):
            w, h = (sizes[k] if sizes is not None else (width, height))
            th = math.radians(phase_deg) + 2.0 * math.pi * k / n_cams
            eye = (radius * math.sin(th), 0.0, radius * math.cos(th))
            R, t = look_at(eye)
            fx = 0.5 * w / math.tan(math.radians(hfov_deg) / 2.0)
            views.append(View(int(f), int(w), int(h), R, t, fx, fx, 0.5 * w, 0.5 * h))
    return views


def random_pose_view(rng, frame: int, width: int, height: int, rmin=3.0, rmax=5.0,
                     hfov_deg: float = 60.0) -> View:
    """A camera at a uniform direction on a sphere of radius U[rmin, rmax],
    looking at the origin (serving requests)."""
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    r = rng.uniform(rmin, rmax)
    R, t = look_at(d * r)
    fx = 0.5 * width / math.tan(math.radians(hfov_deg) / 2.0)
    return View(int(frame), int(width), int(height), R, t, fx, fx, 0.5 * width, 0.5 * height)


# ---------------------------------------------------------------- lifespans

def lifespans_tiny(n: int, seed: int):
    """start = floor(U[0,3)), length uniform integer in {1,2,3}."""
    rng = np.random.default_rng(seed)
    start = np.floor(rng.uniform(0.0, 3.0, size=n)).astype(np.int32)
    length = rng.integers(1, 4, size=n).astype(np.int32)
    return start.copy(), start, (start + length).astype(np.int32)


@dataclass
class Pool:
    """A sliding pool: slots [0, num_gs) are the optimisable set, slots
    [num_gs, 2*num_gs) the frozen (matured) store.  All arrays are host numpy."""
    num_gs: int
    swin: int
    sh_degree: int
    params: np.ndarray          # [F, 2*num_gs] float32
    birth: np.ndarray           # [2*num_gs] int32
    start: np.ndarray
    expire: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def slots(self) -> int:
        return self.params.shape[1]


def steady_window_pool(num_gs: int, swin: int, sh_degree: int, st: int, seed: int) -> Pool:
    """A pool as it stands in steady state at window [st, st+swin): block k of
    the optimisable set (size num_gs/swin) has lifespan [b, b+swin) where b is
    the unique frame in [st, st+swin) with b = k (mod swin); its matured
    snapshot holds the previous lifespan [b-swin, b).  Every frame of the
    window therefore has exactly num_gs active slots, and about 1/swin of them
    retire and 1/swin are born per frame.  Requires st >= swin."""
    assert num_gs % swin == 0 and st >= swin
    S = num_gs // swin
    params = np.concatenate([make_gaussians(num_gs, sh_degree, seed),
                             make_gaussians(num_gs, sh_degree, seed + 1000,
                                            shift=log_scale_shift(num_gs))], axis=1)
    birth = np.zeros(2 * num_gs, np.int32)
    start = np.zeros(2 * num_gs, np.int32)
    expire = np.zeros(2 * num_gs, np.int32)
    for k in range(swin):
        b = st + ((k - st) % swin)
        sl = slice(k * S, (k + 1) * S)
        ms = slice(num_gs + k * S, num_gs + (k + 1) * S)
        birth[sl] = b
        start[sl] = b
        expire[sl] = b + swin
        birth[ms] = b - swin
        start[ms] = b - swin
        expire[ms] = b
    return Pool(num_gs, swin, sh_degree, params, birth, start, expire)


def add_faint_gaussians(pool: Pool, fraction: float, seed: int, lo: float = -7.0, hi: float = -3.5) -> int:
    """Give a seeded `fraction` of the optimisable slots [0, num_gs)
    near-transparent opacity logits, uniform in [lo, hi] (opacity 0.0009 ..
    0.029): the low-opacity tail that a trained model carries and that
    relocation works on.  With the default range about half of them start
    below opacity 0.005; the rest lie just above it.  Changes pool.params in
    place and returns the number of slots changed."""
    rng = np.random.default_rng(seed)
    k = int(round(fraction * pool.num_gs))
    idx = rng.choice(pool.num_gs, size=k, replace=False)
    pool.params[ROW_LOGIT, idx] = rng.uniform(lo, hi, size=k).astype(np.float32)
    return k


def uneven_window_pool(n_total: int, n_base: int, W: int, sh_degree: int, seed: int,
                       max_len: int = 27) -> Pool:
    """Pool for a W-frame window with uneven per-frame active sets: n_base
    Gaussians span all W frames; the rest have start ~ U{0..W-1} and length
    ~ U{1..max_len} (clipped to the window).  All slots are optimisable; the
    frozen half is empty (expire = start = -1, never active)."""
    rng = np.random.default_rng(seed + 7)
    params = make_gaussians(n_total, sh_degree, seed)
    start = np.zeros(n_total, np.int32)
    expire = np.full(n_total, W, np.int32)
    m = n_total - n_base
    s = rng.integers(0, W, size=m)
    ln = rng.integers(1, max_len + 1, size=m)
    start[n_base:] = s
    expire[n_base:] = np.minimum(s + ln, W)
    params = np.concatenate([params, np.zeros_like(params)], axis=1)
    birth = np.concatenate([start, np.full(n_total, -1, np.int32)])
    start2 = np.concatenate([start, np.full(n_total, -1, np.int32)])
    expire2 = np.concatenate([expire, np.full(n_total, -1, np.int32)])
    return Pool(n_total, W, sh_degree, params, birth, start2, expire2)


def serving_pool(n_active: int, n_frames: int, sh_degree: int, seed: int,
                 lo: float = 0.01, hi: float = 0.02) -> Pool:
    """Resident pool for serving a clip: n_active Gaussians are live at every
    frame; at each frame f >= 1 a fraction u ~ U[lo, hi] of the live ones
    expire and as many new ones are born with lifespan [f, n_frames).  All
    slots are resident; num_gs = total slots, no frozen half."""
    rng = np.random.default_rng(seed + 11)
    counts = [0] + [int(round(rng.uniform(lo, hi) * n_active)) for _ in range(1, n_frames)]
    total = n_active + sum(counts)
    start = np.zeros(total, np.int32)
    expire = np.full(total, n_frames, np.int32)
    live = np.arange(n_active)
    nxt = n_active
    for f in range(1, n_frames):
        c = counts[f]
        pick = rng.choice(live.shape[0], size=c, replace=False)
        expire[live[pick]] = f
        new = np.arange(nxt, nxt + c)
        start[new] = f
        live = np.concatenate([np.delete(live, pick), new])
        nxt += c
    params = make_gaussians(total, sh_degree, seed, shift=log_scale_shift(n_active))
    return Pool(total, n_frames, sh_degree, params, start.copy(), start, expire)


def random_images(views, seed: int) -> np.ndarray:
    """Uniform [0,1) float32 images concatenated view after view, each planar
    [3, H, W] (used as targets or upstream gradients in parity tests)."""
    rng = np.random.default_rng(seed)
    n = sum(3 * v.width * v.height for v in views)
    return rng.uniform(0.0, 1.0, size=n).astype(np.float32)
